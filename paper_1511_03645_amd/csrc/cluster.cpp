// Berger-Rigoutsos clustering of flagged cells into rectangular patches
// (Davis & LeVeque Sec. 3, citing Berger & Rigoutsos 1991), proper-nesting
// regions and flag buffering, on the host.
//
// The clustering is deterministic: a box is shrunk to the bounding box of its
// flags; accepted when its efficiency (flagged fraction) reaches the cutoff,
// both sides are within the maximum and every cell is allowed; otherwise cut
// at the interior hole of the row/column signatures nearest the centre, else
// at the strongest sign change of the signatures' second difference, else in
// halves along the longer side; parts keep at least `minside` cells (1 when
// the box holds disallowed cells); lower/left part first.
#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <vector>

#include "abi_guard.h"
#include "wp.h"

namespace {

// Summed-area tables of the flag image and of its disallowed cells over a
// window (i0, j0, nx, ny) of an image of row pitch `pitch`, so that the flag
// count of any box, and so a box's row and column signatures, cost O(1) per
// entry instead of a scan of the box.  Coordinates are window-relative.
struct Sat {
    int nx, ny;
    const int *F, *B;   // (nx + 1) x (ny + 1), entry (i, j) sums cells [0, i) x [0, j)
    Sat(const uint8_t *f, const uint8_t *ok, size_t pitch, int i0, int j0, int nx_, int ny_) : nx(nx_), ny(ny_)
    {
        // the tables live on between calls (no page faults, no clearing: the
        // zero row and column are set, every other entry is written); each
        // row's running sums first, then added to the row above
        static thread_local std::vector<int> tf, tb, rf, rb;
        const size_t W = (size_t)nx + 1;
        // the second of each pair is tested: a failed allocation of it leaves
        // the first grown and the test still true on the next call
        if (tb.size() < W * (ny + 1)) {
            tf.resize(W * (ny + 1));
            tb.resize(W * (ny + 1));
        }
        if (rb.size() < (size_t)nx) {
            rf.resize(nx);
            rb.resize(nx);
        }
        int *Fw = tf.data(), *Bw = tb.data();
        std::fill_n(Fw, W, 0);
        std::fill_n(Bw, W, 0);
        for (int j = 0; j < ny; ++j) {
            const uint8_t *fr = f + (size_t)(j0 + j) * pitch + i0;
            const uint8_t *okr = ok ? ok + (size_t)(j0 + j) * pitch + i0 : nullptr;
            int sf = 0, sb = 0;
            for (int i = 0; i < nx; ++i) {
                const bool a = !okr || okr[i];
                sf += a && fr[i];
                sb += !a;
                rf[i] = sf;
                rb[i] = sb;
            }
            const int *fa = Fw + j * W + 1, *ba = Bw + j * W + 1;
            int *fo = Fw + (j + 1) * W, *bo = Bw + (j + 1) * W;
            fo[0] = bo[0] = 0;
            for (int i = 0; i < nx; ++i) fo[i + 1] = fa[i] + rf[i];
            for (int i = 0; i < nx; ++i) bo[i + 1] = ba[i] + rb[i];
        }
        F = Fw;
        B = Bw;
    }
    static int box(const int *S, size_t W, int i0, int j0, int i1, int j1)
    {
        return S[j1 * W + i1] - S[j0 * W + i1] - S[j1 * W + i0] + S[j0 * W + i0];
    }
    int flags(int i0, int j0, int i1, int j1) const { return box(F, (size_t)nx + 1, i0, j0, i1, j1); }
    int bad(int i0, int j0, int i1, int j1) const { return box(B, (size_t)nx + 1, i0, j0, i1, j1); }
};

struct Key {
    long long a, b, c, d;
    bool operator<(const Key &o) const
    {
        if (a != o.a) return a < o.a;
        if (b != o.b) return b < o.b;
        if (c != o.c) return c < o.c;
        return d < o.d;
    }
};

void cluster_box(const Sat &im, int i0, int j0, int w, int h, double eff_min, int maxside, int minside,
                 std::vector<wp_patch> &out)
{
    // shrink to the bounding box of the flags
    const long long nflag = im.flags(i0, j0, i0 + w, j0 + h);
    if (nflag == 0) return;
    {
        int a = 0, b = w - 1, c = 0, d = h - 1;
        while (im.flags(i0 + a, j0, i0 + a + 1, j0 + h) == 0) ++a;
        while (im.flags(i0 + b, j0, i0 + b + 1, j0 + h) == 0) --b;
        while (im.flags(i0, j0 + c, i0 + w, j0 + c + 1) == 0) ++c;
        while (im.flags(i0, j0 + d, i0 + w, j0 + d + 1) == 0) --d;
        i0 += a;
        j0 += c;
        w = b - a + 1;
        h = d - c + 1;
    }
    const bool all_ok = im.bad(i0, j0, i0 + w, j0 + h) == 0;
    const double eff = (double)nflag / ((double)w * h);
    if (eff >= eff_min && w <= maxside && h <= maxside && all_ok) {
        out.push_back(wp_patch{i0, j0, w, h});
        return;
    }
    const int ms = all_ok ? minside : 1;
    std::vector<long long> sig[2];
    sig[0].resize(w);
    sig[1].resize(h);
    for (int i = 0; i < w; ++i) sig[0][i] = im.flags(i0 + i, j0, i0 + i + 1, j0 + h);
    for (int j = 0; j < h; ++j) sig[1][j] = im.flags(i0, j0 + j, i0 + w, j0 + j + 1);
    const int len[2] = {w, h};
    bool found = false;
    int cut_ax = 0, cut_at = 0;
    // 1. holes (interior zero signatures), nearest the centre
    Key best{0, 0, 0, 0};
    for (int ax = 0; ax < 2; ++ax) {
        const int n = len[ax];
        for (int k = 1; k < n - 1; ++k) {
            if (sig[ax][k] != 0 || k < ms || n - k < ms) continue;
            Key key{std::llabs(2LL * k + 1 - n), ax, k, 0};
            if (!found || key < best) {
                best = key;
                found = true;
                cut_ax = ax;
                cut_at = k;
            }
        }
    }
    // 2. strongest inflection of the signature (sign change of the second
    //    difference), cut between k and k+1
    if (!found) {
        for (int ax = 0; ax < 2; ++ax) {
            const int n = len[ax];
            const std::vector<long long> &s = sig[ax];
            for (int k = 1; k < n - 2; ++k) {
                const long long a = s[k - 1] - 2 * s[k] + s[k + 1];
                const long long b = s[k] - 2 * s[k + 1] + s[k + 2];
                const int c = k + 1;
                if (!((a < 0 && b > 0) || (a > 0 && b < 0)) || c < ms || n - c < ms) continue;
                Key key{-std::llabs(b - a), std::llabs(2LL * c - n), ax, c};
                if (!found || key < best) {
                    best = key;
                    found = true;
                    cut_ax = ax;
                    cut_at = c;
                }
            }
        }
    }
    // 3. halves of the longer side
    if (!found) {
        const int ax = w >= h ? 0 : 1;
        const int n = len[ax], c = n / 2;
        if (c >= ms && n - c >= ms) {
            found = true;
            cut_ax = ax;
            cut_at = c;
        }
    }
    if (!found) {
        out.push_back(wp_patch{i0, j0, w, h});
        return;
    }
    if (cut_ax == 0) {
        cluster_box(im, i0, j0, cut_at, h, eff_min, maxside, minside, out);
        cluster_box(im, i0 + cut_at, j0, w - cut_at, h, eff_min, maxside, minside, out);
    } else {
        cluster_box(im, i0, j0, w, cut_at, eff_min, maxside, minside, out);
        cluster_box(im, i0, j0 + cut_at, w, h - cut_at, eff_min, maxside, minside, out);
    }
}

}  // namespace

// Proper-nesting region of a level within the window [wi0, wi0 + ww) x
// [wj0, wj0 + wh), which must hold all of its patches: cells of the patches
// that have no neighbour (8-neighbourhood, inside the domain nx x ny)
// outside every patch.  mask is ww x wh.
void wp_nesting_mask(const std::vector<wp_patch> &patches, int nx, int ny, int wi0, int wj0, int ww, int wh,
                     std::vector<uint8_t> &mask)
{
    // "inside" on the window grown by one cell: outside the domain counts as
    // inside (no neighbour there), domain cells outside the window are in no
    // patch; then a 3 x 3 erosion, along rows and then along columns
    const int pw = ww + 2, ph = wh + 2;
    static thread_local std::vector<uint8_t> in, row;
    in.assign((size_t)pw * ph, 0);
    row.resize((size_t)pw * ph);
    // only the frame around the window can lie outside the domain
    for (int b = 0; b < ph; ++b)
        for (int a = 0; a < pw; a += (b == 0 || b == ph - 1) ? 1 : pw - 1) {
            const int i = wi0 - 1 + a, j = wj0 - 1 + b;
            if (i < 0 || i >= nx || j < 0 || j >= ny) in[(size_t)b * pw + a] = 1;
        }
    for (const auto &p : patches)
        for (int j = p.jlo; j < p.jlo + p.ny; ++j)
            std::fill_n(&in[(size_t)(j - wj0 + 1) * pw + (p.ilo - wi0 + 1)], p.nx, (uint8_t)1);
    for (int b = 0; b < ph; ++b) {
        const uint8_t *x = &in[(size_t)b * pw];
        uint8_t *y = &row[(size_t)b * pw];
        for (int a = 1; a < pw - 1; ++a) y[a] = x[a - 1] & x[a] & x[a + 1];
    }
    mask.assign((size_t)ww * wh, 0);
    for (int b = 1; b < ph - 1; ++b) {
        const uint8_t *x = &in[(size_t)b * pw + 1], *up = &row[(size_t)(b - 1) * pw + 1];
        const uint8_t *mid = &row[(size_t)b * pw + 1], *dn = &row[(size_t)(b + 1) * pw + 1];
        uint8_t *m = &mask[(size_t)(b - 1) * ww];
        for (int a = 0; a < ww; ++a) m[a] = x[a] & up[a] & mid[a] & dn[a];
    }
}

// Box dilation by k cells (flag buffering around flagged cells) of an
// nx x ny image: a running count along each row, then along each column.
void wp_dilate(const std::vector<uint8_t> &f, int nx, int ny, int k, std::vector<uint8_t> &out)
{
    if (k <= 0) {
        out = f;
        return;
    }
    out.resize((size_t)nx * ny);
    static thread_local std::vector<uint8_t> rows;
    rows.resize((size_t)nx * ny);
    std::vector<int> pre(nx + 1);
    for (int j = 0; j < ny; ++j) {
        const uint8_t *r = &f[(size_t)j * nx];
        uint8_t *o = &rows[(size_t)j * nx];
        pre[0] = 0;
        for (int i = 0; i < nx; ++i) pre[i + 1] = pre[i] + (r[i] != 0);
        for (int i = 0; i < nx; ++i) o[i] = pre[std::min(i + k + 1, nx)] - pre[std::max(i - k, 0)] > 0;
    }
    // along columns: per column the count of row-dilated cells in rows
    // j - k .. j + k, slid down one row at a time
    std::vector<int> cnt(nx, 0);
    for (int j = 0; j < std::min(k, ny); ++j)
        for (int i = 0; i < nx; ++i) cnt[i] += rows[(size_t)j * nx + i];
    for (int j = 0; j < ny; ++j) {
        if (j + k < ny) {
            const uint8_t *a = &rows[(size_t)(j + k) * nx];
            for (int i = 0; i < nx; ++i) cnt[i] += a[i];
        }
        if (j - k - 1 >= 0) {
            const uint8_t *d = &rows[(size_t)(j - k - 1) * nx];
            for (int i = 0; i < nx; ++i) cnt[i] -= d[i];
        }
        uint8_t *o = &out[(size_t)j * nx];
        for (int i = 0; i < nx; ++i) o[i] = cnt[i] > 0;
    }
}

// The boxes of an nx x ny flag image restricted to `allowed` (see wp_cluster).
// Clustering starts by shrinking the whole image to the bounding box of its
// (allowed) flags, so the tables cover that box only.
void wp_cluster_boxes(const uint8_t *flags, const uint8_t *allowed, int nx, int ny, double efficiency, int maxside,
                      int minside, std::vector<wp_patch> &out)
{
    out.clear();
    int a = nx, b = ny, c = -1, d = -1;
    for (int j = 0; j < ny; ++j) {
        const uint8_t *fr = flags + (size_t)j * nx;
        const uint8_t *okr = allowed ? allowed + (size_t)j * nx : nullptr;
        int lo = -1, hi = -1;
        for (int i = 0; i < nx; ++i)
            if (fr[i] && (!okr || okr[i])) {
                if (lo < 0) lo = i;
                hi = i;
            }
        if (lo < 0) continue;
        a = std::min(a, lo);
        c = std::max(c, hi);
        b = std::min(b, j);
        d = j;
    }
    if (c < 0) return;
    const Sat im(flags, allowed, (size_t)nx, a, b, c - a + 1, d - b + 1);
    cluster_box(im, 0, 0, c - a + 1, d - b + 1, efficiency, maxside, minside, out);
    for (wp_patch &p : out) {
        p.ilo += a;
        p.jlo += b;
    }
}

extern "C" int wp_cluster(const uint8_t *flags, const uint8_t *allowed, int nx, int ny, double efficiency,
                          int maxside, int minside, wp_patch *out, int cap, int *npatches)
{
    WP_ABI_TRY
    if (!flags || nx < 1 || ny < 1 || maxside < 1 || minside < 1 || !npatches || (cap > 0 && !out))
        return WP_EINVAL;
    std::vector<wp_patch> boxes;
    wp_cluster_boxes(flags, allowed, nx, ny, efficiency, maxside, minside, boxes);
    *npatches = (int)boxes.size();
    for (int k = 0; k < (int)boxes.size() && k < cap; ++k) out[k] = boxes[k];
    return WP_OK;
    WP_ABI_CATCH(nullptr)
}
