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

#include "wp.h"

namespace {

struct Img {
    int nx, ny;
    const uint8_t *f;    // flagged (already restricted to allowed)
    const uint8_t *ok;   // allowed
    bool flag(int i, int j) const { return f[(size_t)j * nx + i] != 0; }
    bool allowed(int i, int j) const { return ok[(size_t)j * nx + i] != 0; }
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

void cluster_box(const Img &im, int i0, int j0, int w, int h, double eff_min, int maxside, int minside,
                 std::vector<wp_patch> &out)
{
    // shrink to the bounding box of the flags
    int imin = i0 + w, imax = i0 - 1, jmin = j0 + h, jmax = j0 - 1;
    long long nflag = 0;
    for (int j = j0; j < j0 + h; ++j)
        for (int i = i0; i < i0 + w; ++i)
            if (im.flag(i, j)) {
                imin = std::min(imin, i);
                imax = std::max(imax, i);
                jmin = std::min(jmin, j);
                jmax = std::max(jmax, j);
                ++nflag;
            }
    if (nflag == 0) return;
    i0 = imin;
    j0 = jmin;
    w = imax - imin + 1;
    h = jmax - jmin + 1;
    bool all_ok = true;
    for (int j = j0; j < j0 + h && all_ok; ++j)
        for (int i = i0; i < i0 + w; ++i)
            if (!im.allowed(i, j)) {
                all_ok = false;
                break;
            }
    const double eff = (double)nflag / ((double)w * h);
    if (eff >= eff_min && w <= maxside && h <= maxside && all_ok) {
        out.push_back(wp_patch{i0, j0, w, h});
        return;
    }
    const int ms = all_ok ? minside : 1;
    std::vector<long long> sig[2];
    sig[0].assign(w, 0);
    sig[1].assign(h, 0);
    for (int j = 0; j < h; ++j)
        for (int i = 0; i < w; ++i)
            if (im.flag(i0 + i, j0 + j)) {
                sig[0][i]++;
                sig[1][j]++;
            }
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

// Proper-nesting region of a level: cells of its patches that have no
// neighbour (8-neighbourhood, inside the domain) outside every patch.
void wp_nesting_mask(const std::vector<wp_patch> &patches, int nx, int ny, std::vector<uint8_t> &mask)
{
    std::vector<uint8_t> inside((size_t)nx * ny, 0);
    for (const auto &p : patches)
        for (int j = p.jlo; j < p.jlo + p.ny; ++j)
            for (int i = p.ilo; i < p.ilo + p.nx; ++i) inside[(size_t)j * nx + i] = 1;
    mask.assign((size_t)nx * ny, 0);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (!inside[(size_t)j * nx + i]) continue;
            bool ok = true;
            for (int dj = -1; dj <= 1 && ok; ++dj)
                for (int di = -1; di <= 1; ++di) {
                    const int a = i + di, b = j + dj;
                    if (a >= 0 && a < nx && b >= 0 && b < ny && !inside[(size_t)b * nx + a]) {
                        ok = false;
                        break;
                    }
                }
            mask[(size_t)j * nx + i] = ok;
        }
}

// Box dilation by k cells (flag buffering around flagged cells).
void wp_dilate(const std::vector<uint8_t> &f, int nx, int ny, int k, std::vector<uint8_t> &out)
{
    out = f;
    if (k <= 0) return;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (!f[(size_t)j * nx + i]) continue;
            for (int b = std::max(j - k, 0); b <= std::min(j + k, ny - 1); ++b)
                for (int a = std::max(i - k, 0); a <= std::min(i + k, nx - 1); ++a) out[(size_t)b * nx + a] = 1;
        }
}

extern "C" int wp_cluster(const uint8_t *flags, const uint8_t *allowed, int nx, int ny, double efficiency,
                          int maxside, int minside, wp_patch *out, int cap, int *npatches)
{
    if (!flags || nx < 1 || ny < 1 || maxside < 1 || minside < 1 || !npatches || (cap > 0 && !out))
        return WP_EINVAL;
    std::vector<uint8_t> ok(allowed ? allowed : flags, (allowed ? allowed : flags) + (size_t)nx * ny);
    if (!allowed) std::fill(ok.begin(), ok.end(), 1);
    std::vector<uint8_t> f((size_t)nx * ny);
    for (size_t k = 0; k < f.size(); ++k) f[k] = (flags[k] && ok[k]) ? 1 : 0;
    Img im{nx, ny, f.data(), ok.data()};
    std::vector<wp_patch> boxes;
    cluster_box(im, 0, 0, nx, ny, efficiency, maxside, minside, boxes);
    *npatches = (int)boxes.size();
    for (int k = 0; k < (int)boxes.size() && k < cap; ++k) out[k] = boxes[k];
    return WP_OK;
}
