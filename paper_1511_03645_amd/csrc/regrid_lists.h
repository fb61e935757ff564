// Cell and face lists of a regrid (Davis & LeVeque Sec. 3: the ghost ring of
// a fine level, the cells a new patch takes from the level below, the coarse
// cells under a level's patches, the coarse-fine faces of refluxing), built
// from per-row column intervals of the patches rather than from masks of the
// level: the work grows with the patches' rows and perimeters, not with the
// level's area.  The lists are written into the caller's vectors and the
// temporaries are kept per thread, so a caller that keeps its vectors
// between regrids allocates nothing once they have grown.  Host code only
// (no HIP), so it also builds with a plain C++ compiler.
#pragma once

#include <algorithm>
#include <array>
#include <climits>
#include <cstdint>
#include <utility>
#include <vector>

#include "wp.h"

namespace wp {

// [i0, i1) x [j0, j1)
struct Rect {
    int i0, j0, i1, j1;
};

// A union of rectangles as merged [a, b) column intervals per row, for the
// rows j0 .. j0 + nrows - 1 (row j's intervals are iv[off[j - j0]] ..
// iv[off[j - j0 + 1] - 1], in increasing a, disjoint and not touching).
struct Spans {
    int j0 = 0, nrows = 0;
    std::vector<int> off{0};
    std::vector<std::pair<int, int>> iv;

    const std::pair<int, int> *row_begin(int j) const
    {
        return (j < j0 || j >= j0 + nrows) ? nullptr : iv.data() + off[j - j0];
    }
    const std::pair<int, int> *row_end(int j) const
    {
        return (j < j0 || j >= j0 + nrows) ? nullptr : iv.data() + off[j - j0 + 1];
    }
    bool contains(int i, int j) const
    {
        const std::pair<int, int> *a = row_begin(j), *b = row_end(j);
        if (a == b) return false;
        // the last interval starting at or before i
        const std::pair<int, int> *k =
            std::upper_bound(a, b, i, [](int v, const std::pair<int, int> &x) { return v < x.first; });
        return k != a && i < (k - 1)->second;
    }
};

// The union of R into s (its blocks reused); rectangles with no cells are
// skipped.
inline void make_spans(const std::vector<Rect> &R, Spans &s)
{
    s.j0 = 0;
    s.nrows = 0;
    s.off.assign(1, 0);
    s.iv.clear();
    int lo = INT_MAX, hi = INT_MIN;
    for (const Rect &r : R)
        if (r.i0 < r.i1 && r.j0 < r.j1) {
            lo = std::min(lo, r.j0);
            hi = std::max(hi, r.j1);
        }
    if (lo >= hi) return;
    s.j0 = lo;
    s.nrows = hi - lo;
    // bucket the rectangles' row intervals by row (counting sort, stable),
    // the rectangles taken in increasing i0 so that every row's intervals
    // arrive sorted, then merge each row's
    static thread_local std::vector<int> start, pos, ord;
    static thread_local std::vector<std::pair<int, int>> raw;
    ord.clear();
    for (int k = 0; k < (int)R.size(); ++k)
        if (R[k].i0 < R[k].i1 && R[k].j0 < R[k].j1) ord.push_back(k);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return R[a].i0 != R[b].i0 ? R[a].i0 < R[b].i0 : a < b; });
    start.assign((size_t)s.nrows + 1, 0);
    for (int k : ord)
        for (int j = R[k].j0; j < R[k].j1; ++j) ++start[j - lo + 1];
    for (int k = 0; k < s.nrows; ++k) start[k + 1] += start[k];
    raw.resize((size_t)start[s.nrows]);
    pos.assign(start.begin(), start.end() - 1);
    for (int k : ord)
        for (int j = R[k].j0; j < R[k].j1; ++j) raw[pos[j - lo]++] = {R[k].i0, R[k].i1};
    s.off.assign((size_t)s.nrows + 1, 0);
    for (int k = 0; k < s.nrows; ++k) {
        auto a = raw.begin() + start[k], b = raw.begin() + start[k + 1];
        for (auto it = a; it != b; ++it) {
            if ((int)s.iv.size() > s.off[k] && it->first <= s.iv.back().second)
                s.iv.back().second = std::max(s.iv.back().second, it->second);
            else
                s.iv.push_back(*it);
        }
        s.off[k + 1] = (int)s.iv.size();
    }
}

// Call emit(a, b) for each maximal run [a, b) of row j that lies in A and
// not in B, in increasing a.
template <class F> void row_difference(const Spans &A, const Spans &B, int j, F &&emit)
{
    const std::pair<int, int> *a = A.row_begin(j), *ae = A.row_end(j);
    const std::pair<int, int> *b = B.row_begin(j), *be = B.row_end(j);
    for (; a != ae; ++a) {
        int x = a->first;
        while (b != be && b->second <= x) ++b;
        for (const std::pair<int, int> *c = b; x < a->second; ++c) {
            if (c == be || c->first >= a->second) {
                emit(x, a->second);
                break;
            }
            if (c->first > x) emit(x, c->first);
            x = std::max(x, c->second);
        }
    }
}

// The patches grown by `grow` cells and clipped to nx x ny.
inline void patch_rects(const std::vector<wp_patch> &P, int grow, int nx, int ny, std::vector<Rect> &R)
{
    R.clear();
    for (const wp_patch &p : P)
        R.push_back(Rect{std::max(p.ilo - grow, 0), std::max(p.jlo - grow, 0), std::min(p.ilo + p.nx + grow, nx),
                         std::min(p.jlo + p.ny + grow, ny)});
}

// Union of the patches grown by `grow`, clipped, into s.
inline void patch_spans(const std::vector<wp_patch> &P, int grow, int nx, int ny, Spans &s)
{
    static thread_local std::vector<Rect> R;
    patch_rects(P, grow, nx, ny, R);
    make_spans(R, s);
}

// The ghost ring of a level's patches: cells inside the level's nx x ny
// domain, within two cells (either direction, corners included) of a patch
// and inside none, as runs (j, a, b) of cells [a, b) of row j, in increasing
// j * nx + a.
inline void ring_runs(const std::vector<wp_patch> &P, int nx, int ny, std::vector<std::array<int, 3>> &out)
{
    static thread_local Spans halo, in;
    patch_spans(P, 2, nx, ny, halo);
    patch_spans(P, 0, nx, ny, in);
    out.clear();
    for (int j = halo.j0; j < halo.j0 + halo.nrows; ++j)
        row_difference(halo, in, j, [&](int a, int b) { out.push_back({j, a, b}); });
}
// The cells of runs (j, a, b) as linear indices j * nx + i, in run order.
inline void run_cells(const std::vector<std::array<int, 3>> &runs, int nx, std::vector<int> &out)
{
    size_t n = 0;
    for (const auto &u : runs) n += (size_t)(u[2] - u[1]);
    out.resize(n);
    size_t k = 0;
    for (const auto &u : runs)
        for (int i = u[1]; i < u[2]; ++i) out[k++] = u[0] * nx + i;
}

// The ring grouped by the cell of the level below (ratio r, NX wide) that
// contains its cells: for each such cell in increasing linear index, (its
// index, the low and high 32 bits of the mask of its fine cells in the ring,
// bit (i % r) + r (j % r)).  Needs r <= 8.
inline void ring_block_list(const std::vector<std::array<int, 3>> &runs, int r, int NX, std::vector<int> &out)
{
    out.clear();
    static thread_local std::vector<unsigned long long> acc;
    static thread_local std::vector<int> touched;
    acc.assign((size_t)NX, 0);
    // indices are non-negative: a power-of-two ratio divides by a shift
    const bool pow2 = (r & (r - 1)) == 0;
    int lr = 0;
    while ((1 << lr) < r) ++lr;
    auto div = [&](int x) { return pow2 ? x >> lr : x / r; };
    for (size_t k = 0; k < runs.size();) {
        // the runs of the r fine rows of one coarse row are contiguous; the
        // coarse cells they touch are collected and sorted, so that a row
        // with runs far apart costs its runs, not the width between them
        const int J = div(runs[k][0]);
        touched.clear();
        for (; k < runs.size() && div(runs[k][0]) == J; ++k) {
            const int j = runs[k][0], a = runs[k][1], b = runs[k][2];
            const int shift = r * (j - J * r);
            for (int I = div(a); I <= div(b - 1); ++I) {
                const int x0 = std::max(a, I * r) - I * r, x1 = std::min(b, I * r + r) - I * r;
                if (!acc[I]) touched.push_back(I);
                acc[I] |= (((1ULL << (x1 - x0)) - 1) << x0) << shift;
            }
        }
        std::sort(touched.begin(), touched.end());
        for (int I : touched) {
            out.push_back(J * NX + I);
            out.push_back((int)(unsigned)(acc[I] & 0xffffffffULL));
            out.push_back((int)(unsigned)(acc[I] >> 32));
            acc[I] = 0;
        }
    }
}

// Coarse cells (linear indices on a canvas NX wide, increasing) covered by
// ratio-aligned, non-overlapping fine patches.
inline void cover_cells(const std::vector<wp_patch> &P, int r, int NX, std::vector<int> &out)
{
    static thread_local std::vector<Rect> R;
    static thread_local Spans s;
    static thread_local std::vector<std::array<int, 3>> runs;
    R.clear();
    for (const wp_patch &p : P) R.push_back(Rect{p.ilo / r, p.jlo / r, (p.ilo + p.nx) / r, (p.jlo + p.ny) / r});
    make_spans(R, s);
    runs.clear();
    for (int j = s.j0; j < s.j0 + s.nrows; ++j)
        for (const std::pair<int, int> *a = s.row_begin(j); a != s.row_end(j); ++a) runs.push_back({j, a->first, a->second});
    run_cells(runs, NX, out);
}

// Cells of the new patches `boxes` outside every old patch (linear indices
// on a level nx wide, increasing).
inline void fresh_cells(const std::vector<wp_patch> &boxes, const std::vector<wp_patch> &old, int nx, int ny,
                        std::vector<int> &out)
{
    static thread_local Spans nw, od;
    static thread_local std::vector<std::array<int, 3>> runs;
    patch_spans(boxes, 0, nx, ny, nw);
    patch_spans(old, 0, nx, ny, od);
    runs.clear();
    for (int j = nw.j0; j < nw.j0 + nw.nrows; ++j)
        row_difference(nw, od, j, [&](int a, int b) { runs.push_back({j, a, b}); });
    run_cells(runs, nx, out);
}

// The coarse-fine faces of refluxing between ratio-r patches P and the cells
// of the level below (NX x NY) that none of them covers.  Each face is
// (coarse cell J * NX + I, axis | 2 if the coarse cell lies before the patch
// (west or south), fine i, fine j of the patch's first edge cell).  They are
// generated patch by patch (for each coarse row of a patch its west then
// east face, then for each coarse column its south then north face) and
// ordered by coarse cell, keeping the generation order among the faces of
// one cell; `groups` gets (first face, count) per coarse cell.
inline void reflux_faces(const std::vector<wp_patch> &P, int r, int NX, int NY, std::vector<int> &flat,
                         std::vector<int> &groups)
{
    flat.clear();
    groups.clear();
    if (P.empty()) return;
    // the covered coarse cells as a mask of the patches' bounding window
    int wi0 = INT_MAX, wj0 = INT_MAX, wi1 = INT_MIN, wj1 = INT_MIN;
    for (const wp_patch &p : P) {
        wi0 = std::min(wi0, p.ilo / r);
        wj0 = std::min(wj0, p.jlo / r);
        wi1 = std::max(wi1, (p.ilo + p.nx) / r);
        wj1 = std::max(wj1, (p.jlo + p.ny) / r);
    }
    const int ww = wi1 - wi0;
    static thread_local std::vector<uint8_t> cov;
    cov.assign((size_t)ww * (wj1 - wj0), 0);
    for (const wp_patch &p : P)
        for (int J = p.jlo / r; J < (p.jlo + p.ny) / r; ++J)
            std::fill_n(&cov[(size_t)(J - wj0) * ww + (p.ilo / r - wi0)], p.nx / r, (uint8_t)1);
    auto covered = [&](int I, int J) {
        return I >= wi0 && I < wi1 && J >= wj0 && J < wj1 && cov[(size_t)(J - wj0) * ww + (I - wi0)];
    };
    static thread_local std::vector<std::array<int, 4>> faces, sorted;
    static thread_local std::vector<unsigned long long> key;
    static thread_local std::vector<int> start, pos;
    faces.clear();
    auto add = [&](int I, int J, int axis, bool before, int fi, int fj) {
        if (I < 0 || J < 0 || I >= NX || J >= NY || covered(I, J)) return;
        faces.push_back({J * NX + I, axis | (before ? 2 : 0), fi, fj});
    };
    for (const wp_patch &p : P) {
        const int I0 = p.ilo / r, J0 = p.jlo / r, W = p.nx / r, H = p.ny / r;
        for (int J = J0; J < J0 + H; ++J) {
            add(I0 - 1, J, 0, true, p.ilo, J * r);
            add(I0 + W, J, 0, false, p.ilo + p.nx - 1, J * r);
        }
        for (int I = I0; I < I0 + W; ++I) {
            add(I, J0 - 1, 1, true, I * r, p.jlo);
            add(I, J0 + H, 1, false, I * r, p.jlo + p.ny - 1);
        }
    }
    if (faces.empty()) return;
    // stable order by cell: a counting sort by coarse row, then each row by
    // (column, generation index)
    int jlo = INT_MAX, jhi = INT_MIN;
    for (const auto &f : faces) {
        jlo = std::min(jlo, f[0] / NX);
        jhi = std::max(jhi, f[0] / NX);
    }
    start.assign((size_t)(jhi - jlo) + 2, 0);
    for (const auto &f : faces) ++start[f[0] / NX - jlo + 1];
    for (size_t k = 1; k < start.size(); ++k) start[k] += start[k - 1];
    key.resize(faces.size());
    pos.assign(start.begin(), start.end() - 1);
    for (size_t k = 0; k < faces.size(); ++k)
        key[pos[faces[k][0] / NX - jlo]++] = ((unsigned long long)(faces[k][0] % NX) << 32) | k;
    for (size_t k = 0; k + 1 < start.size(); ++k) std::sort(key.begin() + start[k], key.begin() + start[k + 1]);
    sorted.resize(faces.size());
    for (size_t k = 0; k < key.size(); ++k) sorted[k] = faces[key[k] & 0xffffffffULL];
    flat.resize(4 * sorted.size());
    for (size_t k = 0; k < sorted.size(); ++k) {
        std::copy(sorted[k].begin(), sorted[k].end(), flat.begin() + 4 * k);
        if (k == 0 || sorted[k][0] != sorted[k - 1][0]) {
            groups.push_back((int)k);
            groups.push_back(0);
        }
        ++groups.back();
    }
}

}  // namespace wp
