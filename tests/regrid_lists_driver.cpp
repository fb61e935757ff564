// Reads patch layouts on stdin and prints the regrid lists that
// regrid_lists.h builds for them, one list per line, for
// test_regrid_lists.py to check against mask-based definitions.
//
// Input per case: nx ny r NX NY, then n and n patches (ilo jlo nx ny), then
// m and m old patches.  Output per case: the ring cells, the ring blocks,
// the covered coarse cells, the new cells, the faces and the face groups.
#include <cstdio>
#include <vector>

#include "regrid_lists.h"

static void put(const std::vector<int> &v)
{
    std::printf("%zu", v.size());
    for (int x : v) std::printf(" %d", x);
    std::printf("\n");
}

static bool get(std::vector<wp_patch> &P)
{
    int n;
    if (std::scanf("%d", &n) != 1) return false;
    P.resize(n);
    for (wp_patch &p : P)
        if (std::scanf("%d %d %d %d", &p.ilo, &p.jlo, &p.nx, &p.ny) != 4) return false;
    return true;
}

int main()
{
    int nx, ny, r, NX, NY;
    while (std::scanf("%d %d %d %d %d", &nx, &ny, &r, &NX, &NY) == 5) {
        std::vector<wp_patch> P, Q;
        if (!get(P) || !get(Q)) return 1;
        std::vector<std::array<int, 3>> runs;
        std::vector<int> v;
        wp::ring_runs(P, nx, ny, runs);
        wp::run_cells(runs, nx, v);
        put(v);
        v.clear();
        if (r <= 8) wp::ring_block_list(runs, r, NX, v);
        put(v);
        wp::cover_cells(P, r, NX, v);
        put(v);
        wp::fresh_cells(P, Q, nx, ny, v);
        put(v);
        std::vector<int> flat, groups;
        wp::reflux_faces(P, r, NX, NY, flat, groups);
        put(flat);
        put(groups);
    }
    return 0;
}
