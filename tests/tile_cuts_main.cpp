// Prints the sink-tile cut of the library's work list for a range of cell sizes, for the host-side test of its
// invariants: one line per (n, S, max_lanes) with the tile count and each tile as L,G,t0,nt.
#include <cstdio>

#include "../paper_2110_11398_amd/csrc/nf_internal.h"

int main() {
    const int lanes[] = {1, 2, 3, 5, 7, 8, 16, 21, 64};
    const int sinks[] = {1, 2, 4};
    for (int ml : lanes)
        for (int S : sinks)
            for (int n = 1; n <= 1100; n++) {
                const int c = anf::tile_count(n, S, ml);
                printf("%d %d %d %d", n, S, ml, c);
                for (int t = 0; t < c; t++) {
                    const anf::TileGeom g = anf::tile_at(n, S, ml, t);
                    printf(" %d,%d,%d,%d", g.L, g.G, g.t0, g.nt);
                }
                printf("\n");
            }
    return 0;
}
