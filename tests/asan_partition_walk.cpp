// Host-only walk over the partition builder's C ABI (dd_partition and its
// queries) on regular, overlapping, tiled, 3D and degenerate layouts, built
// with AddressSanitizer on the host side: out-of-bounds writes into exactly
// sized output arrays, use after free and leaks end the program with an error.
// No device call is made.
#include <cstdio>
#include <vector>
#include "cbd.h"
int main() {
    struct C { int d, n, m, delta, mode, leaf; };
    std::vector<C> cs = {{2,64,16,1,2,0},{2,256,4,8,1,8},{2,48,12,1,2,0},{2,60,6,2,2,4},{2,32,4,1,0,0},
                         {2,16,2,1,2,0},{3,32,4,1,2,0},{3,12,4,1,1,3},{2,512,64,1,2,0},{2,512,1,0,0,8},
                         {3,64,8,1,2,0},{2,2,1,0,0,0},{3,2,1,0,0,0},{2,128,128,0,0,0}};
    long tot = 0;
    for (auto c : cs) {
        cbd_partition q = nullptr;
        int rc = dd_partition(c.d, c.n, c.m, c.delta, c.mode, c.leaf, &q);
        if (rc) { printf("case %d %d %d: rc %d %s\n", c.d, c.n, c.m, rc, cbd_last_error()); continue; }
        int D, Lt, Lr; long total;
        dd_partition_info(q, &D, &Lt, &Lr, &total);
        for (int i = 0; i < D; ++i) {
            int size, nl, rl;
            dd_subdomain_info(q, i, &size, &nl, &rl);
            std::vector<int> idx(size);
            dd_subdomain_index(q, i, idx.data());
            for (int l = 0; l <= rl; ++l) {
                int nb = 0;
                dd_level_boxes(q, i, l, &nb, nullptr, nullptr);
                std::vector<int> lohi(nb * 2 * c.d), par(nb);
                dd_level_boxes(q, i, l, &nb, lohi.data(), par.data());
                tot += nb;
            }
            tot += size;
        }
        dd_subdomain_info(q, D, nullptr, nullptr, nullptr);
        dd_level_boxes(q, 0, 99, nullptr, nullptr, nullptr);
        cbd_partition_free(q);
    }
    printf("asan partition walk ok, %ld\n", tot);
    return 0;
}
