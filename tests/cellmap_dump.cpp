// Test driver (CPU): prints the dense cell matrix G that the library composes for one
// half step (cellmap.cpp), for a problem given on the command line, so that the tests
// can apply it to corner data and compare with the oracle.  The problem descriptor's
// time-sum weights come from the library's own hw_fill_weights.
//   usage: cellmap_dump d m method c dt h0 h1 taylor_stages
// method: 0 dissipative full, 1 dissipative simple, 2 conservative.
// Output: n_in n_out, then G row by row (input-major).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hw_kernels.h"

int main(int argc, char** argv)
{
    if (argc != 9) return 2;
    hw_problem p;
    std::memset(&p, 0, sizeof p);
    p.d = std::atoi(argv[1]);
    p.m = std::atoi(argv[2]);
    p.method = std::atoi(argv[3]);
    p.c = std::atof(argv[4]);
    p.dt = std::atof(argv[5]);
    const double h[3] = {std::atof(argv[6]), std::atof(argv[7]), 1.0};
    p.taylor_stages = std::atoi(argv[8]);
    ProblemDesc D;
    std::memset(&D, 0, sizeof D);
    D.d = p.d;
    D.m = p.m;
    D.variant = p.method == HW_CONSERVATIVE ? HWV_CONS : (p.method == HW_DISS_SIMPLE ? HWV_DISS_SIMPLE : HWV_DISS_FULL);
    hw_fill_weights(p, h, D);
    std::vector<double> G;
    int n_in = 0, n_out = 0;
    hw_cell_map(D, G, n_in, n_out);
    std::printf("%d %d\n", n_in, n_out);
    for (int i = 0; i < n_in; ++i) {
        for (int o = 0; o < n_out; ++o) std::printf("%.17g ", G[(size_t)i * n_out + o]);
        std::printf("\n");
    }
    return 0;
}
