// Test driver (CPU): prints the dense cell matrix G that the library composes for one
// half step (cellmap.cpp), for a problem given on the command line, so that the tests
// can apply it to corner data and compare with the oracle.
//   usage: cellmap_dump d m variant lam2_0 lam2_1 tau taylor_stages
// variant: 0 dissipative full, 1 dissipative simple, 2 conservative.  The time-sum
// weights are filled as the library's problem descriptor defines them (F, cuQ, cuR,
// cvQ, cvR; see hw_device.h).  Output: n_in n_out, then G row by row (input-major).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "hw_kernels.h"

static double fact(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

int main(int argc, char** argv)
{
    if (argc != 8) return 2;
    ProblemDesc D;
    std::memset(&D, 0, sizeof D);
    D.d = std::atoi(argv[1]);
    D.m = std::atoi(argv[2]);
    D.variant = std::atoi(argv[3]);
    const double lam2[2] = {std::atof(argv[4]), std::atof(argv[5])};
    const double tau = std::atof(argv[6]);
    const int S = std::atoi(argv[7]);
    D.tau = tau;
    for (int i = 0; i < 3; ++i) {
        const double q = i < D.d ? lam2[i] : 0.0;
        D.lam2[i] = q;
        for (int a = 0; a <= HW_MAXM + 1; ++a)
            for (int b = 0; b <= HW_MAXM + 1; ++b) D.F[i][a][b] = fact(a + 2 * b) / fact(a) * std::pow(q, b) / fact(b);
    }
    auto keep = [S](int s) { return S <= 0 || s <= S; };
    for (int j = 0; j < HW_MAXJ; ++j) {
        const double jf = fact(j);
        if (D.variant == HWV_CONS) {
            D.cuQ[j] = jf / fact(2 * j);
            D.cuR[j] = tau * jf / fact(2 * j + 1);
        } else {
            D.cuQ[j] = keep(2 * j + 1) ? tau * jf / fact(2 * j + 1) : 0.0;
            D.cuR[j] = keep(2 * j + 2) ? jf / fact(2 * j + 2) : 0.0;
            D.cvQ[j] = keep(2 * j) ? jf / fact(2 * j) : 0.0;
            D.cvR[j] = keep(2 * j + 1) ? jf / (tau * fact(2 * j + 1)) : 0.0;
        }
    }
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
