// Dense matrix of one half step on one cell (host side).
//
// The half step maps the data of a cell's 2^d corner nodes linearly to its output
// node (Sec. 3.1 and Sec. 4.1: interpolate, evolve the Taylor series in time, evaluate
// at the centre).  The map is the same for every cell of a problem (the corners of
// cells at non-periodic walls are mirrored images, Sec. 3.1.3, applied to the data
// before the map), so it can be formed once per problem as a matrix G and applied per
// cell as a dense product.  G is composed here in FP64 from the same pieces the
// generic kernel applies one dimension at a time: the 1-D Hermite operators, the
// scaled second-derivative rows of the modified first step, and the closed-form
// time-sum weights of the problem descriptor (which carry lambda, tau and any
// truncation of the series).
#include "hw_kernels.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <vector>

#include "hermite_tables.h"


// Closed-form time-sum weights of the problem descriptor (Sec. 3.1.2 and Sec. 3.3 for
// the dissipative method, Sec. 4.1 eq. (convUpdate) and Sec. 4.3 for the conservative
// one): with tau = dt/2 and q_i = (lambda_i/2)^2, lambda_i = c dt / h_i,
//   F[i][a][b] = (a+2b)!/a! q_i^b / b!   (one dimension's factor of (tau^2 L)^j),
//   dissipative: cuQ[j] = tau j!/(2j+1)!, cuR[j] = j!/(2j+2)!, cvQ[j] = j!/(2j)!,
//                cvR[j] = j!/(tau (2j+1)!), each zero where its stage (2j+1, 2j+2, 2j,
//                2j+1) lies beyond a taylor_stages truncation;
//   conservative: cuQ[j] = j!/(2j)!, cuR[j] = tau j!/(2j+1)! (start-up odd sum).
void hw_fill_weights(const hw_problem& p, const double h[3], ProblemDesc& D)
{
    auto fact = [](int n) {
        double r = 1.0;
        for (int i = 2; i <= n; ++i) r *= i;
        return r;
    };
    const double tau = 0.5 * p.dt;
    D.tau = tau;
    std::memset(D.F, 0, sizeof D.F);
    for (int i = 0; i < 3; ++i) {
        const double lam = (i < p.d) ? p.c * p.dt / h[i] : 0.0;
        const double q = 0.25 * lam * lam;
        D.lam2[i] = q;
        for (int a = 0; a <= HW_MAXM + 1; ++a)
            for (int b = 0; b <= HW_MAXM + 1; ++b)
                D.F[i][a][b] = fact(a + 2 * b) / fact(a) * std::pow(q, b) / fact(b);
    }
    const int S = p.taylor_stages;
    auto keep = [S](int s) { return S <= 0 || s <= S; };
    for (int j = 0; j < HW_MAXJ; ++j) {
        const double jf = fact(j);
        if (p.method == HW_CONSERVATIVE) {
            D.cuQ[j] = jf / fact(2 * j);
            D.cuR[j] = tau * jf / fact(2 * j + 1);
            D.cvQ[j] = D.cvR[j] = 0.0;
        } else {
            D.cuQ[j] = keep(2 * j + 1) ? tau * jf / fact(2 * j + 1) : 0.0;
            D.cuR[j] = keep(2 * j + 2) ? jf / fact(2 * j + 2) : 0.0;
            D.cvQ[j] = keep(2 * j) ? jf / fact(2 * j) : 0.0;
            D.cvR[j] = keep(2 * j + 1) ? jf / (tau * fact(2 * j + 1)) : 0.0;
        }
    }
}

namespace {

int ipow_h(int b, int e)
{
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// One 1-D operator: value of row r at input (side s, coefficient l).
struct Op1 {
    const double* H = nullptr; // row-major, `ld` columns, column s * md + l
    int ld = 0, md = 0;
    int row_shift = 0;     // row r reads row r + row_shift of H
    bool d2 = false;       // scale row r by (r + 2)(r + 1)
    int lmax = 1 << 20;    // inputs with l >= lmax are cut (data truncated)
    double at(int r, int s, int l) const
    {
        if (l >= lmax) return 0.0;
        const double w = H[(r + row_shift) * ld + s * md + l];
        return d2 ? w * (r + 2) * (r + 1) : w;
    }
};

struct Layout {
    int d, nu, nv, mu, mv; // coefficients per node (u, v) and per dimension
    int n_in() const { return (1 << d) * (nu + nv); }
};

// rows R^d of the tensor product of ops[0..d-1] applied to the u (vblock = false) or v
// block of every corner: mat[k][in]
std::vector<double> tensor(const Layout& L, const std::array<Op1, 3>& ops, int R, bool vblock)
{
    const int rows = ipow_h(R, L.d), n_in = L.n_in();
    const int md = vblock ? L.mv : L.mu, ncoef = vblock ? L.nv : L.nu;
    std::vector<double> mat((size_t)rows * n_in, 0.0);
    for (int k = 0; k < rows; ++k) {
        int kk[3] = {0, 0, 0};
        for (int i = 0, rem = k; i < L.d; ++i, rem /= R) kk[i] = rem % R;
        for (int c = 0; c < (1 << L.d); ++c)
            for (int l = 0; l < ncoef; ++l) {
                double w = 1.0;
                for (int i = 0, rem = l; i < L.d; ++i, rem /= md) w *= ops[i].at(kk[i], (c >> i) & 1, rem % md);
                mat[(size_t)k * n_in + c * (L.nu + L.nv) + (vblock ? L.nu : 0) + l] += w;
            }
    }
    return mat;
}

} // namespace

bool hw_dense_supported(int d, int m, int method, int precision)
{
    if (precision != 0 && precision != 1) return false;
    if (d == 1) return method == 2 ? m >= 0 && m <= 6 : m >= 1 && m <= 6;
    // 2-D conservative m = 6: the composed matrix sums terms of up to ~1e4 times the result,
    // so its rounding error exceeds the factorised kernel's several times; the generic
    // kernel keeps that case
    if (d == 2) return method == 2 ? m >= 0 && m <= 5 : m >= 1 && m <= 6;
    return false;
}

void hw_cell_map(const ProblemDesc& D, std::vector<double>& G, int& n_in, int& n_out)
{
    const int d = D.d, m = D.m, M = m + 1, P = 2 * m + 2;
    const bool cons = D.variant == HWV_CONS;
    const bool simple = D.variant == HWV_DISS_SIMPLE || d == 1;
    Layout L{d, ipow_h(M, d), cons ? 0 : ipow_h(m, d), M, m};
    n_in = L.n_in();
    n_out = cons ? L.nu : L.nu + L.nv;
    const double* Hm = kHermiteAll + kHermiteOffset[m];
    Op1 full{Hm, P, M};
    Op1 d2{Hm, P, M, 2, true};
    Op1 tr, vop;
    if (m >= 1) {
        const double* Hv = kHermiteAll + kHermiteOffset[m - 1];
        tr = Op1{Hv, 2 * m, m};
        tr.lmax = m; // u data truncated to l <= m-1, columns s * m + l of H_{m-1}
        vop = Op1{Hv, 2 * m, m};
    }
    // coefficient fields as rows over the inputs
    const int E = cons ? P : (simple ? P : 2 * m); // extent of Q and R (and A)
    const int P0E = simple ? P : M;                // extent of p0
    std::vector<double> p0, Q, R, A;
    const int ED = ipow_h(E, d), n = n_in;
    if (cons) {
        A = tensor(L, {full, full, full}, P, false);
    } else if (!simple) {
        Op1 fc = full; // centre rows 0..m
        p0 = tensor(L, {fc, fc, fc}, M, false);
        Q = tensor(L, {vop, vop, vop}, 2 * m, true);
        R.assign((size_t)ED * n, 0.0);
        for (int i = 0; i < d; ++i) {
            std::array<Op1, 3> ops{tr, tr, tr};
            ops[i] = d2;
            const std::vector<double> c = tensor(L, ops, 2 * m, false);
            for (size_t e = 0; e < R.size(); ++e) R[e] += D.lam2[i] * c[e];
        }
    } else {
        p0 = tensor(L, {full, full, full}, P, false);
        Q.assign((size_t)ED * n, 0.0);
        if (m >= 1) {
            const std::vector<double> q0 = tensor(L, {vop, vop, vop}, 2 * m, true);
            const int KvD = ipow_h(2 * m, d);
            for (int e = 0; e < KvD; ++e) {
                int off = 0;
                for (int i = 0, rem = e, st = 1; i < d; ++i, rem /= 2 * m, st *= P) off += (rem % (2 * m)) * st;
                for (int in = 0; in < n; ++in) Q[(size_t)off * n + in] = q0[(size_t)e * n + in];
            }
        }
        R.assign((size_t)ED * n, 0.0);
        for (int e = 0; e < ED; ++e)
            for (int i = 0, st = 1; i < d; ++i, st *= P) {
                const int k = (e / st) % P;
                if (k + 2 >= P) continue;
                const double w = D.lam2[i] * (k + 2) * (k + 1);
                for (int in = 0; in < n; ++in) R[(size_t)e * n + in] += w * p0[(size_t)(e + 2 * st) * n + in];
            }
    }

    // closed-form time sums: output alpha = sum over beta with alpha + 2 beta < E of
    // g(alpha, beta) (coefficient of Q, R or A by j = |beta|)
    G.assign((size_t)n_in * n_out, 0.0);
    std::vector<double> row(n);
    for (int o = 0; o < n_out; ++o) {
        const bool is_u = o < L.nu;
        const int c = is_u ? o : o - L.nu, Mo = is_u ? M : m;
        int a[3] = {0, 0, 0}, bmax[3] = {0, 0, 0};
        for (int i = 0, rem = c; i < d; ++i, rem /= Mo) {
            a[i] = rem % Mo;
            bmax[i] = (E - 1 - a[i]) / 2;
        }
        std::fill(row.begin(), row.end(), 0.0);
        if (is_u && !cons) {
            int off = 0;
            for (int i = 0, st = 1; i < d; ++i, st *= P0E) off += a[i] * st;
            for (int in = 0; in < n; ++in) row[in] = p0[(size_t)off * n + in];
        }
        const double* cq = is_u ? D.cuQ : D.cvQ;
        const double* cr = is_u ? D.cuR : D.cvR;
        for (int b2 = 0; b2 <= (d > 2 ? bmax[2] : 0); ++b2)
            for (int b1 = 0; b1 <= (d > 1 ? bmax[1] : 0); ++b1)
                for (int b0 = 0; b0 <= bmax[0]; ++b0) {
                    const int b[3] = {b0, b1, b2};
                    double g = 1.0;
                    int idx = 0;
                    for (int i = 0, st = 1; i < d; ++i, st *= E) {
                        g *= D.F[i][a[i]][b[i]];
                        idx += (a[i] + 2 * b[i]) * st;
                    }
                    const int j = b0 + b1 + b2;
                    if (cons) {
                        const double w = g * D.cuQ[j];
                        for (int in = 0; in < n; ++in) row[in] += w * A[(size_t)idx * n + in];
                    } else {
                        const double wq = g * cq[j], wr = g * cr[j];
                        for (int in = 0; in < n; ++in)
                            row[in] += wq * Q[(size_t)idx * n + in] + wr * R[(size_t)idx * n + in];
                    }
                }
        for (int in = 0; in < n; ++in) G[(size_t)in * n_out + o] = row[in];
    }
}
