// Generic half-step kernels: one 64-lane workgroup per output node ("cell"),
// grid-stride over a work list of (problem, cell), any d <= 3, any m <= 6.
//
// Per cell: gather the 2^d corner nodes into LDS (ghost corners by odd/even
// mirroring, Sec. 3.1.3), build the tensor-product Hermite interpolants one
// dimension at a time (Sec. 2.2, the dimension-by-dimension reconstruction of
// Sec. 6), evaluate the Taylor series in time at t + dt/2 with closed-form weights,
// and store the output node.
//
// Time evolution (Sec. 3.1.2 and Sec. 3.3, dissipative).  With L = c^2 Lap acting
// on scaled coefficients, Q = I_{m-1..m-1} v, and R = tau^2 c^2 sum_i d_i^2 c^(i)
// (c^(i) = I_{m-1,..,m (dim i),..,m-1} u for the modified first step, c^(i) =
// I_{m..m} u for the straightforward extension), the recursion of the paper sums
// in closed form to
//   u' = p0 + tau sum_j (tau^2 L)^j Q/(2j+1)! + sum_j (tau^2 L)^j R/(2j+2)!
//   v' =      sum_j (tau^2 L)^j Q/(2j)!     + (1/tau) sum_j (tau^2 L)^j R/(2j+1)!
// with [(tau^2 L)^j a]_alpha = sum_{|beta| = j} j!/prod beta_i!
//   prod_i (alpha_i + 2 beta_i)!/alpha_i! (lambda_i/2)^(2 beta_i) a_{alpha + 2 beta}.
// Conservative (Sec. 4.1 eq. (convUpdate), Sec. 4.3): u_new = 2 sum_j
// (tau^2 L)^j a/(2j)! - u_old with a = I_{m..m} u, the Pascal-matrix formula of
// Sec. 4.3 with the factor (c dt/(2h))^2i.

#include <mutex>

#include "hw_device.h"
#include "hw_kernels.h"

#define GW 64

namespace {

__device__ __forceinline__ int ipow(int b, int e)
{
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

// Apply one 1-D operator per dimension, dims 0..D-1 in turn.  `in` has extent K in
// every dimension (x fastest); ops[dim] is R[dim] x (current extent) row-major.  The
// last pass writes (or accumulates, scaled) into dest.  bufA/bufB: scratch of
// K^D elements each, not aliasing in or dest.
template <typename T, int D>
__device__ void tensor_apply(const T* in, int K, const T* const* ops, const int* R, T* bufA,
                             T* bufB, T* dest, T scale, bool accumulate, int lane)
{
    int ext[3] = {K, K, K};
    const T* src = in;
    for (int dim = 0; dim < D; ++dim) {
        const bool last = (dim == D - 1);
        T* dst = last ? dest : ((dim & 1) ? bufB : bufA);
        int stride = 1;
        for (int i = 0; i < dim; ++i) stride *= ext[i];
        int outer = 1;
        for (int i = dim + 1; i < D; ++i) outer *= ext[i];
        const int Kd = ext[dim], Rd = R[dim];
        const T* op = ops[dim];
        const int total = stride * Rd * outer;
        for (int e = lane; e < total; e += GW) {
            const int lo = e % stride;
            const int r = (e / stride) % Rd;
            const int hi = e / (stride * Rd);
            const T* s = src + lo + hi * stride * Kd;
            const T* o = op + r * Kd;
            T a = T(0);
            // four terms per round: their LDS reads are in flight together
            int k = 0;
            for (; k + 4 <= Kd; k += 4) {
                const T o0 = o[k], o1 = o[k + 1], o2 = o[k + 2], o3 = o[k + 3];
                const T s0 = s[k * stride], s1 = s[(k + 1) * stride], s2 = s[(k + 2) * stride],
                        s3 = s[(k + 3) * stride];
                a += o0 * s0;
                a += o1 * s1;
                a += o2 * s2;
                a += o3 * s3;
            }
            for (; k < Kd; ++k) a += o[k] * s[k * stride];
            if (last) {
                if (accumulate) dst[e] += scale * a;
                else dst[e] = scale * a;
            } else {
                dst[e] = a;
            }
        }
        __syncthreads();
        ext[dim] = Rd;
        src = dst;
    }
}

struct Corners {
    int node[3][2];  // input node index per dimension and side
    int ghost[3][2]; // 1 if that corner lies outside a non-periodic wall
};

struct Geom {
    int bc[3], ext_from[3], ext_to[3], to_grid;
};

template <int D>
__device__ void find_corners(const Geom& G, int64_t cell, Corners& cr)
{
    int64_t c = cell;
    for (int i = 0; i < D; ++i) {
        const int oi = (int)(c % G.ext_to[i]);
        c /= G.ext_to[i];
        const int ext = G.ext_from[i];
        for (int s = 0; s < 2; ++s) {
            int j, gh = 0;
            if (G.to_grid == 1) {          // dual node i+1/2: primal i, i+1
                j = oi + s;
                if (G.bc[i] == 0 && j >= ext) j -= ext;
            } else {                       // primal node i: dual i-1/2, i+1/2
                j = oi - 1 + s;
                if (G.bc[i] == 0) {
                    if (j < 0) j += ext;
                } else if (j < 0) {
                    j = 0;
                    gh = 1;
                } else if (j >= ext) {
                    j = ext - 1;
                    gh = 1;
                }
            }
            cr.node[i][s] = j;
            cr.ghost[i][s] = gh;
        }
    }
}

template <int D>
__device__ inline Geom geom_of(const ProblemDesc& P)
{
    Geom G;
    for (int i = 0; i < 3; ++i) {
        G.bc[i] = P.bc[i];
        G.ext_from[i] = P.ext_from[i];
        G.ext_to[i] = P.ext_to[i];
    }
    G.to_grid = P.to_grid;
    return G;
}

// Wall points of the face normal to dimension i: the input grid's nodes in the other
// dimensions, one ghost position added at each end of a non-periodic one.
template <int D>
__device__ int64_t face_points(const Geom& P, int i)
{
    int64_t n = 1;
    for (int t = 0; t < D; ++t)
        if (t != i) n *= (P.bc[t] == 0) ? P.ext_from[t] : P.ext_from[t] + 2;
    return n;
}

// Inhomogeneous wall data of ghost corner s at coefficient l (Sec. 3.1.3): the sum over
// its ghost dimensions r (applied in increasing order) of 2 W_r at the ghost position,
// times the reflection signs of the ghost dimensions applied after r.  W_r at the ghost
// is the record's normal expansion (degrees 2j Dirichlet, 2j+1 Neumann, about the wall)
// shifted by half a cell outwards.  The record is read at the wall point whose
// tangential positions are the corner's after the dimensions before r were reflected.
template <int D>
__device__ double wall_term(const Geom& P, const Corners& cr, const int* s, const int* l, int Md,
                            const double* __restrict__ rec)
{
    const int rs = ipow(Md, D);
    double total = 0.0;
    for (int r = 0; r < D; ++r) {
        if (!cr.ghost[r][s[r]]) continue;
        double sgn = 1.0;
        for (int g = r + 1; g < D; ++g)
            if (cr.ghost[g][s[g]]) {
                const bool odd = (l[g] & 1);
                if ((P.bc[g] == 1) ? !odd : odd) sgn = -sgn;
            }
        int64_t off = 0;
        for (int i = 0; i < r; ++i)
            if (P.bc[i] != 0) off += 2 * face_points<D>(P, i);
        if (s[r] == 1) off += face_points<D>(P, r);
        int64_t pt = 0, stride = 1;
        for (int t = 0; t < D; ++t) {
            if (t == r) continue;
            int pos, ext;
            if (P.bc[t] == 0) {
                ext = P.ext_from[t];
                pos = cr.node[t][s[t]];
            } else {
                ext = P.ext_from[t] + 2;
                if (t < r && cr.ghost[t][s[t]]) pos = s[t] == 0 ? 0 : P.ext_from[t] + 1;
                else pos = cr.node[t][s[t]] + 1;
            }
            pt += pos * stride;
            stride *= ext;
        }
        const double* rw = rec + (off + pt) * rs;
        const double delta = s[r] == 0 ? -0.5 : 0.5;
        double sum = 0.0;
        for (int j = 0; j < Md; ++j) {
            const int k = (P.bc[r] == 1) ? 2 * j : 2 * j + 1;
            if (k < l[r]) continue;
            int c = 0, cs = 1;
            for (int t = 0; t < D; ++t) {
                c += (t == r ? j : l[t]) * cs;
                cs *= Md;
            }
            // binomial(k, l_r) delta^(k - l_r)
            double b = 1.0;
            for (int q = 0; q < l[r]; ++q) b = b * (k - q) / (q + 1);
            for (int q = 0; q < k - l[r]; ++q) b *= delta;
            sum += b * rw[c];
        }
        total += sgn * 2.0 * sum;
    }
    return total;
}

// Gather corner data into the mixed layout j_i = s_i*Md + l_i (extent 2*Md per dim).
// Mirrored corners: coefficient l along the wall normal times (-1)^(l+1) for
// Dirichlet, (-1)^l for Neumann, plus the wall data's term when `walls` is given;
// with `zero_base` the node data count as zero (only the wall terms are gathered).
template <typename T, int D>
__device__ void gather(const Geom& P, const Corners& cr, const T* __restrict__ data, int Md,
                       T* X, int lane, const double* walls = nullptr, bool zero_base = false)
{
    const int K = 2 * Md;
    const int total = ipow(K, D);
    const int ncoef = ipow(Md, D);
    for (int e = lane; e < total; e += GW) {
        int rem = e, node = 0, nstride = 1, coef = 0, cstride = 1;
        int sv[3] = {0, 0, 0}, lv[3] = {0, 0, 0};
        bool any_ghost = false;
        T sign = T(1);
        for (int i = 0; i < D; ++i) {
            const int jd = rem % K;
            rem /= K;
            const int s = jd / Md, l = jd % Md;
            sv[i] = s;
            lv[i] = l;
            node += cr.node[i][s] * nstride;
            nstride *= P.ext_from[i];
            coef += l * cstride;
            cstride *= Md;
            if (cr.ghost[i][s]) {
                any_ghost = true;
                const bool odd = (l & 1);
                const bool neg = (P.bc[i] == 1) ? !odd : odd;
                if (neg) sign = -sign;
            }
        }
        T x = zero_base ? T(0) : sign * data[(int64_t)node * ncoef + coef];
        if (walls && any_ghost) x += T(wall_term<D>(P, cr, sv, lv, Md, walls));
        X[e] = x;
    }
}

// Tables of the current problem staged in LDS (ahead of the cell scratch): the block of
// 1-D operators of its m (H_m, scaled second-derivative rows, H_{m-1} on u and on v)
// and the time-sum weights F[3][8][8], cuQ, cuR, cvQ, cvR (FP64).
constexpr int TAB_OPS = 680; // >= operator block of m = 6: 14*14 + 2*12*14 + 12*12
constexpr int TAB_W = 3 * (HW_MAXM + 2) * (HW_MAXM + 2) + 4 * HW_MAXJ;
__host__ __device__ constexpr int ops_len(int m)
{
    return (2 * m + 2) * (2 * m + 2) + 2 * m * (2 * m + 2) + (m >= 1 ? 2 * m * (2 * m + 2) + 4 * m * m : 0);
}
template <typename T>
__host__ __device__ constexpr size_t tab_bytes()
{
    return ((TAB_OPS * sizeof(T) + 15) / 16) * 16 + TAB_W * sizeof(double);
}
static_assert(ops_len(HW_MAXM) <= TAB_OPS, "operator block must fit its LDS region");

struct WTab {
    const double* F; // [3][HW_MAXM + 2][HW_MAXM + 2]
    const double *cuQ, *cuR, *cvQ, *cvR;
    __device__ double f(int i, int a, int b) const { return F[(i * (HW_MAXM + 2) + a) * (HW_MAXM + 2) + b]; }
};

template <typename T, int D>
__device__ void diss_cell(const ProblemDesc& P, const T* lops, const WTab& WT, int64_t cell, T* sm,
                          int lane, const ForcingArgs& FA)
{
    const int m = P.m, M = m + 1, Pn = 2 * m + 2, K = Pn, Kv = 2 * m;
    const bool simple = (P.variant == HWV_DISS_SIMPLE) || D == 1;
    const int E = simple ? Pn : 2 * m;
    const int KD = ipow(K, D), ED = ipow(E, D);
    T* Xu = sm;
    T* Xv = Xu + KD;
    T* bufA = Xv + ipow(Kv, D);
    T* bufB = bufA + KD;
    T* Q = bufB + KD;
    T* Rr = Q + ED;
    T* P0 = Rr + ED; // M^D (full variant) or Pn^D (simple)

    const int P0E = simple ? Pn : M;
    const int n_p0 = ipow(P0E, D);
    T* wk = (T*)P.work + cell * (int64_t)P.work_stride; // split form: p0 | Q | R
    if (P.split == 2) {
        // time evolution only: the interpolants come from the first kernel
        for (int e = lane; e < n_p0; e += GW) P0[e] = wk[e];
        for (int e = lane; e < ED; e += GW) {
            Q[e] = wk[n_p0 + e];
            Rr[e] = wk[n_p0 + ED + e];
        }
        __syncthreads();
    } else {
    Corners cr;
    const Geom G = geom_of<D>(P);
    find_corners<D>(G, cell, cr);
    const bool walls = P.to_grid == 0 && FA.wall_u != nullptr;
    gather<T, D>(G, cr, (const T*)P.u_in, M, Xu, lane, walls ? FA.wall_u : nullptr, FA.correction != 0);
    gather<T, D>(G, cr, (const T*)P.v_in, m, Xv, lane, walls ? FA.wall_v : nullptr, FA.correction != 0);
    __syncthreads();

    const T* full = lops;
    const T* d2 = lops + (P.op.d2 - P.op.full);
    const T* tr = lops + (P.op.trunc - P.op.full);
    const T* vop = lops + (P.op.vop - P.op.full);
    const T* o3[3];
    int R3[3];

    // p0 = I_{m..m} u: centre rows 0..m only (modified variant), all rows (simple)
    for (int i = 0; i < 3; ++i) {
        o3[i] = full;
        R3[i] = simple ? Pn : M;
    }
    tensor_apply<T, D>(Xu, K, o3, R3, bufA, bufB, P0, T(1), false, lane);

    // Q = I_{m-1..m-1} v
    for (int i = 0; i < 3; ++i) {
        o3[i] = vop;
        R3[i] = Kv;
    }
    if (!simple) {
        tensor_apply<T, D>(Xv, Kv, o3, R3, bufA, bufB, Q, T(1), false, lane);
        // R = sum_i (lambda_i/2)^2 (k_i+2)(k_i+1) c^(i)_{k+2e_i}
        for (int i = 0; i < D; ++i) {
            for (int j = 0; j < 3; ++j) {
                o3[j] = (j == i) ? d2 : tr;
                R3[j] = Kv;
            }
            tensor_apply<T, D>(Xu, K, o3, R3, bufA, bufB, Rr, T(P.lam2[i]), i > 0, lane);
        }
    } else {
        // q0 has extent 2m; embed into Q with extent Pn (zero padded)
        tensor_apply<T, D>(Xv, Kv, o3, R3, bufA, bufB, Rr, T(1), false, lane);
        const int KvD = ipow(Kv, D);
        for (int e = lane; e < ED; e += GW) Q[e] = T(0);
        __syncthreads();
        for (int e = lane; e < KvD; e += GW) {
            int rem = e, off = 0, st = 1;
            for (int i = 0; i < D; ++i) {
                off += (rem % Kv) * st;
                rem /= Kv;
                st *= Pn;
            }
            Q[off] = Rr[e];
        }
        __syncthreads();
        // R = sum_i (lambda_i/2)^2 (k_i+2)(k_i+1) p0_{k+2e_i}
        for (int e = lane; e < ED; e += GW) {
            T acc = T(0);
            int st = 1;
            for (int i = 0; i < D; ++i) {
                const int k = (e / st) % Pn;
                if (k + 2 < Pn) acc += T(P.lam2[i] * (k + 2) * (k + 1)) * P0[e + 2 * st];
                st *= Pn;
            }
            Rr[e] = acc;
        }
        __syncthreads();
    }
    if (P.split == 1) {
        // interpolation only: hand p0, Q and R to the second kernel through memory
        for (int e = lane; e < n_p0; e += GW) wk[e] = P0[e];
        for (int e = lane; e < ED; e += GW) {
            wk[n_p0 + e] = Q[e];
            wk[n_p0 + ED + e] = Rr[e];
        }
        return;
    }
    }

    // time sums at tau = dt/2, one output coefficient per lane
    const int Mu_tot = ipow(M, D), Mv_tot = ipow(m, D);
    T* uo = (T*)P.u_out + cell * Mu_tot;
    T* vo = (T*)P.v_out + cell * Mv_tot;
    for (int o = lane; o < Mu_tot + Mv_tot; o += GW) {
        const bool is_u = o < Mu_tot;
        const int c = is_u ? o : o - Mu_tot;
        const int Mo = is_u ? M : m;
        int a[3] = {0, 0, 0}, bmax[3] = {0, 0, 0};
        int rem = c;
        for (int i = 0; i < D; ++i) {
            a[i] = rem % Mo;
            rem /= Mo;
            bmax[i] = (E - 1 - a[i]) / 2;
        }
        T acc = T(0);
        if (is_u) {
            int off = 0, st = 1;
            for (int i = 0; i < D; ++i) {
                off += a[i] * st;
                st *= P0E;
            }
            acc = P0[off];
        }
        const double* cq = is_u ? WT.cuQ : WT.cvQ;
        const double* crr = is_u ? WT.cuR : WT.cvR;
        for (int b2 = 0; b2 <= bmax[2]; ++b2)
            for (int b1 = 0; b1 <= bmax[1]; ++b1)
                for (int b0 = 0; b0 <= bmax[0]; ++b0) {
                    const int j = b0 + b1 + b2;
                    double g = WT.f(0, a[0], b0);
                    if (D > 1) g *= WT.f(1, a[1], b1);
                    if (D > 2) g *= WT.f(2, a[2], b2);
                    const int idx = (a[0] + 2 * b0) + E * ((a[1] + 2 * b1) + E * (a[2] + 2 * b2));
                    acc += T(g * cq[j]) * Q[idx] + T(g * crr[j]) * Rr[idx];
                }
        T* dst = is_u ? uo + c : vo + c;
        *dst = FA.correction ? *dst + acc : acc;
    }
    if (FA.coef == nullptr) return;

    // forcing: u' += sum_r sum_j tau^(r+2)/(2j+r+2)! [L^j f_r], v' += sum_r sum_j
    // tau^(r+1)/(2j+r+1)! [L^j f_r] with [L^j a]_alpha = sum_|beta|=j g(alpha,beta)
    // a_(alpha+2 beta); f_r has extent 2m per dimension.  Every lane adds to the
    // outputs it wrote above.
    const int KvD = ipow(Kv, D);
    const double* fc = FA.coef + cell * (int64_t)FA.orders * KvD;
    for (int r = 0; r < FA.orders; ++r) {
        __syncthreads();
        for (int e = lane; e < KvD; e += GW) bufA[e] = T(fc[(int64_t)r * KvD + e]);
        __syncthreads();
        for (int o = lane; o < Mu_tot + Mv_tot; o += GW) {
            const bool is_u = o < Mu_tot;
            const int c = is_u ? o : o - Mu_tot;
            const int Mo = is_u ? M : m;
            int a[3] = {0, 0, 0}, bmax[3] = {0, 0, 0};
            int rem = c;
            for (int i = 0; i < D; ++i) {
                a[i] = rem % Mo;
                rem /= Mo;
                bmax[i] = (Kv - 1 - a[i]) / 2;
            }
            const double* w = FA.w + ((is_u ? 0 : HW_MAXF) + r) * HW_MAXJ;
            T acc = T(0);
            for (int b2 = 0; b2 <= bmax[2]; ++b2)
                for (int b1 = 0; b1 <= bmax[1]; ++b1)
                    for (int b0 = 0; b0 <= bmax[0]; ++b0) {
                        double g = WT.f(0, a[0], b0);
                        if (D > 1) g *= WT.f(1, a[1], b1);
                        if (D > 2) g *= WT.f(2, a[2], b2);
                        const int idx = (a[0] + 2 * b0) + Kv * ((a[1] + 2 * b1) + Kv * (a[2] + 2 * b2));
                        acc += T(g * w[b0 + b1 + b2]) * bufA[idx];
                    }
            if (is_u) uo[c] += acc;
            else vo[c] += acc;
        }
    }
}

template <typename T, int D>
__device__ void cons_cell(const ProblemDesc& P, const T* lops, const WTab& WT, int64_t cell, T* sm,
                          int lane, const ForcingArgs& FA)
{
    const int m = P.m, M = m + 1, Pn = 2 * m + 2, K = Pn;
    const int KD = ipow(K, D);
    const bool startup = (P.variant == HWV_CONS_STARTUP) && P.v_in != nullptr;
    T* Xu = sm;
    T* Xv = Xu + KD;
    T* bufA = Xv + KD;
    T* bufB = bufA + KD;
    T* A = bufB + KD;
    T* B = A + KD;

    Corners cr;
    const Geom G = geom_of<D>(P);
    find_corners<D>(G, cell, cr);
    const bool walls = P.to_grid == 0 && FA.wall_u != nullptr && P.variant == HWV_CONS;
    gather<T, D>(G, cr, (const T*)P.u_in, M, Xu, lane, walls ? FA.wall_u : nullptr, FA.correction != 0);
    if (startup) gather<T, D>(G, cr, (const T*)P.v_in, M, Xv, lane);
    __syncthreads();
    const T* full = lops;
    const T* o3[3] = {full, full, full};
    const int R3[3] = {Pn, Pn, Pn};
    tensor_apply<T, D>(Xu, K, o3, R3, bufA, bufB, A, T(1), false, lane);
    if (startup) tensor_apply<T, D>(Xv, K, o3, R3, bufA, bufB, B, T(1), false, lane);

    const int Mu_tot = ipow(M, D);
    T* uo = (T*)P.u_out + cell * Mu_tot;
    const T* uold = (const T*)P.u_old;
    for (int c = lane; c < Mu_tot; c += GW) {
        int a[3] = {0, 0, 0}, bmax[3] = {0, 0, 0};
        int rem = c;
        for (int i = 0; i < D; ++i) {
            a[i] = rem % M;
            rem /= M;
            bmax[i] = (Pn - 1 - a[i]) / 2;
        }
        T acc = T(0);
        for (int b2 = 0; b2 <= bmax[2]; ++b2)
            for (int b1 = 0; b1 <= bmax[1]; ++b1)
                for (int b0 = 0; b0 <= bmax[0]; ++b0) {
                    const int j = b0 + b1 + b2;
                    double g = WT.f(0, a[0], b0);
                    if (D > 1) g *= WT.f(1, a[1], b1);
                    if (D > 2) g *= WT.f(2, a[2], b2);
                    const int idx = (a[0] + 2 * b0) + Pn * ((a[1] + 2 * b1) + Pn * (a[2] + 2 * b2));
                    acc += T(g * WT.cuQ[j]) * A[idx];
                    if (startup) acc += T(g * WT.cuR[j]) * B[idx];
                }
        if (FA.correction) uo[c] += T(2) * acc;
        else if (P.variant == HWV_CONS) uo[c] = T(2) * acc - uold[cell * Mu_tot + c];
        else uo[c] = acc;
    }
    if (FA.coef == nullptr || P.variant != HWV_CONS) return;

    // forcing (eq. (wavequ)): u_new += 2 sum_k sum_j tau^(2k+2)/(2j+2k+2)! [L^j f_2k],
    // the even time derivatives f_2k of f at the middle time, extent 2m+2 per dimension;
    // every lane adds to the outputs it wrote above
    const int PD = ipow(Pn, D);
    const double* fc = FA.coef + cell * (int64_t)FA.orders * PD;
    for (int r = 0; r < FA.orders; r += 2) {
        __syncthreads();
        for (int e = lane; e < PD; e += GW) bufA[e] = T(fc[(int64_t)r * PD + e]);
        __syncthreads();
        const double* w = FA.w + r * HW_MAXJ;
        for (int c = lane; c < Mu_tot; c += GW) {
            int a[3] = {0, 0, 0}, bmax[3] = {0, 0, 0};
            int rem = c;
            for (int i = 0; i < D; ++i) {
                a[i] = rem % M;
                rem /= M;
                bmax[i] = (Pn - 1 - a[i]) / 2;
            }
            T acc = T(0);
            for (int b2 = 0; b2 <= bmax[2]; ++b2)
                for (int b1 = 0; b1 <= bmax[1]; ++b1)
                    for (int b0 = 0; b0 <= bmax[0]; ++b0) {
                        double g = WT.f(0, a[0], b0);
                        if (D > 1) g *= WT.f(1, a[1], b1);
                        if (D > 2) g *= WT.f(2, a[2], b2);
                        const int idx = (a[0] + 2 * b0) + Pn * ((a[1] + 2 * b1) + Pn * (a[2] + 2 * b2));
                        acc += T(2.0 * g * w[b0 + b1 + b2]) * bufA[idx];
                    }
            uo[c] += acc;
        }
    }
}

template <typename T, int D>
__global__ void __launch_bounds__(GW)
k_half_step(const ProblemDesc* __restrict__ descs, const int64_t* __restrict__ prefix, int nprob,
            int64_t total, const T* __restrict__ ops, ForcingArgs FA)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* lops = reinterpret_cast<T*>(smem_raw);
    double* lw = reinterpret_cast<double*>(smem_raw + ((TAB_OPS * sizeof(T) + 15) / 16) * 16);
    T* sm = reinterpret_cast<T*>(smem_raw + tab_bytes<T>());
    const WTab WT{lw, lw + 3 * (HW_MAXM + 2) * (HW_MAXM + 2), lw + 3 * (HW_MAXM + 2) * (HW_MAXM + 2) + HW_MAXJ,
                  lw + 3 * (HW_MAXM + 2) * (HW_MAXM + 2) + 2 * HW_MAXJ,
                  lw + 3 * (HW_MAXM + 2) * (HW_MAXM + 2) + 3 * HW_MAXJ};
    const int lane = threadIdx.x;
    int cur = -1;
    for (int64_t g = blockIdx.x; g < total; g += gridDim.x) {
        int lo = 0, hi = nprob;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (prefix[mid] <= g) lo = mid;
            else hi = mid;
        }
        const ProblemDesc& P = descs[lo];
        if (lo != cur) {
            // stage the problem's operators and weights (the previous cell is finished:
            // the loop ends with a barrier)
            const T* src = ops + P.op.full;
            const int len = ops_len(P.m);
            for (int i = lane; i < len; i += GW) lops[i] = src[i];
            const double* F = &P.F[0][0][0];
            for (int i = lane; i < 3 * (HW_MAXM + 2) * (HW_MAXM + 2); i += GW) lw[i] = F[i];
            for (int i = lane; i < HW_MAXJ; i += GW) {
                const int o = 3 * (HW_MAXM + 2) * (HW_MAXM + 2);
                lw[o + i] = P.cuQ[i];
                lw[o + HW_MAXJ + i] = P.cuR[i];
                lw[o + 2 * HW_MAXJ + i] = P.cvQ[i];
                lw[o + 3 * HW_MAXJ + i] = P.cvR[i];
            }
            __syncthreads();
            cur = lo;
        }
        int64_t cell = g - prefix[lo];
        if (FA.cells) cell = FA.cells[cell];
        if (P.variant <= HWV_DISS_SIMPLE) diss_cell<T, D>(P, lops, WT, cell, sm, lane, FA);
        else cons_cell<T, D>(P, lops, WT, cell, sm, lane, FA);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// energy (conservative): per-cell <I f, I g>_{m+1} with the Gram block of the
// high coefficients; FP64 accumulation, per-workgroup partial sums.
// ---------------------------------------------------------------------------
template <typename T, int D>
__global__ void __launch_bounds__(GW)
k_energy(EnergyDesc E, const double* __restrict__ dops, double* __restrict__ partials)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* sm = reinterpret_cast<double*>(smem_raw);
    const int m = E.m, M = m + 1, K = 2 * M;
    const int KD = ipow(K, D), MD = ipow(M, D);
    double* Xf = sm;
    double* Xg = Xf + KD;
    double* bufA = Xg + KD;
    double* bufB = bufA + KD;
    double* Fh = bufB + KD;
    double* Gh = Fh + MD;
    double* GG = Gh + MD;
    double* red = GG + MD;
    const int lane = threadIdx.x;
    const double* hi = dops + E.hi_off;
    const double* gram = dops + E.gram_off;
    Geom P;
    P.to_grid = E.center_grid;
    for (int i = 0; i < 3; ++i) {
        P.bc[i] = E.bc[i];
        P.ext_from[i] = E.ext_from[i];
        P.ext_to[i] = E.ext_to[i];
    }
    double part = 0.0;
    for (int64_t cell = blockIdx.x; cell < E.n_cells; cell += gridDim.x) {
        Corners cr;
        find_corners<D>(P, cell, cr);
        const int ncoef = ipow(M, D);
        for (int e = lane; e < KD; e += GW) {
            int rem = e, node = 0, nstride = 1, coef = 0, cstride = 1;
            double sign = 1.0;
            for (int i = 0; i < D; ++i) {
                const int jd = rem % K;
                rem /= K;
                const int s = jd / M, l = jd % M;
                node += cr.node[i][s] * nstride;
                nstride *= P.ext_from[i];
                coef += l * cstride;
                cstride *= M;
                if (cr.ghost[i][s]) {
                    const bool odd = (l & 1);
                    if ((P.bc[i] == 1) ? !odd : odd) sign = -sign;
                }
            }
            Xf[e] = sign * (double)((const T*)E.f)[(int64_t)node * ncoef + coef];
            Xg[e] = sign * (double)((const T*)E.g)[(int64_t)node * ncoef + coef];
        }
        __syncthreads();
        const double* o3[3] = {hi, hi, hi};
        const int R3[3] = {M, M, M};
        tensor_apply<double, D>(Xf, K, o3, R3, bufA, bufB, Fh, 1.0, false, lane);
        tensor_apply<double, D>(Xg, K, o3, R3, bufA, bufB, Gh, 1.0, false, lane);
        const double* g3[3] = {gram, gram, gram};
        tensor_apply<double, D>(Gh, M, g3, R3, bufA, bufB, GG, 1.0, false, lane);
        double w = E.hfac;
        int64_t c = cell;
        for (int i = 0; i < D; ++i) {
            const int oi = (int)(c % E.ext_to[i]);
            c /= E.ext_to[i];
            if (E.bc[i] != 0 && E.center_grid == 0 && (oi == 0 || oi == E.ext_to[i] - 1)) w *= 0.5;
        }
        double s = 0.0;
        for (int e = lane; e < MD; e += GW) s += Fh[e] * GG[e];
        part += w * s;
        __syncthreads();
    }
    red[lane] = part;
    __syncthreads();
    if (lane == 0) {
        double t = 0.0;
        for (int i = 0; i < GW; ++i) t += red[i];
        partials[blockIdx.x] = t;
    }
}

// Sum of the per-workgroup energy partials of both passes in one fixed order (lane k
// adds partials k, k + 64, ...; then lane 0 adds the 64 lane sums in order), written as
// E = 2 (sum of pass 0 - sum of pass 1) to one device word.
__global__ void __launch_bounds__(GW)
k_energy_finish(const double* __restrict__ partials, int n0, int stride1, int n1, double* __restrict__ e_out)
{
    __shared__ double red[2][GW];
    const int lane = threadIdx.x;
    double s0 = 0.0, s1 = 0.0;
    for (int i = lane; i < n0; i += GW) s0 += partials[i];
    for (int i = lane; i < n1; i += GW) s1 += partials[stride1 + i];
    red[0][lane] = s0;
    red[1][lane] = s1;
    __syncthreads();
    if (lane == 0) {
        double t0 = 0.0, t1 = 0.0;
        for (int i = 0; i < GW; ++i) {
            t0 += red[0][i];
            t1 += red[1][i];
        }
        e_out[0] = 2.0 * (t0 - t1);
    }
}

// Partial sums of the allocation-free energy call: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never passes its name to a kernel:
// the name is a host-side stand-in; the device address comes from hipGetSymbolAddress
// (once per device, below).
static __device__ __align__(256) double scratch[2 * HW_ENERGY_MAX_GROUPS];

template <typename Tin, typename Tout>
__global__ void k_convert(const Tin* __restrict__ src, Tout* __restrict__ dst, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (Tout)src[i];
}

} // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t hw_generic_lds_bytes(int d, int m, int variant, int elem_size)
{
    const int Pn = 2 * m + 2, K = Pn, Kv = 2 * m, M = m + 1;
    auto pw = [](int b, int e) {
        size_t r = 1;
        for (int i = 0; i < e; ++i) r *= (size_t)b;
        return r;
    };
    size_t n;
    if (variant <= HWV_DISS_SIMPLE) {
        const bool simple = (variant == HWV_DISS_SIMPLE) || d == 1;
        const int E = simple ? Pn : 2 * m;
        n = 3 * pw(K, d) + pw(Kv, d) + 2 * pw(E, d) + (simple ? pw(Pn, d) : pw(M, d));
    } else {
        n = 6 * pw(K, d);
    }
    return n * (size_t)elem_size + (elem_size == 8 ? tab_bytes<double>() : tab_bytes<float>());
}

size_t hw_energy_lds_bytes(int d, int m)
{
    const int M = m + 1, K = 2 * M;
    size_t kd = 1, md = 1;
    for (int i = 0; i < d; ++i) {
        kd *= K;
        md *= M;
    }
    return (4 * kd + 3 * md + GW) * sizeof(double);
}

template <typename T, int D>
static hipError_t launch_hs(const ProblemDesc* descs, const int64_t* prefix, int nprob, int64_t total,
                            const void* ops, size_t lds, int grid, hipStream_t st, ForcingArgs fa)
{
    auto kern = k_half_step<T, D>;
    if (lds > 64 * 1024) {
        hipError_t e = hw_lds_limit<k_half_step<T, D>>(lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(GW), lds, st, descs, prefix, nprob, total,
                       (const T*)ops, fa);
    return hipGetLastError();
}

hipError_t hw_launch_generic(int d, bool fp64, const ProblemDesc* descs, const int64_t* prefix,
                             int nprob, int64_t total, const void* ops, size_t lds, int grid,
                             hipStream_t st, const ForcingArgs* forcing)
{
    ForcingArgs fa;
    if (forcing) fa = *forcing;
    if (fp64) {
        if (d == 1) return launch_hs<double, 1>(descs, prefix, nprob, total, ops, lds, grid, st, fa);
        if (d == 2) return launch_hs<double, 2>(descs, prefix, nprob, total, ops, lds, grid, st, fa);
        return launch_hs<double, 3>(descs, prefix, nprob, total, ops, lds, grid, st, fa);
    }
    if (d == 1) return launch_hs<float, 1>(descs, prefix, nprob, total, ops, lds, grid, st, fa);
    if (d == 2) return launch_hs<float, 2>(descs, prefix, nprob, total, ops, lds, grid, st, fa);
    return launch_hs<float, 3>(descs, prefix, nprob, total, ops, lds, grid, st, fa);
}

template <typename T, int D>
static hipError_t launch_en(const EnergyDesc& E, const double* dops, double* partials, int grid,
                            hipStream_t st)
{
    const size_t lds = hw_energy_lds_bytes(D, E.m);
    auto kern = k_energy<T, D>;
    if (lds > 64 * 1024) {
        hipError_t e = hw_lds_limit<k_energy<T, D>>(lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(GW), lds, st, E, dops, partials);
    return hipGetLastError();
}

hipError_t hw_launch_energy(int d, bool fp64, const EnergyDesc& E, const double* dops,
                            double* partials, int grid, hipStream_t st)
{
    if (fp64) {
        if (d == 1) return launch_en<double, 1>(E, dops, partials, grid, st);
        if (d == 2) return launch_en<double, 2>(E, dops, partials, grid, st);
        return launch_en<double, 3>(E, dops, partials, grid, st);
    }
    if (d == 1) return launch_en<float, 1>(E, dops, partials, grid, st);
    if (d == 2) return launch_en<float, 2>(E, dops, partials, grid, st);
    return launch_en<float, 3>(E, dops, partials, grid, st);
}

// Device address of `scratch` on the current device, looked up once per device.
static hipError_t scratch_address(double** out)
{
    static std::mutex mu;
    static double* addr[HW_MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= HW_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double*>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t hw_launch_energy_noalloc(int d, bool fp64, const EnergyDesc& E0, int grid0, const EnergyDesc& E1,
                                    int grid1, const double* dops, double* e_out, hipStream_t st)
{
    if (grid0 < 1 || grid1 < 1 || grid0 > HW_ENERGY_MAX_GROUPS || grid1 > HW_ENERGY_MAX_GROUPS)
        return hipErrorInvalidValue;
    double* part = nullptr;
    hipError_t e = scratch_address(&part);
    if (e != hipSuccess) return e;
    e = hw_launch_energy(d, fp64, E0, dops, part, grid0, st);
    if (e != hipSuccess) return e;
    e = hw_launch_energy(d, fp64, E1, dops, part + HW_ENERGY_MAX_GROUPS, grid1, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(GW), 0, st, part, grid0, HW_ENERGY_MAX_GROUPS, grid1, e_out);
    return hipGetLastError();
}

hipError_t hw_launch_convert(const void* src, bool src64, void* dst, bool dst64, int64_t n,
                             hipStream_t st)
{
    const int block = 256;
    int64_t g = (n + block - 1) / block;
    const int grid = (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
    if (src64 && dst64)
        hipLaunchKernelGGL((k_convert<double, double>), dim3(grid), dim3(block), 0, st,
                           (const double*)src, (double*)dst, n);
    else if (src64)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(grid), dim3(block), 0, st,
                           (const double*)src, (float*)dst, n);
    else if (dst64)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(grid), dim3(block), 0, st,
                           (const float*)src, (double*)dst, n);
    else
        hipLaunchKernelGGL((k_convert<float, float>), dim3(grid), dim3(block), 0, st,
                           (const float*)src, (float*)dst, n);
    return hipGetLastError();
}
