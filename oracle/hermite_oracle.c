/*
 * Plain FP64 CPU oracle for the Hermite methods for the scalar wave equation
 * (Appelo, Hagstrom & Vargas, "Hermite Methods for the Scalar Wave Equation").
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load this library.  It shares no code, header, table or helper
 * with the GPU library: the Hermite matrices are obtained here by their own
 * elimination, the time stepping follows the paper's stage recursion (dissipative
 * method) and its repeated-Laplacian Taylor sum (conservative method), whereas the
 * GPU path uses precomputed closed-form weights.
 *
 * Every routine is deliberately plain: dimension-by-dimension application of the
 * 1-D Hermite operators (the tensor product of Sec. 2.2), the recursion of
 * Sec. 3.1.2 / Sec. 3.3 stage by stage, evaluation at the half step, one output node
 * at a time.  OpenMP only distributes output nodes over threads.
 *
 * Conventions (shared with the GPU library only as an interface, not as code):
 *   node index  = i0 + n0*(i1 + n1*i2)                 (x fastest)
 *   coefficient = l0 + M*(l1 + M*l2), M = m+1 for u, m for v (x fastest)
 *   value       = h^l / l! d^l f (scaled Taylor coefficient, Sec. 2.2)
 *   periodic:   n_i nodes per dimension on both grids
 *   otherwise:  primal n_i + 1 nodes (i = 0..n_i), dual n_i nodes (i + 1/2)
 *
 * Parity is pinned by the CPU tests: exact evolution of polynomial data, the
 * d'Alembert closed forms at c dt = h, convergence rates against exact plane waves,
 * bounded long runs at c dt = h and conservation of the discrete energy.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "hermite_oracle.h"

#define MAXD 3
#define MAXM 8
#define MAXP (2 * MAXM + 2)

/* ------------------------------------------------------------------------- */
/* 1-D Hermite operator, Sec. 2.2 eqs. (Hermn),(Hermcon).                      */
/* In the scaled variable z = (x - x_c)/h the cell is [-1/2, 1/2].  The         */
/* interpolant sum_k a_k z^k must reproduce h^l/l! d^l at both ends for         */
/* l = 0..m, i.e.  sum_k binom(k,l) z_s^(k-l) a_k = data_{s,l},  z_s = s - 1/2.  */
/* The matrix of that linear system is inverted by Gauss-Jordan elimination     */
/* with partial pivoting in long double.                                       */
/* ------------------------------------------------------------------------- */
static double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

int hwo_hermite_matrix(int m, double *H)
{
    if (m < 0 || m > MAXM || !H) return -1;
    const int M = m + 1, P = 2 * m + 2;
    long double A[MAXP][2 * MAXP];
    /* row r = s*M + l (condition), column k (monomial); augmented with identity */
    for (int s = 0; s < 2; ++s)
        for (int l = 0; l < M; ++l) {
            const int r = s * M + l;
            const long double z = (long double)s - 0.5L;
            for (int k = 0; k < P; ++k) {
                long double v = 0.0L;
                if (k >= l) {
                    v = (long double)binom(k, l);
                    for (int e = 0; e < k - l; ++e) v *= z;
                }
                A[r][k] = v;
            }
            for (int k = 0; k < P; ++k) A[r][P + k] = (r == k) ? 1.0L : 0.0L;
        }
    for (int col = 0; col < P; ++col) {
        int piv = col;
        for (int r = col + 1; r < P; ++r)
            if (fabsl(A[r][col]) > fabsl(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0L) return -2;
        if (piv != col)
            for (int k = 0; k < 2 * P; ++k) {
                long double t = A[col][k];
                A[col][k] = A[piv][k];
                A[piv][k] = t;
            }
        const long double inv = 1.0L / A[col][col];
        for (int k = 0; k < 2 * P; ++k) A[col][k] *= inv;
        for (int r = 0; r < P; ++r) {
            if (r == col || A[r][col] == 0.0L) continue;
            const long double f = A[r][col];
            for (int k = 0; k < 2 * P; ++k) A[r][k] -= f * A[col][k];
        }
    }
    /* A^{-1} maps conditions to monomial coefficients: H[k][s*M+l] */
    for (int k = 0; k < P; ++k)
        for (int j = 0; j < P; ++j) H[k * P + j] = (double)A[k][P + j];
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Problem geometry (Sec. 2.1).                                                */
/* ------------------------------------------------------------------------- */
static int pw(int b, int e)
{
    int r = 1;
    while (e-- > 0) r *= b;
    return r;
}

static int64_t grid_extent(const hwo_problem *p, int grid, int dim)
{
    if (p->bc[dim] == HWO_PERIODIC) return p->n[dim];
    return grid == HWO_PRIMAL ? (int64_t)p->n[dim] + 1 : (int64_t)p->n[dim];
}

int64_t hwo_nodes(const hwo_problem *p, int grid)
{
    int64_t c = 1;
    for (int i = 0; i < p->d; ++i) c *= grid_extent(p, grid, i);
    return c;
}

static double hdim(const hwo_problem *p, int i) { return (p->xr[i] - p->xl[i]) / p->n[i]; }

/* Corner lookup for one output node.  For the half step to the dual grid the   */
/* output node i+1/2 is the centre of primal cell [i, i+1]; for the half step    */
/* to the primal grid the output node i is the centre of dual cell               */
/* [i-1/2, i+1/2].  Outside a non-periodic wall the corner is a ghost: the       */
/* mirror image of the adjacent interior dual node, with coefficient l in the    */
/* normal direction multiplied by (-1)^(l+1) (Dirichlet, odd extension) or       */
/* (-1)^l (Neumann, even extension), Sec. 3.1.3.                                 */
typedef struct {
    int64_t node[1 << MAXD];       /* input node of corner sigma                */
    int ghost[1 << MAXD][MAXD];    /* 1 if corner sigma is a ghost in that dim  */
    int side[1 << MAXD][MAXD];     /* ghost side: -1 beyond the low wall, +1 beyond */
                                   /* the high wall, 0 inside                     */
    int64_t idx[1 << MAXD][MAXD];  /* input node index per dim (mirrored)        */
} corners_t;

static void find_corners(const hwo_problem *p, int to_grid, const int64_t out_idx[MAXD],
                         corners_t *cr)
{
    const int d = p->d;
    const int from_grid = 1 - to_grid;
    for (int sig = 0; sig < (1 << d); ++sig) {
        int64_t node = 0, stride = 1;
        for (int i = 0; i < d; ++i) {
            const int s = (sig >> i) & 1;
            const int64_t ext = grid_extent(p, from_grid, i);
            int64_t j;
            int gh = 0, side = 0;
            if (to_grid == HWO_DUAL) {
                j = out_idx[i] + s; /* primal i (s=0) and i+1 (s=1) */
                if (p->bc[i] == HWO_PERIODIC) j %= ext;
            } else {
                j = out_idx[i] - 1 + s; /* dual i-1/2 (s=0) and i+1/2 (s=1) */
                if (p->bc[i] == HWO_PERIODIC) {
                    j = (j + ext) % ext;
                } else if (j < 0) {
                    j = 0; /* ghost at -1/2 mirrors dual node 1/2 */
                    gh = 1;
                    side = -1;
                } else if (j >= ext) {
                    j = ext - 1; /* ghost at n+1/2 mirrors dual node n-1/2 */
                    gh = 1;
                    side = 1;
                }
            }
            cr->ghost[sig][i] = gh;
            cr->side[sig][i] = side;
            cr->idx[sig][i] = j;
            node += j * stride;
            stride *= ext;
        }
        cr->node[sig] = node;
    }
}

static double ghost_sign(const hwo_problem *p, const corners_t *cr, int sig, const int *l)
{
    double s = 1.0;
    for (int i = 0; i < p->d; ++i) {
        if (!cr->ghost[sig][i]) continue;
        const int odd = (l[i] & 1);
        if (p->bc[i] == HWO_DIRICHLET) s *= odd ? 1.0 : -1.0; /* (-1)^(l+1) */
        else s *= odd ? -1.0 : 1.0;                            /* (-1)^l     */
    }
    return s;
}

/* ------------------------------------------------------------------------- */
/* Inhomogeneous and time-dependent wall data (Sec. 3.1.3).  The ghost           */
/* polynomial is fixed by requiring the interpolant centred at the wall node to  */
/* match the interior data on one side and the boundary condition on the wall:   */
/* its even normal part (Dirichlet: u = g and, through the PDE, its even normal  */
/* derivatives) or odd normal part (Neumann) is prescribed, the rest comes from  */
/* the interior.  With W that prescribed part (even / odd in the normal          */
/* variable), the interpolant is p = R(q) + W where q is the interior polynomial */
/* and R its homogeneous odd / even reflection; matching p at the interior       */
/* corner gives the ghost data                                                   */
/*     ghost = R(interior) + 2 W(ghost position),                                */
/* which is the homogeneous mirror of Sec. 3.1.3 when W = 0.  At a corner ghost   */
/* in several dimensions the walls are applied one dimension after another in    */
/* increasing order, each to the result of the previous one.                     */
/*                                                                               */
/* Wall records (one per wall point, Mrec^d values with Mrec = m+1 for u and m   */
/* for v, coefficient index x fastest): in the normal dimension the index j      */
/* stands for the normal degree k = 2j (Dirichlet) or 2j+1 (Neumann); each entry */
/* is the scaled Taylor coefficient h^k/k! d^k_normal h^l/l! d^l_tangential of   */
/* the solution at the wall point, at the time of the half step's input data.    */
/* Faces: for every non-periodic dimension i in increasing order, the low wall   */
/* then the high wall.  Wall points of face i: the input (dual) grid's node       */
/* positions in every other dimension t, extended by one ghost position at each  */
/* end when t is non-periodic (index 0 = -1/2 beyond the low wall, n_t+1 = beyond */
/* the high wall; periodic t: the n_t dual nodes), x fastest.                    */
/* ------------------------------------------------------------------------- */
typedef struct {
    const double *data; /* all faces' records, or NULL (homogeneous walls) */
    int Mrec;           /* coefficients per dimension of a record          */
} walls_t;

static int64_t face_points(const hwo_problem *p, int i)
{
    int64_t n = 1;
    for (int t = 0; t < p->d; ++t) {
        if (t == i) continue;
        n *= (p->bc[t] == HWO_PERIODIC) ? p->n[t] : p->n[t] + 2;
    }
    return n;
}

static double refl_sign(int bc, int l)
{
    const int odd = l & 1;
    if (bc == HWO_DIRICHLET) return odd ? 1.0 : -1.0; /* (-1)^(l+1) */
    return odd ? -1.0 : 1.0;                           /* (-1)^l     */
}

static double wall_term(const hwo_problem *p, const corners_t *cr, int sig, const int *l,
                        const walls_t *w)
{
    const int d = p->d;
    const int rec = pw(w->Mrec, d);
    double total = 0.0;
    for (int r = 0; r < d; ++r) {
        if (!cr->side[sig][r]) continue;
        /* reflections of the dimensions applied after r */
        double sgn = 1.0;
        for (int g = r + 1; g < d; ++g)
            if (cr->side[sig][g]) sgn *= refl_sign(p->bc[g], l[g]);
        /* face offset: faces of earlier non-periodic dimensions, then this side */
        int64_t off = 0;
        for (int i = 0; i < r; ++i)
            if (p->bc[i] != HWO_PERIODIC) off += 2 * face_points(p, i);
        if (cr->side[sig][r] > 0) off += face_points(p, r);
        /* wall point: dims before r already reflected (ghost position if ghost), */
        /* dims after r still at the mirrored interior node                       */
        int64_t pt = 0, stride = 1;
        for (int t = 0; t < d; ++t) {
            if (t == r) continue;
            int64_t pos, ext;
            if (p->bc[t] == HWO_PERIODIC) {
                ext = p->n[t];
                pos = cr->idx[sig][t];
            } else {
                ext = p->n[t] + 2;
                if (t < r && cr->side[sig][t] < 0) pos = 0;
                else if (t < r && cr->side[sig][t] > 0) pos = p->n[t] + 1;
                else pos = cr->idx[sig][t] + 1;
            }
            pt += pos * stride;
            stride *= ext;
        }
        const double *rw = w->data + (off + pt) * (int64_t)rec;
        /* W at the ghost position, a distance h/2 beyond the wall: Taylor shift of */
        /* the normal expansion by delta = -1/2 (low) or +1/2 (high)                */
        const double delta = cr->side[sig][r] < 0 ? -0.5 : 0.5;
        double sum = 0.0;
        for (int j = 0; j < w->Mrec; ++j) {
            const int k = (p->bc[r] == HWO_DIRICHLET) ? 2 * j : 2 * j + 1;
            if (k < l[r]) continue;
            int c = 0, cs = 1;
            for (int t = 0; t < d; ++t) {
                c += (t == r ? j : l[t]) * cs;
                cs *= w->Mrec;
            }
            sum += binom(k, l[r]) * pow(delta, k - l[r]) * rw[c];
        }
        total += sgn * 2.0 * sum;
    }
    return total;
}

/* ------------------------------------------------------------------------- */
/* Tensor-product interpolant I_{md_1..md_d} (Sec. 2.2, eqs. (Hermn2),        */
/* (Hermcon2) and their mixed-degree variants).  corner data: coefficient       */
/* arrays with M_data entries per dimension; only l_i <= md_i is used.          */
/* Result a[k], k_i = 0..2 md_i + 1, flattened x fastest.                      */
/* The input is arranged with per-dimension index j_i = s_i (md_i+1) + l_i and  */
/* the 1-D operator H_{md_i} is applied along each dimension in turn.           */
/* ------------------------------------------------------------------------- */
typedef struct {
    double H[MAXM + 1][MAXP * MAXP]; /* H_q for q = 0..m */
} tables_t;

static void load_tables(int m, tables_t *t)
{
    for (int q = 0; q <= m; ++q) hwo_hermite_matrix(q, t->H[q]);
}

static void tensor_interp(const hwo_problem *p, const tables_t *tb, const corners_t *cr,
                          const double *data, int M_data, const int md[MAXD], const walls_t *w,
                          double *a, double *work)
{
    const int d = p->d;
    int ext[MAXD] = {1, 1, 1};
    int total = 1;
    for (int i = 0; i < d; ++i) {
        ext[i] = 2 * md[i] + 2;
        total *= ext[i];
    }
    /* gather: a[j] with j_i = s_i*(md_i+1) + l_i */
    for (int idx = 0; idx < total; ++idx) {
        int rem = idx, sig = 0, l[MAXD] = {0, 0, 0}, coef = 0, cstride = 1;
        for (int i = 0; i < d; ++i) {
            const int j = rem % ext[i];
            rem /= ext[i];
            const int s = j / (md[i] + 1);
            l[i] = j % (md[i] + 1);
            sig |= s << i;
            coef += l[i] * cstride;
            cstride *= M_data;
        }
        a[idx] = ghost_sign(p, cr, sig, l) * data[cr->node[sig] * (int64_t)pw(M_data, d) + coef];
        if (w && w->data) {
            int any = 0;
            for (int i = 0; i < d; ++i) any |= cr->side[sig][i];
            if (any) a[idx] += wall_term(p, cr, sig, l, w);
        }
    }
    /* dimension-by-dimension application of H_{md_i} */
    int stride = 1;
    for (int i = 0; i < d; ++i) {
        const int P = ext[i];
        const double *H = tb->H[md[i]];
        for (int idx = 0; idx < total; ++idx) {
            const int k = (idx / stride) % P;
            const int base = idx - k * stride;
            double acc = 0.0;
            for (int j = 0; j < P; ++j) acc += H[k * P + j] * a[base + j * stride];
            work[idx] = acc;
        }
        memcpy(a, work, sizeof(double) * total);
        stride *= P;
    }
}

/* embed an array with extents ext[] into a zero-padded array with extent P in   */
/* every dimension                                                               */
static void embed(int d, const int ext[MAXD], const double *src, int P, double *dst)
{
    const int Ptot = pw(P, d);
    memset(dst, 0, sizeof(double) * Ptot);
    int total = 1;
    for (int i = 0; i < d; ++i) total *= ext[i];
    for (int idx = 0; idx < total; ++idx) {
        int rem = idx, off = 0, st = 1;
        for (int i = 0; i < d; ++i) {
            off += (rem % ext[i]) * st;
            rem /= ext[i];
            st *= P;
        }
        dst[off] = src[idx];
    }
}

/* scaled second derivative along dim i summed over dims (the Laplacian acting on  */
/* scaled Taylor coefficients): (d^2/dx_i^2 f)_k = (k_i+2)(k_i+1)/h_i^2 f_{k+2e_i} */
static void scaled_laplacian(const hwo_problem *p, int P, const double *f, double *out)
{
    const int d = p->d;
    const int total = pw(P, d);
    for (int idx = 0; idx < total; ++idx) {
        double acc = 0.0;
        int stride = 1;
        for (int i = 0; i < d; ++i) {
            const int k = (idx / stride) % P;
            if (k + 2 < P) {
                const double h = hdim(p, i);
                acc += (double)(k + 2) * (double)(k + 1) / (h * h) * f[idx + 2 * stride];
            }
            stride *= P;
        }
        out[idx] = acc;
    }
}

/* ------------------------------------------------------------------------- */
/* Dissipative half step for one output node (Sec. 3.1.2 in 1-D; Sec. 3.3 with  */
/* the modified first step for d >= 2, or the straightforward extension).       */
/* ------------------------------------------------------------------------- */
typedef struct {
    double *p0, *q0, *ci, *U, *V, *Un, *Vn, *work, *tmp, *uacc, *vacc;
} scratch_t;

static void scratch_alloc(scratch_t *s, int d, int m)
{
    const int P = 2 * m + 2;
    const int T = pw(P, d);
    double *b = (double *)calloc((size_t)T * 11, sizeof(double));
    s->p0 = b;
    s->q0 = b + T;
    s->ci = b + 2 * T;
    s->U = b + 3 * T;
    s->V = b + 4 * T;
    s->Un = b + 5 * T;
    s->Vn = b + 6 * T;
    s->work = b + 7 * T;
    s->tmp = b + 8 * T;
    s->uacc = b + 9 * T;
    s->vacc = b + 10 * T;
}

/* fcell: forcing of this cell, n_orders blocks of (2m)^d scaled space-time Taylor       */
/* coefficients phi[r][k] = h^k/k! d^k/dx^k d^r/dt^r f at the cell centre and the start  */
/* of the half step (or NULL).  Stage s receives dt^s/s! phi[s-1] in V_s, eq.            */
/* (recursion_diss_1d_2) of Sec. 3.1.2 applied in every dimension.                        */
static void diss_cell(const hwo_problem *p, const tables_t *tb, const corners_t *cr,
                      const double *u_in, const double *v_in, const double *fcell, int n_orders,
                      const walls_t *wu, const walls_t *wv, double *u_out, double *v_out,
                      scratch_t *s)
{
    const int d = p->d, m = p->m, M = m + 1, Mv = m, P = 2 * m + 2;
    const int T = pw(P, d);
    const double dt = p->dt, c2 = p->c * p->c;
    int md[MAXD], ext[MAXD];

    /* U_0 = I_{m..m} u (degree 2m+1 per dimension) */
    for (int i = 0; i < d; ++i) md[i] = m;
    tensor_interp(p, tb, cr, u_in, M, md, wu, s->tmp, s->work);
    memcpy(s->p0, s->tmp, sizeof(double) * T);
    /* V_0 = I_{m-1..m-1} v (degree 2m-1 per dimension), zero padded */
    for (int i = 0; i < d; ++i) {
        md[i] = m - 1;
        ext[i] = 2 * m;
    }
    tensor_interp(p, tb, cr, v_in, Mv, md, wv, s->tmp, s->work);
    embed(d, ext, s->tmp, P, s->q0);

    memcpy(s->U, s->p0, sizeof(double) * T);
    memcpy(s->V, s->q0, sizeof(double) * T);

    /* accumulate the Taylor series evaluated at t = t0 + dt/2, i.e. weight 2^-s */
    double *uacc = s->uacc, *vacc = s->vacc;
    for (int k = 0; k < T; ++k) {
        uacc[k] = s->U[k];
        vacc[k] = s->V[k];
    }

    const int modified = (p->method == HWO_DISS_FULL && d >= 2);
    const int nf = fcell ? n_orders : 0;
    const int s_limit = p->taylor_stages > 0 ? p->taylor_stages : d * (2 * m + 2) + 2 + nf;
    const int Fv = pw(2 * m, d);
    double wgt = 1.0, fac = 1.0;
    for (int st = 1; st <= s_limit; ++st) {
        wgt *= 0.5;
        fac *= dt / st; /* dt^s / s! */
        /* U_s = dt/s V_{s-1} */
        for (int k = 0; k < T; ++k) s->Un[k] = dt / st * s->V[k];
        if (st == 1 && modified) {
            /* V_1 = c^2 dt sum_i (k_i+2)(k_i+1)/h_i^2 c^(i)_{k+2e_i}, where c^(i) is the */
            /* interpolant of degree m data in dimension i and m-1 in the others.       */
            memset(s->Vn, 0, sizeof(double) * T);
            for (int i = 0; i < d; ++i) {
                for (int j = 0; j < d; ++j) {
                    md[j] = (j == i) ? m : m - 1;
                    ext[j] = 2 * md[j] + 2;
                }
                tensor_interp(p, tb, cr, u_in, M, md, wu, s->tmp, s->work);
                embed(d, ext, s->tmp, P, s->ci);
                const double h = hdim(p, i);
                int stride = 1;
                for (int j = 0; j < i; ++j) stride *= P;
                for (int idx = 0; idx < T; ++idx) {
                    const int k = (idx / stride) % P;
                    if (k + 2 < P)
                        s->Vn[idx] += c2 * dt * (double)(k + 2) * (double)(k + 1) / (h * h) *
                                      s->ci[idx + 2 * stride];
                }
            }
            /* the modified first step is defined for indices 0..2m-1 only */
            for (int idx = 0; idx < T; ++idx) {
                int rem = idx, keep = 1;
                for (int j = 0; j < d; ++j) {
                    if (rem % P > 2 * m - 1) keep = 0;
                    rem /= P;
                }
                if (!keep) s->Vn[idx] = 0.0, s->Un[idx] = 0.0;
            }
        } else {
            /* V_s = c^2 dt/s Laplacian(U_{s-1}) */
            scaled_laplacian(p, P, s->U, s->tmp);
            for (int k = 0; k < T; ++k) s->Vn[k] = c2 * dt / st * s->tmp[k];
        }
        if (st - 1 < nf) {
            /* forcing: V_s += dt^s/s! phi[s-1], phi embedded from extent 2m into P */
            const double *ph = fcell + (int64_t)(st - 1) * Fv;
            for (int q = 0; q < Fv; ++q) {
                int rem = q, off = 0, stp = 1;
                for (int i = 0; i < d; ++i) {
                    off += (rem % (2 * m)) * stp;
                    rem /= 2 * m;
                    stp *= P;
                }
                s->Vn[off] += fac * ph[q];
            }
        }
        int nonzero = 0;
        for (int k = 0; k < T; ++k) {
            s->U[k] = s->Un[k];
            s->V[k] = s->Vn[k];
            uacc[k] += wgt * s->U[k];
            vacc[k] += wgt * s->V[k];
            nonzero |= (s->U[k] != 0.0) | (s->V[k] != 0.0);
        }
        if (!nonzero && p->taylor_stages <= 0 && st >= nf) break; /* the series has terminated */
    }

    /* evaluation at the cell centre: coefficients l <= m (u), l <= m-1 (v) */
    const int Mu_tot = pw(M, d), Mv_tot = pw(Mv, d);
    for (int c = 0; c < Mu_tot; ++c) {
        int rem = c, off = 0, st = 1;
        for (int i = 0; i < d; ++i) {
            off += (rem % M) * st;
            rem /= M;
            st *= P;
        }
        u_out[c] = uacc[off];
    }
    for (int c = 0; c < Mv_tot; ++c) {
        int rem = c, off = 0, st = 1;
        for (int i = 0; i < d; ++i) {
            off += (rem % Mv) * st;
            rem /= Mv;
            st *= P;
        }
        v_out[c] = vacc[off];
    }
}

static void out_index(const hwo_problem *p, int grid, int64_t node, int64_t idx[MAXD])
{
    for (int i = 0; i < MAXD; ++i) idx[i] = 0;
    for (int i = 0; i < p->d; ++i) {
        const int64_t e = grid_extent(p, grid, i);
        idx[i] = node % e;
        node /= e;
    }
}

static int check_problem(const hwo_problem *p)
{
    if (!p || p->d < 1 || p->d > MAXD || p->m < 0 || p->m > MAXM) return -1;
    for (int i = 0; i < p->d; ++i) {
        if (p->n[i] < 1 || !(p->xr[i] > p->xl[i])) return -1;
        if (p->bc[i] < HWO_PERIODIC || p->bc[i] > HWO_NEUMANN) return -1;
    }
    return 0;
}

static int nthreads_or_default(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

int hwo_diss_half(const hwo_problem *p, int to_grid, const double *u_in, const double *v_in,
                  double *u_out, double *v_out, const int64_t *sel, int64_t nsel, int nthreads)
{
    return hwo_diss_half_ext(p, to_grid, u_in, v_in, NULL, 0, NULL, NULL, u_out, v_out, sel, nsel,
                             nthreads);
}

int hwo_diss_half_forced(const hwo_problem *p, int to_grid, const double *u_in, const double *v_in,
                         const double *f_coef, int n_orders, double *u_out, double *v_out,
                         const int64_t *sel, int64_t nsel, int nthreads)
{
    return hwo_diss_half_ext(p, to_grid, u_in, v_in, f_coef, n_orders, NULL, NULL, u_out, v_out, sel,
                             nsel, nthreads);
}

int hwo_diss_half_ext(const hwo_problem *p, int to_grid, const double *u_in, const double *v_in,
                      const double *f_coef, int n_orders, const double *wall_u, const double *wall_v,
                      double *u_out, double *v_out, const int64_t *sel, int64_t nsel, int nthreads)
{
    if (n_orders < 0 || (n_orders > 0 && !f_coef)) return -1;
    if ((wall_u == NULL) != (wall_v == NULL)) return -1;
    if (check_problem(p) || p->m < 1 || (p->method != HWO_DISS_FULL && p->method != HWO_DISS_SIMPLE))
        return -1;
    const int d = p->d, M = p->m + 1, Mv = p->m;
    const int Mu_tot = pw(M, d), Mv_tot = pw(Mv, d);
    const int64_t count = sel ? nsel : hwo_nodes(p, to_grid);
    tables_t *tb = (tables_t *)malloc(sizeof(tables_t));
    load_tables(p->m, tb);
    const int nt = nthreads_or_default(nthreads);
#pragma omp parallel num_threads(nt)
    {
        scratch_t s;
        scratch_alloc(&s, d, p->m);
#pragma omp for schedule(static)
        for (int64_t q = 0; q < count; ++q) {
            const int64_t node = sel ? sel[q] : q;
            int64_t idx[MAXD];
            corners_t cr;
            out_index(p, to_grid, node, idx);
            find_corners(p, to_grid, idx, &cr);
            const double *fcell =
                n_orders > 0 ? f_coef + node * (int64_t)n_orders * pw(2 * p->m, d) : NULL;
            const walls_t wu = {to_grid == HWO_PRIMAL ? wall_u : NULL, M};
            const walls_t wv = {to_grid == HWO_PRIMAL ? wall_v : NULL, Mv};
            diss_cell(p, tb, &cr, u_in, v_in, fcell, n_orders, &wu, &wv, u_out + q * Mu_tot,
                      v_out + q * Mv_tot, &s);
        }
        free(s.p0);
    }
    free(tb);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Conservative method (Sec. 4.1 eq. (convUpdate), Sec. 4.3): the even Taylor    */
/* sum of eq. (update), 2 sum_l (c dt/2)^(2l)/(2l)! Laplacian^l of the cell       */
/* interpolant at the cell centre, minus the old value at the same node.         */
/* ------------------------------------------------------------------------- */
static void cons_even_odd_sum(const hwo_problem *p, const double *a, double tau, int odd,
                              double *acc, double *cur, double *tmp)
{
    /* acc = sum_l tau^(2l+odd)/(2l+odd)! (c^2 Laplacian)^l a */
    const int d = p->d, P = 2 * p->m + 2, T = pw(P, d);
    const double c2 = p->c * p->c;
    double coef = odd ? tau : 1.0;
    memcpy(cur, a, sizeof(double) * T);
    for (int k = 0; k < T; ++k) acc[k] = coef * cur[k];
    for (int l = 1; l <= d * (P / 2) + 1; ++l) {
        scaled_laplacian(p, P, cur, tmp);
        int nonzero = 0;
        for (int k = 0; k < T; ++k) {
            cur[k] = c2 * tmp[k];
            nonzero |= cur[k] != 0.0;
        }
        if (!nonzero) break;
        const int e = 2 * l + odd;
        coef = coef * tau * tau / ((double)e * (double)(e - 1));
        for (int k = 0; k < T; ++k) acc[k] += coef * cur[k];
    }
}

/* With a forcing term (u_tt = c^2 Lap u + f, eq. (wavequ)) the even time derivatives */
/* in eq. (update) obey d^2r u/dt^2r = c^2 Lap d^(2r-2) u/dt^(2r-2) + d^(2r-2) f/dt^(2r-2), */
/* so D_0 = a, D_r = c^2 Lap D_(r-1) + phi_(2r-2) and the sum is                       */
/* sum_r (dt/2)^(2r)/(2r)! D_r.  phi_q: the q-th time derivative of f at the cell      */
/* centre and the middle time, (2m+2)^d scaled Taylor coefficients.                    */
static void cons_forced_sum(const hwo_problem *p, const double *a, double tau, const double *fcell,
                            int n_orders, double *acc, double *cur, double *tmp)
{
    const int d = p->d, P = 2 * p->m + 2, T = pw(P, d);
    const double c2 = p->c * p->c;
    memcpy(cur, a, sizeof(double) * T);
    memcpy(acc, a, sizeof(double) * T);
    double coef = 1.0;
    for (int r = 1; r <= d * (P / 2) + 1 + n_orders; ++r) {
        scaled_laplacian(p, P, cur, tmp);
        int nonzero = 0;
        for (int k = 0; k < T; ++k) cur[k] = c2 * tmp[k];
        const int q = 2 * r - 2;
        if (q < n_orders)
            for (int k = 0; k < T; ++k) cur[k] += fcell[(int64_t)q * T + k];
        for (int k = 0; k < T; ++k) nonzero |= cur[k] != 0.0;
        if (!nonzero && q + 2 >= n_orders) break;
        coef = coef * tau * tau / ((double)(2 * r) * (double)(2 * r - 1));
        for (int k = 0; k < T; ++k) acc[k] += coef * cur[k];
    }
}

int hwo_cons_half(const hwo_problem *p, int to_grid, const double *u_from, const double *u_old,
                  double *u_new, const int64_t *sel, int64_t nsel, int nthreads)
{
    return hwo_cons_half_ext(p, to_grid, u_from, u_old, NULL, 0, NULL, u_new, sel, nsel, nthreads);
}

int hwo_cons_half_ext(const hwo_problem *p, int to_grid, const double *u_from, const double *u_old,
                      const double *f_coef, int n_orders, const double *wall_u, double *u_new,
                      const int64_t *sel, int64_t nsel, int nthreads)
{
    if (check_problem(p) || p->method != HWO_CONSERVATIVE) return -1;
    if (n_orders < 0 || (n_orders > 0 && !f_coef)) return -1;
    const int d = p->d, m = p->m, M = m + 1, P = 2 * m + 2;
    const int Mu_tot = pw(M, d), T = pw(P, d);
    const int64_t count = sel ? nsel : hwo_nodes(p, to_grid);
    tables_t *tb = (tables_t *)malloc(sizeof(tables_t));
    load_tables(m, tb);
    const int nt = nthreads_or_default(nthreads);
#pragma omp parallel num_threads(nt)
    {
        double *b = (double *)calloc((size_t)T * 5, sizeof(double));
        double *a = b, *acc = b + T, *cur = b + 2 * T, *tmp = b + 3 * T, *work = b + 4 * T;
        int md[MAXD];
        for (int i = 0; i < MAXD; ++i) md[i] = m;
#pragma omp for schedule(static)
        for (int64_t q = 0; q < count; ++q) {
            const int64_t node = sel ? sel[q] : q;
            int64_t idx[MAXD];
            corners_t cr;
            out_index(p, to_grid, node, idx);
            find_corners(p, to_grid, idx, &cr);
            const walls_t wu = {to_grid == HWO_PRIMAL ? wall_u : NULL, M};
            tensor_interp(p, tb, &cr, u_from, M, md, &wu, a, work);
            if (n_orders > 0)
                cons_forced_sum(p, a, 0.5 * p->dt, f_coef + node * (int64_t)n_orders * T, n_orders, acc,
                                cur, tmp);
            else
                cons_even_odd_sum(p, a, 0.5 * p->dt, 0, acc, cur, tmp);
            for (int c = 0; c < Mu_tot; ++c) {
                int rem = c, off = 0, st = 1;
                for (int i = 0; i < d; ++i) {
                    off += (rem % M) * st;
                    rem /= M;
                    st *= P;
                }
                u_new[q * Mu_tot + c] = 2.0 * acc[off] - u_old[node * Mu_tot + c];
            }
        }
        free(b);
    }
    free(tb);
    return 0;
}

/* Second time level for the conservative method: the exact Taylor evolution of   */
/* the primal cell interpolants of u0 and v0 (both of degree m data) over dt/2,    */
/* evaluated at the dual nodes.                                                   */
int hwo_cons_startup(const hwo_problem *p, const double *u0, const double *v0, double *u_half,
                     int nthreads)
{
    if (check_problem(p) || p->method != HWO_CONSERVATIVE) return -1;
    const int d = p->d, m = p->m, M = m + 1, P = 2 * m + 2;
    const int Mu_tot = pw(M, d), T = pw(P, d);
    const int64_t count = hwo_nodes(p, HWO_DUAL);
    tables_t *tb = (tables_t *)malloc(sizeof(tables_t));
    load_tables(m, tb);
    const int nt = nthreads_or_default(nthreads);
#pragma omp parallel num_threads(nt)
    {
        double *b = (double *)calloc((size_t)T * 6, sizeof(double));
        double *a = b, *acc = b + T, *cur = b + 2 * T, *tmp = b + 3 * T, *work = b + 4 * T,
               *acc2 = b + 5 * T;
        int md[MAXD];
        for (int i = 0; i < MAXD; ++i) md[i] = m;
#pragma omp for schedule(static)
        for (int64_t node = 0; node < count; ++node) {
            int64_t idx[MAXD];
            corners_t cr;
            out_index(p, HWO_DUAL, node, idx);
            find_corners(p, HWO_DUAL, idx, &cr);
            tensor_interp(p, tb, &cr, u0, M, md, NULL, a, work);
            cons_even_odd_sum(p, a, 0.5 * p->dt, 0, acc, cur, tmp);
            if (v0) {
                tensor_interp(p, tb, &cr, v0, M, md, NULL, a, work);
                cons_even_odd_sum(p, a, 0.5 * p->dt, 1, acc2, cur, tmp);
                for (int k = 0; k < T; ++k) acc[k] += acc2[k];
            }
            for (int c = 0; c < Mu_tot; ++c) {
                int rem = c, off = 0, st = 1;
                for (int i = 0; i < d; ++i) {
                    off += (rem % M) * st;
                    rem /= M;
                    st *= P;
                }
                u_half[node * Mu_tot + c] = acc[off];
            }
        }
        free(b);
    }
    free(tb);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Seminorms.  For the conservative method the discrete energy (Sec. 4.2,      */
/* eq. (Vconst) and Sec. 5.2) is |P+|^2 + |P-|^2 in the |.|_{m+1} seminorm,     */
/* which by the scheme (eq. (eqn)) and the self-adjointness of interpolation    */
/* equals 2(|p^n|^2 - <p^{n+1/2}, p^{n-1/2}>).  The semi-inner product of two    */
/* piecewise polynomials is summed cell by cell:                                 */
/*   <f,g>_cell = prod_i h_i^(1-2q) sum_{a,b} f_a g_b prod_i G[a_i][b_i],        */
/*   G[a][b] = a!/(a-q)! b!/(b-q)! int_{-1/2}^{1/2} z^(a+b-2q) dz, a,b >= q.    */
/* A cell that straddles a non-periodic wall lies half inside the domain in      */
/* that dimension; by the odd/even reflection its integrand is symmetric, so it  */
/* is weighted by 1/2 per such dimension.                                        */
/* ------------------------------------------------------------------------- */
static double falling(int a, int q)
{
    double r = 1.0;
    for (int i = 0; i < q; ++i) r *= (double)(a - i);
    return r;
}

static double gram(int a, int b, int q)
{
    if (a < q || b < q) return 0.0;
    const int e = a + b - 2 * q;
    const double integral = (e % 2) ? 0.0 : 2.0 * pow(0.5, e + 1) / (double)(e + 1);
    return falling(a, q) * falling(b, q) * integral;
}

/* semi-inner product over the cells centred at the nodes of grid `center_grid`   */
/* (interpolating data f, g that live on the other grid)                          */
static double seminorm_pair(const hwo_problem *p, int center_grid, const double *f,
                            const double *g, int mdata, int q, int nthreads)
{
    const int d = p->d, M = mdata + 1, P = 2 * mdata + 2, T = pw(P, d);
    const int64_t count = hwo_nodes(p, center_grid);
    tables_t *tb = (tables_t *)malloc(sizeof(tables_t));
    load_tables(mdata, tb);
    double G[MAXP][MAXP];
    for (int a = 0; a < P; ++a)
        for (int b = 0; b < P; ++b) G[a][b] = gram(a, b, q);
    double hfac = 1.0;
    for (int i = 0; i < d; ++i) hfac *= pow(hdim(p, i), 1.0 - 2.0 * q);
    const int nt = nthreads_or_default(nthreads);
    double total = 0.0;
#pragma omp parallel num_threads(nt) reduction(+ : total)
    {
        double *b = (double *)calloc((size_t)T * 3, sizeof(double));
        double *fa = b, *ga = b + T, *work = b + 2 * T;
        int md[MAXD];
        for (int i = 0; i < MAXD; ++i) md[i] = mdata;
        double sum = 0.0, comp = 0.0; /* Kahan summation over this thread's cells */
#pragma omp for schedule(static)
        for (int64_t node = 0; node < count; ++node) {
            int64_t idx[MAXD];
            corners_t cr;
            out_index(p, center_grid, node, idx);
            find_corners(p, center_grid, idx, &cr);
            tensor_interp(p, tb, &cr, f, M, md, NULL, fa, work);
            tensor_interp(p, tb, &cr, g, M, md, NULL, ga, work);
            double w = hfac;
            for (int i = 0; i < d; ++i)
                if (p->bc[i] != HWO_PERIODIC && center_grid == HWO_PRIMAL &&
                    (idx[i] == 0 || idx[i] == p->n[i]))
                    w *= 0.5;
            double cell = 0.0;
            for (int ia = 0; ia < T; ++ia) {
                if (fa[ia] == 0.0) continue;
                for (int ib = 0; ib < T; ++ib) {
                    int ra = ia, rb = ib;
                    double gg = 1.0;
                    for (int i = 0; i < d; ++i) {
                        gg *= G[ra % P][rb % P];
                        ra /= P;
                        rb /= P;
                    }
                    cell += fa[ia] * gg * ga[ib];
                }
            }
            const double y = w * cell - comp;
            const double t = sum + y;
            comp = (t - sum) - y;
            sum = t;
        }
        total += sum;
        free(b);
    }
    free(tb);
    return total;
}

double hwo_cons_energy(const hwo_problem *p, int grid_a, const double *u_a, const double *u_b_new,
                       const double *u_b_old, int nthreads)
{
    if (check_problem(p) || p->method != HWO_CONSERVATIVE) return NAN;
    const int q = p->m + 1;
    /* cells of the data on grid A are centred at the nodes of the other grid */
    const double aa = seminorm_pair(p, 1 - grid_a, u_a, u_a, p->m, q, nthreads);
    const double bb = seminorm_pair(p, grid_a, u_b_new, u_b_old, p->m, q, nthreads);
    return 2.0 * (aa - bb);
}

double hwo_seminorm(const hwo_problem *p, int data_grid, const double *f, const double *g,
                    int mdata, int q, int nthreads)
{
    if (check_problem(p)) return NAN;
    return seminorm_pair(p, 1 - data_grid, f, g, mdata, q, nthreads);
}

double hwo_diss_energy(const hwo_problem *p, int data_grid, const double *u, const double *v,
                       int nthreads)
{
    /* c^2 |I_m u|^2_{m+1} + |I_{m-1} v|^2_m (Sec. 3.2, eq. (stable1)), 1-D */
    if (check_problem(p) || p->d != 1 || p->m < 1) return NAN;
    const double uu = seminorm_pair(p, 1 - data_grid, u, u, p->m, p->m + 1, nthreads);
    const double vv = seminorm_pair(p, 1 - data_grid, v, v, p->m - 1, p->m, nthreads);
    return p->c * p->c * uu + vv;
}
