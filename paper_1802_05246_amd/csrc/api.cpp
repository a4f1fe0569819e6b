// Host side of libhermite_wave: validation, state buffers, per-problem weight
// tables, the half-step sequence and its hipGraph capture, the energy reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/hermite_wave.h"
#include "hermite_tables.h"
#include "hw_kernels.h"

namespace {

thread_local std::string g_err;

hw_status fail(hw_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            return fail(HW_EHIP, "%s failed: %s", #expr, hipGetErrorString(_e));          \
    } while (0)

double fact(int n)
{
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

int ipow(int b, int e)
{
    int r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

struct Prob {
    hw_problem p{};
    int ext[2][3]{};      // node extents [grid][dim]
    int64_t nodes[2]{};
    int Mu = 0, Mv = 0;   // coefficients per node of u and v
    void* u[2][2]{};      // [grid][slot]
    void* v[2]{};         // dissipative: [grid]
    void* v0tmp = nullptr;
    double h[3]{};
};

} // namespace

struct hw_solver {
    std::vector<Prob> probs;
    int d = 0;
    bool fp64 = true;
    int precision = HW_FP64;
    bool use_tiled = false;
    bool use_cmap = false;        // composed-map MFMA kernel (3-D dissipative, m = 3)
    bool use_batch2d = false;     // batched 2-D path: one persistent launch per (m, method) class
    struct BatchClass {
        int m = 0;
        bool cons = false;
        std::vector<int> probs;            // problems of the class
        DenseArgs* args = nullptr;         // device [phase 0..1][slot parity 0..1][class member]
        int4* tiles[2] = {nullptr, nullptr}; // work list per phase: {member, x0, y0, 0}
        int ntiles[2] = {0, 0};
        int tx = 64;                       // tile code (see set_tile)
    };
    std::vector<BatchClass> bclasses;
    std::vector<int> dense_tx;    // per problem: tile code of the dense kernel (autotuned, see set_tile)
    void* cmap_tables = nullptr;
    bool state_set = false;
    int64_t half_steps = 0;
    size_t elem = 8;
    // device-side tables
    void* ops = nullptr;          // operator pool in the state precision
    double* dops = nullptr;       // FP64 pool for the energy kernel
    std::vector<OpOffsets> op_off; // per m
    std::vector<int> hi_off, gram_off;
    ProblemDesc* descs = nullptr; // [phase 0..1][slot parity 0..1][nprob]
    ProblemDesc* startup_desc = nullptr;
    int64_t* startup_prefix = nullptr;
    int64_t* prefix = nullptr;
    std::vector<int64_t> h_prefix;
    int64_t total_cells[2]{};     // per phase
    size_t lds = 0;
    int grid = 0;
    double* partials = nullptr;
    double* forcing_w = nullptr;  // [2][HW_MAXF][HW_MAXJ] (single problems)
    int64_t* wall_cells = nullptr; // primal nodes whose cell has a ghost corner (single problems)
    int64_t* wall_prefix = nullptr; // {0, n_wall_cells}
    int64_t n_wall_cells = 0;
    void* tiled_tables = nullptr; // weights of the tiled kernel for this problem's lam2 and tau
    std::vector<char> dense;      // per problem: served by the per-lane dense kernel (d <= 2)
    std::vector<const void*> dense_G;  // per problem: its cell matrix in the state precision
    std::vector<void*> dense_alloc;    // the distinct cell matrices (problems with equal maps share)
    std::vector<const void*> cm2_tabs; // per problem: tables of the 2-D composed-map form (or null)
    int64_t* gen_prefix = nullptr;     // prefix sums of the generic kernel's cells (dense problems: 0)
    int64_t gen_total[2]{};
    bool any_generic = true;
    bool split = false;           // two-kernel form
    void* work = nullptr;         // its interpolant workspace
    ProblemDesc* split_descs = nullptr; // [phase][stage 1, 2]
    int energy_grid = 0;
    hipStream_t cap_stream = nullptr;
    // batched 2-D solvers: one capture stream per further class and fork / join events, so
    // that each class's chain of launches is a branch of its own in the captured graph
    std::vector<hipStream_t> class_streams;
    std::vector<hipEvent_t> class_events;   // [0]: fork, [c]: join of class c
    // a small single 1-D problem: its dense arguments per half step k mod 4 on the device, for
    // the one-launch step graph (null otherwise)
    DenseArgs* d1_args = nullptr;
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    std::vector<ProblemDesc> h_descs;
};

namespace {

hw_status validate(const hw_problem* p)
{
    if (!p) return fail(HW_EINVAL, "null problem");
    if (p->d < 1 || p->d > 3) return fail(HW_EINVAL, "d = %d outside 1..3", p->d);
    if (p->method < HW_DISS_FULL || p->method > HW_CONSERVATIVE)
        return fail(HW_EINVAL, "unknown method %d", p->method);
    const int mlo = (p->method == HW_CONSERVATIVE) ? 0 : 1;
    if (p->m < mlo || p->m > HW_MAXM)
        return fail(HW_EINVAL, "m = %d outside %d..%d for this method", p->m, mlo, HW_MAXM);
    if (p->precision < HW_FP64 || p->precision > HW_BF16)
        return fail(HW_EINVAL, "unknown precision %d", p->precision);
    if (p->kernel < HW_KERNEL_AUTO || p->kernel > HW_KERNEL_BATCH)
        return fail(HW_EINVAL, "unknown kernel selector %d", p->kernel);
    if (!(p->c > 0.0) || !(p->dt > 0.0) || !std::isfinite(p->c) || !std::isfinite(p->dt))
        return fail(HW_EINVAL, "c and dt must be positive and finite");
    if (p->taylor_stages < 0) return fail(HW_EINVAL, "taylor_stages must be >= 0");
    double hmin = 1e300;
    for (int i = 0; i < p->d; ++i) {
        if (p->n[i] < 2) return fail(HW_EINVAL, "n[%d] = %d < 2", i, p->n[i]);
        if (!(p->xr[i] > p->xl[i])) return fail(HW_EINVAL, "xr[%d] <= xl[%d]", i, i);
        if (p->bc[i] < HW_PERIODIC || p->bc[i] > HW_NEUMANN)
            return fail(HW_EINVAL, "unknown boundary condition %d in dim %d", p->bc[i], i);
        hmin = std::fmin(hmin, (p->xr[i] - p->xl[i]) / p->n[i]);
    }
    int64_t nodes = 1;
    for (int i = 0; i < p->d; ++i) nodes *= (int64_t)p->n[i] + 1;
    if (nodes * ipow(p->m + 1, p->d) > ((int64_t)1 << 40))
        return fail(HW_EINVAL, "problem too large");
    if (nodes > INT32_MAX) return fail(HW_EINVAL, "more than 2^31 nodes per grid");
    if (p->c * p->dt > hmin * (1.0 + 1e-12))
        return fail(HW_ECFL, "c*dt = %.17g exceeds min h = %.17g (stability needs c dt <= h)",
                    p->c * p->dt, hmin);
    return HW_OK;
}

void fill_geometry(Prob& P)
{
    const hw_problem& p = P.p;
    for (int g = 0; g < 2; ++g) {
        P.nodes[g] = 1;
        for (int i = 0; i < 3; ++i) {
            int e = 1;
            if (i < p.d) e = (p.bc[i] == HW_PERIODIC) ? p.n[i] : (g == 0 ? p.n[i] + 1 : p.n[i]);
            P.ext[g][i] = e;
            P.nodes[g] *= e;
        }
    }
    P.Mu = ipow(p.m + 1, p.d);
    P.Mv = (p.method == HW_CONSERVATIVE) ? 0 : ipow(p.m, p.d);
    for (int i = 0; i < 3; ++i) P.h[i] = i < p.d ? (p.xr[i] - p.xl[i]) / p.n[i] : 1.0;
}

// Operator pools: per m, H_m (full), its scaled second-derivative rows, H_{m-1} on
// the u inputs and H_{m-1} on the v inputs; FP64 pool adds the energy operators.
void build_ops(hw_solver* s, std::vector<double>& pool, std::vector<double>& dpool)
{
    s->op_off.assign(HW_MAXM + 1, OpOffsets{0, 0, 0, 0});
    s->hi_off.assign(HW_MAXM + 1, 0);
    s->gram_off.assign(HW_MAXM + 1, 0);
    for (int m = 0; m <= HW_MAXM; ++m) {
        const int M = m + 1, P = 2 * m + 2, K = 2 * M;
        const double* Hm = kHermiteAll + kHermiteOffset[m];
        OpOffsets o;
        o.full = (int)pool.size();
        for (int r = 0; r < P; ++r)
            for (int k = 0; k < K; ++k) pool.push_back(Hm[r * P + k]);
        o.d2 = (int)pool.size();
        for (int r = 0; r < 2 * m; ++r)
            for (int k = 0; k < K; ++k) pool.push_back(Hm[(r + 2) * P + k] * (r + 2) * (r + 1));
        o.trunc = (int)pool.size();
        o.vop = o.trunc;
        if (m >= 1) {
            const double* Hv = kHermiteAll + kHermiteOffset[m - 1];
            const int Pv = 2 * m;
            for (int r = 0; r < Pv; ++r)
                for (int k = 0; k < K; ++k) {
                    const int sd = k / M, l = k % M;
                    pool.push_back(l < m ? Hv[r * Pv + sd * m + l] : 0.0);
                }
            o.vop = (int)pool.size();
            for (int r = 0; r < Pv; ++r)
                for (int k = 0; k < Pv; ++k) pool.push_back(Hv[r * Pv + k]);
        }
        s->op_off[m] = o;
        // energy: rows m+1..P-1 of H_m, and the Gram block of the (m+1)-th derivative
        s->hi_off[m] = (int)dpool.size();
        for (int r = M; r < P; ++r)
            for (int k = 0; k < K; ++k) dpool.push_back(Hm[r * P + k]);
        s->gram_off[m] = (int)dpool.size();
        const int q = m + 1;
        for (int a = q; a < P; ++a)
            for (int b = q; b < P; ++b) {
                const int e = a + b - 2 * q;
                const double integral = (e % 2) ? 0.0 : 2.0 * std::pow(0.5, e + 1) / (e + 1);
                dpool.push_back(fact(a) / fact(a - q) * fact(b) / fact(b - q) * integral);
            }
    }
}

// descriptor of problem P for half step `phase` (0: first half of a full step) with
// conservative slot parity q
ProblemDesc make_desc(const hw_solver* s, const Prob& P, int phase, int q)
{
    ProblemDesc D;
    std::memset(&D, 0, sizeof D);
    const hw_problem& p = P.p;
    D.d = p.d;
    D.m = p.m;
    for (int i = 0; i < 3; ++i) D.bc[i] = (i < p.d) ? p.bc[i] : HW_PERIODIC;
    D.op = s->op_off[p.m];
    hw_fill_weights(p, P.h, D);
    if (p.method == HW_CONSERVATIVE) {
        D.variant = HWV_CONS;
        const int to = phase == 0 ? HW_PRIMAL : HW_DUAL;
        const int from = 1 - to;
        // phase 0 reads the dual at slot q, phase 1 the primal just written (slot 1-q)
        const int from_slot = (phase == 0) ? q : 1 - q;
        D.to_grid = to;
        D.u_in = P.u[from][from_slot];
        D.u_old = P.u[to][q];
        D.u_out = P.u[to][1 - q];
        for (int i = 0; i < 3; ++i) {
            D.ext_from[i] = P.ext[from][i];
            D.ext_to[i] = P.ext[to][i];
        }
        D.n_out = (int)P.nodes[to];
    } else {
        D.variant = (p.method == HW_DISS_SIMPLE) ? HWV_DISS_SIMPLE : HWV_DISS_FULL;
        const int from = phase == 0 ? HW_PRIMAL : HW_DUAL;
        const int to = 1 - from;
        D.to_grid = to;
        D.u_in = P.u[from][0];
        D.v_in = P.v[from];
        D.u_out = P.u[to][0];
        D.v_out = P.v[to];
        for (int i = 0; i < 3; ++i) {
            D.ext_from[i] = P.ext[from][i];
            D.ext_to[i] = P.ext[to][i];
        }
        D.n_out = (int)P.nodes[to];
    }
    return D;
}

hw_status check_solver(const hw_solver* s)
{
    if (!s) return fail(HW_EINVAL, "null solver");
    return HW_OK;
}

DenseArgs dense_args(const hw_solver* s, int k, int i);

// A 2-D dense kernel variant as one tile code: c > 0 is the per-lane gather form with
// tiles of c x (256 / c) cells, c = -32 / -64 the LDS-staged form (whole node records) with
// tiles of |c| x (256 / |c|), c = -1032 / -1064 the row-chunked staged form with tiles
// (|c| - 1000) wide, c = -2016 the composed-map form on the matrix cores (strips of 16
// cells walking rows)
int tile_width(int code) { return code > 0 ? code : (-code) % 1000; }
int staged_form(int code) { return code > 0 ? 0 : (-code) / 1000 + 1; }
void set_tile(DenseArgs& a, int code)
{
    a.tile_x = tile_width(code);
    a.staged = staged_form(code);
}
// the list launch's variant argument (0, 32 / 64, 1032 / 1064)
int staged_width(int code) { return code < 0 ? -code : 0; }

// a tile code the dense kernels can launch (a choice imposed through HW_TUNE_FORCE may not be)
hw_status check_tile(int code, int m, bool cons, bool fp64)
{
    if (code > 0 && code <= 256 && 256 % code == 0) return HW_OK;
    if (code < 0 && -code < 2000 && (tile_width(code) == 32 || tile_width(code) == 64) &&
        hw_dense_staged_fits(m, cons, fp64, tile_width(code), staged_form(code)))
        return HW_OK;
    if (code == -2016 && hw_cmap2d_supported(m)) return HW_OK;
    return fail(HW_EUNSUPPORTED, "dense tile choice %d not available for m=%d method=%s %s", code, m,
                cons ? "conservative" : "dissipative", fp64 ? "fp64" : "fp32");
}

// rows per strip of the composed-map form on one problem: long chunks (each re-reads one
// node row) while the launch keeps at least 2048 workgroups
int cmap2d_rows(const DenseArgs& a)
{
    const int strips = (a.ext_to[0] + 15) / 16;
    int ry = 256;
    while (ry > 16 && (int64_t)strips * ((a.ext_to[1] + ry - 1) / ry) < 2048) ry /= 2;
    return ry;
}

// one 2-D dense launch in the form the descriptor names
hipError_t launch_dense_any(const DenseArgs& a, int d, int m, bool cons, bool fp64, hipStream_t st)
{
    if (a.staged == 3) return hw_launch_cmap2d(a, m, cons, fp64, cmap2d_rows(a), st);
    return hw_launch_dense(a, d, m, cons, fp64, st);
}

// one batched launch over a class's work list in the form its tile code names
hipError_t launch_list_any(const DenseArgs* args, const int4* items, int n, int m, bool cons, bool fp64,
                           int code, hipStream_t st)
{
    if (staged_form(code) == 3) return hw_launch_cmap2d_list(args, items, n, m, cons, fp64, st);
    return hw_launch_dense_list(args, items, n, m, cons, fp64, staged_width(code), st);
}

// one half step of the problems of batch class C (phase: direction, q: conservative slot parity)
hw_status launch_class_half(const hw_solver* s, const hw_solver::BatchClass& C, int phase, int q, hipStream_t st)
{
    const size_t n = C.probs.size();
    HIP_TRY(launch_list_any(C.args + (size_t)(phase * 2 + q) * n, C.tiles[phase], C.ntiles[phase], C.m, C.cons,
                            s->fp64, C.tx, st));
    return HW_OK;
}

hw_status launch_half(hw_solver* s, int phase, int q, hipStream_t st)
{
    const int np = (int)s->probs.size();
    if (s->use_batch2d) {
        for (const auto& C : s->bclasses) {
            const hw_status r = launch_class_half(s, C, phase, q, st);
            if (r != HW_OK) return r;
        }
        return HW_OK;
    }
    if (s->use_tiled || s->use_cmap) {
        const Prob& P = s->probs[0];
        const ProblemDesc& D = s->h_descs[(size_t)(phase * 2 + q) * np];
        TiledArgs a;
        for (int i = 0; i < 3; ++i) {
            a.ext_from[i] = D.ext_from[i];
            a.ext_to[i] = D.ext_to[i];
            a.bc[i] = D.bc[i];
            a.lam2[i] = D.lam2[i];
        }
        a.to_grid = D.to_grid;
        a.u_in = D.u_in;
        a.v_in = D.v_in;
        a.u_out = D.u_out;
        a.v_out = D.v_out;
        a.tau = D.tau;
        a.tables = s->use_cmap ? s->cmap_tables : s->tiled_tables;
        a.u_old = D.u_old;
        a.cons = D.variant == HWV_CONS ? 1 : 0;
        (void)P;
        if (s->use_cmap) HIP_TRY(hw_launch_cmap3d(a, s->fp64, st));
        else HIP_TRY(hw_launch_tiled(a, s->precision, st));
        return HW_OK;
    }
    if (!s->dense.empty()) {
        for (int i = 0; i < np; ++i) {
            if (!s->dense[i]) continue;
            const ProblemDesc& D = s->h_descs[(size_t)(phase * 2 + q) * np + i];
            const DenseArgs a = dense_args(s, phase * 2 + q, i);
            HIP_TRY(launch_dense_any(a, s->d, D.m, D.variant == HWV_CONS, s->fp64, st));
        }
        if (!s->any_generic) return HW_OK;
        HIP_TRY(hw_launch_generic(s->d, s->fp64, s->descs + (size_t)(phase * 2 + q) * np,
                                  s->gen_prefix + (size_t)phase * (np + 1), np, s->gen_total[phase], s->ops,
                                  s->lds, s->grid, st));
        return HW_OK;
    }
    const ProblemDesc* descs = s->descs + (size_t)(phase * 2 + q) * np;
    const int64_t* prefix = s->prefix + (size_t)phase * (np + 1);
    if (s->split) {
        for (int st2 = 0; st2 < 2; ++st2)
            HIP_TRY(hw_launch_generic(s->d, s->fp64, s->split_descs + phase * 2 + st2, prefix, 1,
                                      s->total_cells[phase], s->ops, s->lds, s->grid, st));
        return HW_OK;
    }
    HIP_TRY(hw_launch_generic(s->d, s->fp64, descs, prefix, np, s->total_cells[phase], s->ops, s->lds,
                              s->grid, st));
    return HW_OK;
}

// Dense-kernel arguments of problem i for half step k = phase * 2 + slot parity.
DenseArgs dense_args(const hw_solver* s, int k, int i)
{
    const int np = (int)s->probs.size();
    const ProblemDesc& D = s->h_descs[(size_t)k * np + i];
    DenseArgs a;
    for (int t = 0; t < 3; ++t) {
        a.ext_from[t] = D.ext_from[t];
        a.ext_to[t] = D.ext_to[t];
        a.bc[t] = D.bc[t];
    }
    a.to_grid = D.to_grid;
    a.u_in = D.u_in;
    a.v_in = D.v_in;
    a.u_old = D.u_old;
    a.u_out = D.u_out;
    a.v_out = D.v_out;
    a.G = s->dense_G[i];
    a.n_cells = D.n_out;
    set_tile(a, s->dense_tx.empty() ? 64 : s->dense_tx[i]);
    a.cm2 = s->cm2_tabs.empty() ? nullptr : s->cm2_tabs[i];
    return a;
}

// Tiles of the variant `code` (tile_width x 256 / tile_width cells) covering the grid
// written in `phase` by the members of a class (member j is problem probs[j]).
void class_tiles(const hw_solver* s, int phase, const std::vector<int>& probs, int code, std::vector<int4>& tiles)
{
    const int np = (int)s->probs.size();
    const int tx = tile_width(code), h = 256 / tx;
    tiles.clear();
    if (staged_form(code) == 3) {
        // composed-map form: strips of 16 cells over chunks of at most 64 cell rows
        for (int j = 0; j < (int)probs.size(); ++j) {
            const ProblemDesc& D = s->h_descs[(size_t)(phase * 2) * np + probs[j]];
            for (int y = 0; y < D.ext_to[1]; y += 64)
                for (int x = 0; x < D.ext_to[0]; x += 16)
                    tiles.push_back(make_int4(j, x, y, std::min(y + 64, D.ext_to[1])));
        }
        return;
    }
    for (int j = 0; j < (int)probs.size(); ++j) {
        const ProblemDesc& D = s->h_descs[(size_t)(phase * 2) * np + probs[j]];
        for (int y = 0; y < D.ext_to[1]; y += h)
            for (int x = 0; x < D.ext_to[0]; x += tx) tiles.push_back(make_int4(j, x, y, 0));
    }
}

// Time `launch` (one warm-up call, three timed) on a private stream; microseconds per call.
template <typename F>
double time_launches(F launch)
{
    hipStream_t ts = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double us = -1.0;
    if (hipStreamCreateWithFlags(&ts, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess) {
        bool ok = launch(ts) == hipSuccess && hipEventRecord(e0, ts) == hipSuccess;
        for (int r = 0; ok && r < 3; ++r) ok = launch(ts) == hipSuccess;
        ok = ok && hipEventRecord(e1, ts) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) us = 1e3 * ms / 3.0;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ts) (void)hipStreamDestroy(ts);
    return us;
}

// zero every state buffer of problem i (before timing launches on it)
void zero_state(hw_solver* s, int i)
{
    const Prob& P = s->probs[i];
    for (int g = 0; g < 2; ++g) {
        for (int sl = 0; sl < 2; ++sl)
            if (P.u[g][sl]) (void)hipMemset(P.u[g][sl], 0, (size_t)P.nodes[g] * P.Mu * s->elem);
        if (P.v[g]) (void)hipMemset(P.v[g], 0, (size_t)P.nodes[g] * P.Mv * s->elem);
    }
}

const std::vector<int> kTileCandidates = {16, 32, 64, 128, -32, -64, -1032, -1064, -2016};

// Tile width of the single-problem dense kernel for 2-D problem i (autotuned).
hw_status tune_dense_single(hw_solver* s, int i)
{
    const Prob& P = s->probs[i];
    if (P.p.d != 2 || !hw_tune_enabled()) return HW_OK;
    zero_state(s, i);
    const bool cons = P.p.method == HW_CONSERVATIVE;
    auto time_us = [&](int cand) {
        DenseArgs a = dense_args(s, 0, i);
        set_tile(a, cand);
        return time_launches([&](hipStream_t ts) { return launch_dense_any(a, 2, P.p.m, cons, s->fp64, ts); });
    };
    s->dense_tx[i] = hw_tune_choose("dense", 2, P.p.m, P.p.method, s->fp64, hw_tune_size_class(P.nodes[1]),
                                    kTileCandidates, time_us);
    return check_tile(s->dense_tx[i], P.p.m, cons, s->fp64);
}

// The batched 2-D path: the problems grouped by (m, method); per class the dense
// kernel's descriptors of every member for the four (phase, slot parity) combinations,
// a tile width timed by the autotuner on the class's largest member, and the work lists.
hw_status setup_batch_classes(hw_solver* s)
{
    const int np = (int)s->probs.size();
    std::map<std::pair<int, int>, int> cls_of;
    for (int i = 0; i < np; ++i) {
        const auto key = std::make_pair(s->probs[i].p.m, s->probs[i].p.method == HW_CONSERVATIVE ? 1 : 0);
        auto it = cls_of.find(key);
        if (it == cls_of.end()) {
            it = cls_of.emplace(key, (int)s->bclasses.size()).first;
            s->bclasses.emplace_back();
            s->bclasses.back().m = key.first;
            s->bclasses.back().cons = key.second != 0;
        }
        s->bclasses[it->second].probs.push_back(i);
    }
    for (auto& C : s->bclasses) {
        const int n = (int)C.probs.size();
        std::vector<DenseArgs> ha((size_t)4 * n);
        for (int k = 0; k < 4; ++k)
            for (int j = 0; j < n; ++j) ha[(size_t)k * n + j] = dense_args(s, k, C.probs[j]);
        if (hipMalloc((void**)&C.args, ha.size() * sizeof(DenseArgs)) != hipSuccess)
            return fail(HW_ENOMEM, "batch descriptor allocation failed");
        auto upload_args = [&](int tx) {
            for (auto& a : ha) set_tile(a, tx);
            return hipMemcpy(C.args, ha.data(), ha.size() * sizeof(DenseArgs), hipMemcpyHostToDevice);
        };
        if (hw_tune_enabled()) {
            int rep = 0;  // member with the most cells
            for (int j = 1; j < n; ++j)
                if (s->probs[C.probs[j]].nodes[1] > s->probs[C.probs[rep]].nodes[1]) rep = j;
            zero_state(s, C.probs[rep]);
            int4* dt = nullptr;
            bool all_cm2 = true; // every member has composed-map tables
            for (int j = 0; j < n; ++j) all_cm2 = all_cm2 && s->cm2_tabs[C.probs[j]] != nullptr;
            auto time_us = [&](int cand) -> double {
                if (staged_form(cand) == 3 && !all_cm2) return -1.0;
                std::vector<int4> tl;
                class_tiles(s, 0, std::vector<int>{C.probs[rep]}, cand, tl);
                for (auto& t : tl) t.x = rep;  // the list names the member's own descriptor
                if (upload_args(cand) != hipSuccess) return -1.0;
                if (dt) (void)hipFree(dt);
                dt = nullptr;
                if (hipMalloc((void**)&dt, tl.size() * sizeof(int4)) != hipSuccess ||
                    hipMemcpy(dt, tl.data(), tl.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess)
                    return -1.0;
                return time_launches([&](hipStream_t ts) {
                    return launch_list_any(C.args, dt, (int)tl.size(), C.m, C.cons, s->fp64, cand, ts);
                });
            };
            C.tx = hw_tune_choose("dense_list", 2, C.m, C.cons ? HW_CONSERVATIVE : HW_DISS_FULL, s->fp64,
                                  hw_tune_size_class(s->probs[C.probs[rep]].nodes[1]), kTileCandidates, time_us);
            if (dt) (void)hipFree(dt);
            const hw_status st = check_tile(C.tx, C.m, C.cons, s->fp64);
            if (st != HW_OK) return st;
            if (staged_form(C.tx) == 3 && !all_cm2)
                return fail(HW_EUNSUPPORTED, "composed-map form: a row of a problem exceeds 4 GB");
        }
        if (upload_args(C.tx) != hipSuccess) return fail(HW_EHIP, "batch descriptor upload failed");
        for (int ph = 0; ph < 2; ++ph) {
            std::vector<int4> tl;
            class_tiles(s, ph, C.probs, C.tx, tl);
            C.ntiles[ph] = (int)tl.size();
            if (hipMalloc((void**)&C.tiles[ph], std::max<size_t>(tl.size(), 1) * sizeof(int4)) != hipSuccess)
                return fail(HW_ENOMEM, "batch work list allocation failed");
            if (!tl.empty() &&
                hipMemcpy(C.tiles[ph], tl.data(), tl.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess)
                return fail(HW_EHIP, "batch work list upload failed");
        }
    }
    return HW_OK;
}

hw_status create_impl(const hw_problem* ps, int count, hw_solver** out)
{
    if (!out) return fail(HW_EINVAL, "null output pointer");
    if (!ps || count < 1) return fail(HW_EINVAL, "need at least one problem");
    for (int i = 0; i < count; ++i) {
        hw_status st = validate(&ps[i]);
        if (st != HW_OK) {
            std::string msg = g_err;
            return fail(st, "problem %d: %s", i, msg.c_str());
        }
        if (ps[i].d != ps[0].d) return fail(HW_EINVAL, "batch problems must share d");
        if ((ps[i].precision == HW_FP64) != (ps[0].precision == HW_FP64))
            return fail(HW_EINVAL, "batch problems must share the precision");
    }
    const hw_problem& p0 = ps[0];
    const bool tiled_ok = count == 1 && hw_tiled_supported(p0.d, p0.m, p0.method, p0.precision);
    if (p0.kernel == HW_KERNEL_TILED && !tiled_ok)
        return fail(HW_EUNSUPPORTED, "no tiled kernel for d=%d m=%d method=%d precision=%d", p0.d,
                    p0.m, p0.method, p0.precision);
    const bool cmap_ok = count == 1 && p0.d == 3 && p0.m == 3 &&
                         (p0.precision == HW_FP64 || p0.precision == HW_FP32);
    if (p0.kernel == HW_KERNEL_COMPOSED && !cmap_ok)
        return fail(HW_EUNSUPPORTED, "the composed-map kernel serves single 3-D problems with m = 3 in FP64 "
                                     "or FP32");
    if (p0.kernel == HW_KERNEL_DENSE)
        for (int i = 0; i < count; ++i)
            if (!hw_dense_supported(ps[i].d, ps[i].m, ps[i].method, ps[i].precision))
                return fail(HW_EUNSUPPORTED, "no dense kernel for d=%d m=%d method=%d precision=%d (problem %d)",
                            ps[i].d, ps[i].m, ps[i].method, ps[i].precision, i);
    if (p0.kernel == HW_KERNEL_BATCH && (p0.d != 2 || p0.precision == HW_BF16))
        return fail(HW_EUNSUPPORTED, "the batched kernel serves 2-D problems in FP64 or FP32");
    if (p0.kernel == HW_KERNEL_SPLIT && (count != 1 || p0.method == HW_CONSERVATIVE))
        return fail(HW_EUNSUPPORTED, "the two-kernel form serves single dissipative problems");
    if (p0.precision == HW_BF16 &&
        (!tiled_ok || p0.kernel == HW_KERNEL_GENERIC || p0.kernel == HW_KERNEL_SPLIT ||
         p0.kernel == HW_KERNEL_DENSE || p0.kernel == HW_KERNEL_COMPOSED || p0.taylor_stages != 0))
        return fail(HW_EUNSUPPORTED, "BF16 operands exist only in the tiled kernel (3-D dissipative full "
                                     "method, m = 3, exact series)");
    for (int i = 0; i < count; ++i)
        if (ps[i].taylor_stages > 0 && ps[i].method == HW_CONSERVATIVE)
            return fail(HW_EINVAL, "taylor_stages applies to the dissipative method only");

    hw_solver* s = new hw_solver();
    s->d = p0.d;
    s->precision = p0.precision;
    s->fp64 = (p0.precision == HW_FP64);
    s->elem = s->fp64 ? 8 : 4;
    s->split = p0.kernel == HW_KERNEL_SPLIT;
    // automatic choice in 3-D, m = 3: the composed-map kernel in FP64 and FP32 (1.9x / 1.3x
    // faster than the tiled kernel on 256^3, with a third of its FP32 rounding error), the
    // tiled kernel for the BF16-operand form, which only it has
    s->use_cmap = cmap_ok && (p0.kernel == HW_KERNEL_COMPOSED || p0.kernel == HW_KERNEL_AUTO);
    s->use_tiled = tiled_ok && p0.kernel != HW_KERNEL_GENERIC && p0.kernel != HW_KERNEL_DENSE && !s->split &&
                   !s->use_cmap && p0.taylor_stages == 0;
    // batches of 2-D problems: one persistent launch per half step over all of them
    s->use_batch2d = p0.d == 2 && p0.precision != HW_BF16 &&
                     (p0.kernel == HW_KERNEL_BATCH || (p0.kernel == HW_KERNEL_AUTO && count > 1));
    if (s->use_batch2d) {
        // every problem of a batched 2-D solver has its cell matrix (conservative m = 6
        // included: the list kernel serves it)
        s->dense.assign(count, 1);
    } else if (!s->use_tiled && !s->use_cmap && !s->split &&
               (p0.kernel == HW_KERNEL_AUTO || p0.kernel == HW_KERNEL_DENSE)) {
        s->dense.assign(count, 0);
        for (int i = 0; i < count; ++i)
            s->dense[i] = hw_dense_supported(ps[i].d, ps[i].m, ps[i].method, ps[i].precision) ? 1 : 0;
        if (std::find(s->dense.begin(), s->dense.end(), 1) == s->dense.end()) s->dense.clear();
    }
    s->dense_tx.assign(count, 64);
    s->probs.resize(count);
    auto cleanup = [&](hw_status st) {
        hw_destroy(s);
        return st;
    };
    for (int i = 0; i < count; ++i) {
        Prob& P = s->probs[i];
        P.p = ps[i];
        fill_geometry(P);
        const bool cons = P.p.method == HW_CONSERVATIVE;
        for (int g = 0; g < 2; ++g) {
            for (int sl = 0; sl < (cons ? 2 : 1); ++sl)
                if (hipMalloc(&P.u[g][sl], (size_t)P.nodes[g] * P.Mu * s->elem) != hipSuccess)
                    return cleanup(fail(HW_ENOMEM, "state allocation failed (problem %d)", i));
            if (!cons && hipMalloc(&P.v[g], (size_t)P.nodes[g] * P.Mv * s->elem) != hipSuccess)
                return cleanup(fail(HW_ENOMEM, "state allocation failed (problem %d)", i));
        }
    }
    // operator pools
    std::vector<double> pool, dpool;
    build_ops(s, pool, dpool);
    if (hipMalloc(&s->ops, pool.size() * s->elem) != hipSuccess ||
        hipMalloc(&s->dops, dpool.size() * sizeof(double)) != hipSuccess)
        return cleanup(fail(HW_ENOMEM, "table allocation failed"));
    if (s->fp64) {
        if (hipMemcpy(s->ops, pool.data(), pool.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(HW_EHIP, "table upload failed"));
    } else {
        std::vector<float> fp(pool.begin(), pool.end());
        if (hipMemcpy(s->ops, fp.data(), fp.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(HW_EHIP, "table upload failed"));
    }
    if (hipMemcpy(s->dops, dpool.data(), dpool.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(HW_EHIP, "table upload failed"));
    // descriptors [phase][q][problem] and per-phase prefix sums of output nodes
    s->h_descs.resize((size_t)4 * count);
    for (int ph = 0; ph < 2; ++ph)
        for (int q = 0; q < 2; ++q)
            for (int i = 0; i < count; ++i)
                s->h_descs[(size_t)(ph * 2 + q) * count + i] = make_desc(s, s->probs[i], ph, q);
    s->h_prefix.assign((size_t)2 * (count + 1), 0);
    size_t lds = 0;
    for (int ph = 0; ph < 2; ++ph) {
        for (int i = 0; i < count; ++i) {
            const ProblemDesc& D = s->h_descs[(size_t)(ph * 2) * count + i];
            s->h_prefix[ph * (count + 1) + i + 1] = s->h_prefix[ph * (count + 1) + i] + D.n_out;
            const int variant = (D.variant == HWV_CONS) ? HWV_CONS_STARTUP : D.variant;
            size_t b = hw_generic_lds_bytes(s->d, D.m, variant, (int)s->elem);
            if (b > lds) lds = b;
        }
        s->total_cells[ph] = s->h_prefix[ph * (count + 1) + count];
    }
    if (lds > 160 * 1024) return cleanup(fail(HW_EUNSUPPORTED, "LDS need %zu B exceeds 160 KiB", lds));
    s->lds = lds;
    int resident = (int)((160 * 1024) / lds);
    if (resident > 16) resident = 16;
    if (resident < 1) resident = 1;
    int64_t g = 256LL * resident * 2;
    const int64_t tmax = s->total_cells[0] > s->total_cells[1] ? s->total_cells[0] : s->total_cells[1];
    if (g > tmax) g = tmax;
    s->grid = (int)(g > 0 ? g : 1);
    if (hipMalloc((void**)&s->descs, s->h_descs.size() * sizeof(ProblemDesc)) != hipSuccess ||
        hipMalloc((void**)&s->prefix, s->h_prefix.size() * sizeof(int64_t)) != hipSuccess ||
        hipMalloc((void**)&s->startup_desc, sizeof(ProblemDesc)) != hipSuccess ||
        hipMalloc((void**)&s->startup_prefix, 2 * sizeof(int64_t)) != hipSuccess ||
        hipMalloc((void**)&s->partials, HW_ENERGY_MAX_GROUPS * sizeof(double)) != hipSuccess)
        return cleanup(fail(HW_ENOMEM, "descriptor allocation failed"));
    if (hipMemcpy(s->descs, s->h_descs.data(), s->h_descs.size() * sizeof(ProblemDesc),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->prefix, s->h_prefix.data(), s->h_prefix.size() * sizeof(int64_t),
                  hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(HW_EHIP, "descriptor upload failed"));
    if (s->split) {
        // workspace of the two-kernel form: per output cell p0 | Q | R
        const int m = p0.m, d = p0.d;
        const bool simple = p0.method == HW_DISS_SIMPLE || d == 1;
        const int P0E = simple ? 2 * m + 2 : m + 1, E = simple ? 2 * m + 2 : 2 * m;
        int stride = 1, ed = 1;
        for (int i = 0; i < d; ++i) {
            stride *= P0E;
            ed *= E;
        }
        stride += 2 * ed;
        const int64_t cells = std::max(s->total_cells[0], s->total_cells[1]);
        if (hipMalloc(&s->work, (size_t)cells * stride * s->elem) != hipSuccess ||
            hipMalloc((void**)&s->split_descs, 4 * sizeof(ProblemDesc)) != hipSuccess)
            return cleanup(fail(HW_ENOMEM, "two-kernel workspace allocation failed"));
        ProblemDesc sd[4];
        for (int ph = 0; ph < 2; ++ph)
            for (int st = 0; st < 2; ++st) {
                sd[ph * 2 + st] = s->h_descs[(size_t)(ph * 2) * count];
                sd[ph * 2 + st].split = st + 1;
                sd[ph * 2 + st].work = s->work;
                sd[ph * 2 + st].work_stride = stride;
            }
        if (hipMemcpy(s->split_descs, sd, sizeof sd, hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(HW_EHIP, "descriptor upload failed"));
    }
    if (count == 1) {
        // forcing weights: u: tau^(r+2) j!/(2j+r+2)!, v: tau^(r+1) j!/(2j+r+1)!, zero for
        // terms beyond a stage truncation (the term enters stage 2j+r+2 / 2j+r+1)
        std::vector<double> fw((size_t)2 * HW_MAXF * HW_MAXJ, 0.0);
        const double tau = 0.5 * p0.dt;
        const int S = p0.taylor_stages;
        for (int r = 0; r < HW_MAXF; ++r)
            for (int j = 0; j < HW_MAXJ; ++j) {
                const int su = 2 * j + r + 2, sv = 2 * j + r + 1;
                if (S <= 0 || su <= S)
                    fw[(size_t)r * HW_MAXJ + j] = std::pow(tau, r + 2) * fact(j) / fact(su);
                if (S <= 0 || sv <= S)
                    fw[(size_t)(HW_MAXF + r) * HW_MAXJ + j] = std::pow(tau, r + 1) * fact(j) / fact(sv);
            }
        if (hipMalloc((void**)&s->forcing_w, fw.size() * sizeof(double)) != hipSuccess)
            return cleanup(fail(HW_ENOMEM, "forcing table allocation failed"));
        if (hipMemcpy(s->forcing_w, fw.data(), fw.size() * sizeof(double), hipMemcpyHostToDevice) !=
            hipSuccess)
            return cleanup(fail(HW_EHIP, "forcing table upload failed"));
    }
    if (count == 1) {
        // primal nodes on a non-periodic wall: the cells of half steps onto the primal grid
        // that have ghost corners (the work list of the wall-data correction)
        const Prob& P = s->probs[0];
        std::vector<int64_t> wc;
        for (int64_t node = 0; node < P.nodes[HW_PRIMAL]; ++node) {
            int64_t r = node;
            bool wall = false;
            for (int i = 0; i < p0.d; ++i) {
                const int e = P.ext[HW_PRIMAL][i];
                const int64_t oi = r % e;
                r /= e;
                if (p0.bc[i] != HW_PERIODIC && (oi == 0 || oi == e - 1)) wall = true;
            }
            if (wall) wc.push_back(node);
        }
        s->n_wall_cells = (int64_t)wc.size();
        if (!wc.empty()) {
            const int64_t pre[2] = {0, s->n_wall_cells};
            if (hipMalloc((void**)&s->wall_cells, wc.size() * sizeof(int64_t)) != hipSuccess ||
                hipMalloc((void**)&s->wall_prefix, sizeof pre) != hipSuccess)
                return cleanup(fail(HW_ENOMEM, "wall cell list allocation failed"));
            if (hipMemcpy(s->wall_cells, wc.data(), wc.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(s->wall_prefix, pre, sizeof pre, hipMemcpyHostToDevice) != hipSuccess)
                return cleanup(fail(HW_EHIP, "wall cell list upload failed"));
        }
    }
    if (!s->dense.empty()) {
        // cell matrices (problems with identical maps share one), and the generic kernel's
        // work list without the dense problems
        std::map<std::vector<double>, void*> made, made2;
        s->dense_G.assign(count, nullptr);
        s->cm2_tabs.assign(count, nullptr);
        for (int i = 0; i < count; ++i) {
            if (!s->dense[i]) continue;
            std::vector<double> G;
            int n_in = 0, n_out = 0;
            hw_cell_map(s->h_descs[i], G, n_in, n_out);
            // the kernel uses corner 0's rows; the others follow by reflection symmetry
            G.resize((size_t)(n_in >> s->d) * n_out);
            if (s->d == 2 && hw_cmap2d_supported(s->probs[i].p.m) &&
                hw_cmap2d_rows_fit(s->probs[i].p.m, s->probs[i].p.method == HW_CONSERVATIVE, s->fp64,
                                   std::max(s->probs[i].ext[0][0], s->probs[i].ext[1][0]))) {
                // tables of the composed-map form (its autotuner candidate)
                auto it2 = made2.find(G);
                if (it2 != made2.end()) {
                    s->cm2_tabs[i] = it2->second;
                } else {
                    void* tabs = nullptr;
                    if (hw_cmap2d_tables_create(G, s->probs[i].p.m, s->probs[i].p.method == HW_CONSERVATIVE, s->fp64,
                                                &tabs) != hipSuccess)
                        return cleanup(fail(HW_EHIP, "composed-map table setup failed"));
                    s->dense_alloc.push_back(tabs);
                    s->cm2_tabs[i] = tabs;
                    made2.emplace(G, tabs);
                }
            }
            auto it = made.find(G);
            if (it != made.end()) {
                s->dense_G[i] = it->second;
                continue;
            }
            std::vector<float> Gf;
            const void* src = G.data();
            size_t bytes = G.size() * sizeof(double);
            if (!s->fp64) {
                Gf.assign(G.begin(), G.end());
                src = Gf.data();
                bytes = Gf.size() * sizeof(float);
            }
            void* dev = nullptr;
            if (hipMalloc(&dev, bytes) != hipSuccess) return cleanup(fail(HW_ENOMEM, "cell matrix allocation failed"));
            s->dense_alloc.push_back(dev);
            if (hipMemcpy(dev, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
                return cleanup(fail(HW_EHIP, "cell matrix upload failed"));
            made.emplace(std::move(G), dev);
            s->dense_G[i] = dev;
        }
        std::vector<int64_t> gp((size_t)2 * (count + 1), 0);
        for (int ph = 0; ph < 2; ++ph) {
            for (int i = 0; i < count; ++i) {
                const int64_t n = s->dense[i] ? 0 : s->h_descs[(size_t)(ph * 2) * count + i].n_out;
                gp[ph * (count + 1) + i + 1] = gp[ph * (count + 1) + i] + n;
            }
            s->gen_total[ph] = gp[ph * (count + 1) + count];
        }
        s->any_generic = std::find(s->dense.begin(), s->dense.end(), 0) != s->dense.end();
        if (hipMalloc((void**)&s->gen_prefix, gp.size() * sizeof(int64_t)) != hipSuccess)
            return cleanup(fail(HW_ENOMEM, "descriptor allocation failed"));
        if (hipMemcpy(s->gen_prefix, gp.data(), gp.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess)
            return cleanup(fail(HW_EHIP, "descriptor upload failed"));
    }
    if (s->use_batch2d) {
        hw_status r = setup_batch_classes(s);
        if (r != HW_OK) return cleanup(r);
        s->dense.clear();  // the classes' launches replace the per-problem dense launches
    } else {
        for (int i = 0; i < count; ++i)
            if (!s->dense.empty() && s->dense[i]) {
                const hw_status st = tune_dense_single(s, i);
                if (st != HW_OK) return cleanup(st);
            }
    }
    if (s->use_cmap && hw_cmap3d_tables_create(s->h_descs[0], s->fp64, &s->cmap_tables) != hipSuccess)
        return cleanup(fail(HW_EHIP, "composed-map table setup failed"));
    if (s->use_tiled) {
        const ProblemDesc& D = s->h_descs[0];
        if (hw_tiled_tables_create(s->precision, D.lam2, D.tau, &s->tiled_tables) != hipSuccess)
            return cleanup(fail(HW_EHIP, "tiled kernel table setup failed"));
    }
    if (s->d == 1 && count == 1 && !s->dense.empty() && s->dense[0] && !s->any_generic) {
        // a 1-D problem of at most 512 cells: a launch per half step costs more than its cells'
        // work, so the step graph runs all its half steps in one single-workgroup launch
        int64_t cells = 0;
        for (int k = 0; k < 4; ++k) cells = std::max<int64_t>(cells, s->h_descs[k].n_out);
        if (cells <= 512) {
            DenseArgs h[4];
            for (int k = 0; k < 4; ++k) h[k] = dense_args(s, k, 0);
            if (hipMalloc((void**)&s->d1_args, sizeof h) != hipSuccess)
                return cleanup(fail(HW_ENOMEM, "argument allocation failed"));
            if (hipMemcpy(s->d1_args, h, sizeof h, hipMemcpyHostToDevice) != hipSuccess)
                return cleanup(fail(HW_EHIP, "argument upload failed"));
        }
    }
    if (hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return cleanup(fail(HW_EHIP, "stream creation failed"));
    if (s->use_batch2d && s->bclasses.size() > 1) {
        // default-priority streams, used only while a graph is captured
        const size_t nb = s->bclasses.size() - 1;
        for (size_t c = 0; c < nb; ++c) {
            hipStream_t st = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
                return cleanup(fail(HW_EHIP, "stream creation failed"));
            s->class_streams.push_back(st);
        }
        for (size_t c = 0; c <= nb; ++c) {
            hipEvent_t ev = nullptr;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
                return cleanup(fail(HW_EHIP, "event creation failed"));
            s->class_events.push_back(ev);
        }
    }
    *out = s;
    return HW_OK;
}

hw_status set_state_impl(hw_solver* s, int i, const double* u, const double* w, hipStream_t st)
{
    if (!s || i < 0 || i >= (int)s->probs.size()) return fail(HW_EINVAL, "bad solver or index");
    if (!u || !w) return fail(HW_EINVAL, "null state pointer");
    Prob& P = s->probs[i];
    HIP_TRY(hw_launch_convert(u, true, P.u[HW_PRIMAL][0], s->fp64, P.nodes[0] * P.Mu, st));
    if (P.p.method == HW_CONSERVATIVE)
        HIP_TRY(hw_launch_convert(w, true, P.u[HW_DUAL][0], s->fp64, P.nodes[1] * P.Mu, st));
    else
        HIP_TRY(hw_launch_convert(w, true, P.v[HW_PRIMAL], s->fp64, P.nodes[0] * P.Mv, st));
    return HW_OK;
}

// The two passes of the energy (Sec. 4.2 eq. (Vconst)): pass 0 = |p_A|^2 on the grid
// not updated last, pass 1 = <p_B^new, p_B^old> on the grid updated last; one partial
// sum per workgroup, at most HW_ENERGY_MAX_GROUPS workgroups (grid-stride over cells).
hw_status energy_passes(hw_solver* s, const void* out, EnergyDesc E[2], int gsz[2])
{
    if (check_solver(s)) return HW_EINVAL;
    if (!out) return fail(HW_EINVAL, "null output");
    if (s->probs.size() != 1) return fail(HW_EINVAL, "energy is per single-problem solver");
    const Prob& P = s->probs[0];
    if (P.p.method != HW_CONSERVATIVE) return fail(HW_EINVAL, "energy is defined for the conservative method");
    if (!s->state_set || s->half_steps < 1) return fail(HW_ESTATE, "energy needs at least one half step");
    const int64_t h = s->half_steps;
    // last update: primal if h is odd, dual if h is even
    const int B = (h & 1) ? HW_PRIMAL : HW_DUAL;
    const int A = 1 - B;
    const int sp = (int)(((h + 1) / 2) & 1), sd = (int)((h / 2) & 1);
    const int slotA = (A == HW_PRIMAL) ? sp : sd;
    const int slotB = (B == HW_PRIMAL) ? sp : sd;
    const void* fa = P.u[A][slotA];
    const void* fb_new = P.u[B][slotB];
    const void* fb_old = P.u[B][1 - slotB];
    const int m = P.p.m;
    double hfac = 1.0;
    for (int i = 0; i < P.p.d; ++i) hfac *= std::pow(P.h[i], 1.0 - 2.0 * (m + 1));
    for (int t = 0; t < 2; ++t) {
        std::memset(&E[t], 0, sizeof E[t]);
        E[t].d = P.p.d;
        E[t].m = m;
        const int data_grid = t == 0 ? A : B;
        E[t].center_grid = 1 - data_grid;
        for (int i = 0; i < 3; ++i) {
            E[t].bc[i] = (i < P.p.d) ? P.p.bc[i] : HW_PERIODIC;
            E[t].ext_from[i] = P.ext[data_grid][i];
            E[t].ext_to[i] = P.ext[E[t].center_grid][i];
        }
        E[t].n_cells = (int)P.nodes[E[t].center_grid];
        E[t].f = t == 0 ? fa : fb_new;
        E[t].g = t == 0 ? fa : fb_old;
        E[t].hfac = hfac;
        E[t].hi_off = s->hi_off[m];
        E[t].gram_off = s->gram_off[m];
        gsz[t] = E[t].n_cells < HW_ENERGY_MAX_GROUPS ? E[t].n_cells : HW_ENERGY_MAX_GROUPS;
    }
    return HW_OK;
}

} // namespace

extern "C" {

const char* hw_last_error(void) { return g_err.c_str(); }

const char* hw_tuning_report(void)
{
    thread_local std::string text;
    text = hw_tune_report_text();
    return text.c_str();
}

hw_status hw_create(const hw_problem* p, hw_solver** out) { return create_impl(p, 1, out); }

hw_status hw_batch_create(const hw_problem* ps, int count, hw_solver** out)
{
    return create_impl(ps, count, out);
}

void hw_destroy(hw_solver* s)
{
    if (!s) return;
    for (auto& kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    for (Prob& P : s->probs) {
        for (int g = 0; g < 2; ++g) {
            for (int sl = 0; sl < 2; ++sl)
                if (P.u[g][sl]) (void)hipFree(P.u[g][sl]);
            if (P.v[g]) (void)hipFree(P.v[g]);
        }
        if (P.v0tmp) (void)hipFree(P.v0tmp);
    }
    if (s->ops) (void)hipFree(s->ops);
    if (s->dops) (void)hipFree(s->dops);
    if (s->descs) (void)hipFree(s->descs);
    if (s->startup_desc) (void)hipFree(s->startup_desc);
    if (s->startup_prefix) (void)hipFree(s->startup_prefix);
    if (s->prefix) (void)hipFree(s->prefix);
    if (s->partials) (void)hipFree(s->partials);
    if (s->forcing_w) (void)hipFree(s->forcing_w);
    if (s->wall_cells) (void)hipFree(s->wall_cells);
    if (s->wall_prefix) (void)hipFree(s->wall_prefix);
    if (s->tiled_tables) hw_tiled_tables_destroy(s->tiled_tables);
    if (s->cmap_tables) (void)hipFree(s->cmap_tables);
    for (void* g : s->dense_alloc) (void)hipFree(g);
    for (auto& C : s->bclasses) {
        if (C.args) (void)hipFree(C.args);
        for (int ph = 0; ph < 2; ++ph)
            if (C.tiles[ph]) (void)hipFree(C.tiles[ph]);
    }
    if (s->gen_prefix) (void)hipFree(s->gen_prefix);
    if (s->work) (void)hipFree(s->work);
    if (s->split_descs) (void)hipFree(s->split_descs);
    if (s->d1_args) (void)hipFree(s->d1_args);
    for (hipEvent_t ev : s->class_events) (void)hipEventDestroy(ev);
    for (hipStream_t st : s->class_streams) (void)hipStreamDestroy(st);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    delete s;
}

hw_status hw_batch_layout(const hw_solver* s, int i, int grid, int64_t* n_nodes, int* n_u, int* n_v)
{
    if (!s || i < 0 || i >= (int)s->probs.size()) return fail(HW_EINVAL, "bad solver or index");
    if (grid != HW_PRIMAL && grid != HW_DUAL) return fail(HW_EINVAL, "bad grid %d", grid);
    const Prob& P = s->probs[i];
    if (n_nodes) *n_nodes = P.nodes[grid];
    if (n_u) *n_u = P.Mu;
    if (n_v) *n_v = P.Mv;
    return HW_OK;
}

hw_status hw_layout(const hw_solver* s, int grid, int64_t* n_nodes, int* n_u, int* n_v)
{
    return hw_batch_layout(s, 0, grid, n_nodes, n_u, n_v);
}

hw_status hw_batch_set_state(hw_solver* s, int i, const double* u, const double* w, void* stream)
{
    hw_status st = set_state_impl(s, i, u, w, (hipStream_t)stream);
    if (st != HW_OK) return st;
    s->half_steps = 0;
    s->state_set = true;
    return HW_OK;
}

hw_status hw_set_state(hw_solver* s, const double* u, const double* w, void* stream)
{
    return hw_batch_set_state(s, 0, u, w, stream);
}

hw_status hw_batch_cons_startup(hw_solver* s, int i, const double* u0, const double* v0, void* stream)
{
    if (!s || i < 0 || i >= (int)s->probs.size()) return fail(HW_EINVAL, "bad solver or index");
    if (!u0) return fail(HW_EINVAL, "null u0");
    Prob& P = s->probs[i];
    if (P.p.method != HW_CONSERVATIVE) return fail(HW_EINVAL, "start-up is for the conservative method");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hw_launch_convert(u0, true, P.u[HW_PRIMAL][0], s->fp64, P.nodes[0] * P.Mu, st));
    if (v0) {
        if (!P.v0tmp && hipMalloc(&P.v0tmp, (size_t)P.nodes[0] * P.Mu * s->elem) != hipSuccess)
            return fail(HW_ENOMEM, "v0 staging allocation failed");
        HIP_TRY(hw_launch_convert(v0, true, P.v0tmp, s->fp64, P.nodes[0] * P.Mu, st));
    }
    ProblemDesc D = make_desc(s, P, 1, 0);
    D.variant = HWV_CONS_STARTUP;
    D.u_in = P.u[HW_PRIMAL][0];
    D.v_in = v0 ? P.v0tmp : nullptr;
    D.u_old = nullptr;
    D.u_out = P.u[HW_DUAL][0];
    int64_t h_pre[2] = {0, D.n_out};
    HIP_TRY(hipMemcpyAsync(s->startup_desc, &D, sizeof D, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->startup_prefix, h_pre, sizeof h_pre, hipMemcpyHostToDevice, st));
    const size_t lds = hw_generic_lds_bytes(s->d, P.p.m, HWV_CONS_STARTUP, (int)s->elem);
    const int grid = (int)(D.n_out < 4096 ? D.n_out : 4096);
    HIP_TRY(hw_launch_generic(s->d, s->fp64, s->startup_desc, s->startup_prefix, 1, D.n_out, s->ops,
                              lds, grid, st));
    HIP_TRY(hipStreamSynchronize(st));
    s->half_steps = 0;
    s->state_set = true;
    return HW_OK;
}

hw_status hw_cons_startup(hw_solver* s, const double* u0, const double* v0, void* stream)
{
    return hw_batch_cons_startup(s, 0, u0, v0, stream);
}

hw_status hw_half_steps(hw_solver* s, int n, void* stream)
{
    if (check_solver(s)) return HW_EINVAL;
    if (n < 0) return fail(HW_EINVAL, "negative step count");
    if (!s->state_set) return fail(HW_ESTATE, "state not set");
    hipStream_t st = (hipStream_t)stream;
    for (int k = 0; k < n; ++k) {
        const int phase = (int)(s->half_steps & 1);
        const int q = (int)((s->half_steps >> 1) & 1);
        hw_status r = launch_half(s, phase, q, st);
        if (r != HW_OK) return r;
        s->half_steps++;
    }
    return HW_OK;
}

hw_status hw_half_step_ext(hw_solver* s, const double* f_coef, int n_orders, const double* wall_u,
                           const double* wall_v, void* stream)
{
    if (check_solver(s)) return HW_EINVAL;
    if (s->probs.size() != 1 || !s->forcing_w)
        return fail(HW_EINVAL, "forcing and wall data apply to single problems");
    const Prob& P = s->probs[0];
    const bool cons = P.p.method == HW_CONSERVATIVE;
    if (n_orders < 0 || n_orders > HW_MAXF)
        return fail(HW_EINVAL, "n_orders must be in 0..%d", HW_MAXF);
    if (n_orders > 0 && !f_coef) return fail(HW_EINVAL, "null forcing coefficients");
    if (cons ? (wall_v != nullptr) : ((wall_u == nullptr) != (wall_v == nullptr)))
        return fail(HW_EINVAL, cons ? "the conservative method has no v wall data"
                                    : "dissipative wall data need both the u and the v records");
    if (!s->state_set) return fail(HW_ESTATE, "state not set");
    hipStream_t st = (hipStream_t)stream;
    const int phase = (int)(s->half_steps & 1);
    const int q = (int)((s->half_steps >> 1) & 1);
    const ProblemDesc* desc = s->descs + (size_t)(phase * 2 + q);
    const bool to_primal = s->h_descs[(size_t)(phase * 2 + q)].to_grid == HW_PRIMAL;
    const bool walls = wall_u != nullptr && to_primal && s->n_wall_cells > 0;
    if (n_orders > 0) {
        // the generic kernel carries the forcing terms (and the wall data with them)
        ForcingArgs fa;
        fa.coef = f_coef;
        fa.orders = n_orders;
        fa.w = s->forcing_w;
        if (walls) {
            fa.wall_u = wall_u;
            fa.wall_v = wall_v;
        }
        HIP_TRY(hw_launch_generic(s->d, s->fp64, desc, s->prefix + (size_t)phase * 2, 1,
                                  s->total_cells[phase], s->ops, s->lds, s->grid, st, &fa));
    } else {
        // the problem's own kernel with homogeneous walls, then the walls' contribution
        // added to the wall cells (the half step is linear in the ghost data)
        hw_status r = launch_half(s, phase, q, st);
        if (r != HW_OK) return r;
        if (walls) {
            ForcingArgs fa;
            fa.wall_u = wall_u;
            fa.wall_v = wall_v;
            fa.cells = s->wall_cells;
            fa.correction = 1;
            const int grid = (int)std::min<int64_t>(s->n_wall_cells, (int64_t)s->grid);
            HIP_TRY(hw_launch_generic(s->d, s->fp64, desc, s->wall_prefix, 1, s->n_wall_cells, s->ops,
                                      s->lds, grid, st, &fa));
        }
    }
    s->half_steps++;
    return HW_OK;
}

hw_status hw_half_step_forced(hw_solver* s, const double* f_coef, int n_orders, void* stream)
{
    return hw_half_step_ext(s, f_coef, n_orders, nullptr, nullptr, stream);
}

static hw_status graph_for(hw_solver* s, int n, hipGraphExec_t* out)
{
    const int q = (int)((s->half_steps >> 1) & 1);
    // the conservative slot parity selects buffers; dissipative steps do not depend on it
    bool any_cons = false;
    for (const Prob& P : s->probs) any_cons |= (P.p.method == HW_CONSERVATIVE);
    auto key = std::make_pair(n, any_cons ? q : 0);
    auto it = s->graphs.find(key);
    if (it != s->graphs.end()) {
        *out = it->second;
        return HW_OK;
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
    hw_status r = HW_OK;
    const int nb = (int)s->class_streams.size();
    if (nb > 0) {
        // batched 2-D problems: a class's half steps depend only on the class's own previous
        // half step, so each class runs its whole chain as a branch of the graph (class 0
        // on the capture stream, class c on class_streams[c - 1]), forked from one event and
        // joined back before the capture ends; branches may then run concurrently
        bool ok = hipEventRecord(s->class_events[0], s->cap_stream) == hipSuccess;
        for (int c = 0; c < nb; ++c)
            ok = ok && hipStreamWaitEvent(s->class_streams[c], s->class_events[0], 0) == hipSuccess;
        if (!ok) r = fail(HW_EHIP, "graph fork failed");
        for (int c = 0; c <= nb && r == HW_OK; ++c) {
            hipStream_t st = c == 0 ? s->cap_stream : s->class_streams[c - 1];
            int64_t hs = s->half_steps;
            for (int k = 0; k < 2 * n && r == HW_OK; ++k, ++hs)
                r = launch_class_half(s, s->bclasses[c], (int)(hs & 1), (int)((hs >> 1) & 1), st);
        }
        // the joins are made whatever happened above, so that no stream is left capturing
        for (int c = 0; c < nb; ++c) {
            const bool j = hipEventRecord(s->class_events[c + 1], s->class_streams[c]) == hipSuccess &&
                           hipStreamWaitEvent(s->cap_stream, s->class_events[c + 1], 0) == hipSuccess;
            if (!j && r == HW_OK) r = fail(HW_EHIP, "graph join failed");
        }
    } else if (s->d1_args) {
        // a small 1-D problem: all 2n half steps in one launch (the first one's index mod 4
        // is 2 q, or any even value for the dissipative method, whose steps ignore q)
        const Prob& P = s->probs[0];
        if (hw_launch_dense1d_steps(s->d1_args, (int)(s->half_steps & 3), 2 * n, P.p.m,
                                    P.p.method == HW_CONSERVATIVE, s->fp64, s->cap_stream) != hipSuccess)
            r = fail(HW_EHIP, "one-launch 1-D step failed");
    } else {
        int64_t hs = s->half_steps;
        for (int k = 0; k < 2 * n && r == HW_OK; ++k, ++hs)
            r = launch_half(s, (int)(hs & 1), (int)((hs >> 1) & 1), s->cap_stream);
    }
    hipError_t e = hipStreamEndCapture(s->cap_stream, &graph);
    if (r != HW_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (e != hipSuccess) return fail(HW_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(HW_EHIP, "graph instantiate failed: %s", hipGetErrorString(e));
    s->graphs[key] = exec;
    *out = exec;
    return HW_OK;
}

hw_status hw_prepare_advance(hw_solver* s, int n)
{
    if (check_solver(s)) return HW_EINVAL;
    if (n < 1 || n > INT32_MAX / 2) return fail(HW_EINVAL, "step count %d outside 1..%d", n, INT32_MAX / 2);
    if (s->half_steps & 1) return fail(HW_ESTATE, "advance needs whole steps (odd half-step count)");
    hipGraphExec_t exec = nullptr;
    return graph_for(s, n, &exec);
}

hw_status hw_batch_advance(hw_solver* s, int n, void* stream)
{
    if (check_solver(s)) return HW_EINVAL;
    if (n < 0 || n > INT32_MAX / 2) return fail(HW_EINVAL, "step count %d outside 0..%d", n, INT32_MAX / 2);
    if (!s->state_set) return fail(HW_ESTATE, "state not set");
    if (s->half_steps & 1) return fail(HW_ESTATE, "advance needs whole steps (odd half-step count)");
    if (n == 0) return HW_OK;
    hipGraphExec_t exec = nullptr;
    hw_status r = graph_for(s, n, &exec);
    if (r != HW_OK) return r;
    HIP_TRY(hipGraphLaunch(exec, (hipStream_t)stream));
    s->half_steps += 2 * (int64_t)n;
    return HW_OK;
}

hw_status hw_advance(hw_solver* s, int n, void* stream) { return hw_batch_advance(s, n, stream); }

hw_status hw_batch_get_state(const hw_solver* s, int i, double* u, double* w, void* stream)
{
    if (!s || i < 0 || i >= (int)s->probs.size()) return fail(HW_EINVAL, "bad solver or index");
    if (!u || !w) return fail(HW_EINVAL, "null output pointer");
    if (!s->state_set) return fail(HW_ESTATE, "state not set");
    const Prob& P = s->probs[i];
    hipStream_t st = (hipStream_t)stream;
    const int64_t h = s->half_steps;
    if (P.p.method == HW_CONSERVATIVE) {
        const int sp = (int)(((h + 1) / 2) & 1), sd = (int)((h / 2) & 1);
        HIP_TRY(hw_launch_convert(P.u[HW_PRIMAL][sp], s->fp64, u, true, P.nodes[0] * P.Mu, st));
        HIP_TRY(hw_launch_convert(P.u[HW_DUAL][sd], s->fp64, w, true, P.nodes[1] * P.Mu, st));
    } else {
        const int g = (int)(h & 1);
        HIP_TRY(hw_launch_convert(P.u[g][0], s->fp64, u, true, P.nodes[g] * P.Mu, st));
        HIP_TRY(hw_launch_convert(P.v[g], s->fp64, w, true, P.nodes[g] * P.Mv, st));
    }
    return HW_OK;
}

hw_status hw_get_state(const hw_solver* s, double* u, double* w, void* stream)
{
    return hw_batch_get_state(s, 0, u, w, stream);
}

int hw_state_grid(const hw_solver* s)
{
    if (!s) return -1;
    const int64_t h = s->half_steps;
    if (s->probs[0].p.method != HW_CONSERVATIVE) return (int)(h & 1);
    // conservative: the first half step of each full step updates the primal grid
    if (h == 0) return HW_DUAL;
    return (h & 1) ? HW_PRIMAL : HW_DUAL;
}

double hw_time(const hw_solver* s)
{
    if (!s) return NAN;
    const Prob& P = s->probs[0];
    if (P.p.method == HW_CONSERVATIVE) return (double)((s->half_steps + 1) / 2) * P.p.dt;
    return 0.5 * (double)s->half_steps * P.p.dt;
}

hw_status hw_energy(hw_solver* s, double* e_out, void* stream)
{
    EnergyDesc E[2];
    int gsz[2];
    hw_status r = energy_passes(s, e_out, E, gsz);
    if (r != HW_OK) return r;
    hipStream_t st = (hipStream_t)stream;
    double total[2];
    for (int t = 0; t < 2; ++t) {
        HIP_TRY(hw_launch_energy(s->d, s->fp64, E[t], s->dops, s->partials, gsz[t], st));
        std::vector<double> part(gsz[t]);
        HIP_TRY(hipMemcpyAsync(part.data(), s->partials, gsz[t] * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        double sum = 0.0, comp = 0.0;
        for (int k = 0; k < gsz[t]; ++k) {
            const double y = part[k] - comp;
            const double tt = sum + y;
            comp = (tt - sum) - y;
            sum = tt;
        }
        total[t] = sum;
    }
    *e_out = 2.0 * (total[0] - total[1]);
    return HW_OK;
}

hw_status hw_energy_noalloc(hw_solver* s, double* e_out_device, void* stream)
{
    EnergyDesc E[2];
    int gsz[2];
    hw_status r = energy_passes(s, e_out_device, E, gsz);
    if (r != HW_OK) return r;
    for (int t = 0; t < 2; ++t)
        if (gsz[t] > HW_ENERGY_MAX_GROUPS)
            return fail(HW_EINVAL, "energy pass %d needs %d partial sums, the static scratch holds %d", t,
                        gsz[t], HW_ENERGY_MAX_GROUPS);
    HIP_TRY(hw_launch_energy_noalloc(s->d, s->fp64, E[0], gsz[0], E[1], gsz[1], s->dops, e_out_device,
                                     (hipStream_t)stream));
    return HW_OK;
}

hw_status hw_probe_stream_triad(int64_t n, double* gbs_out)
{
    if (!gbs_out || n < 1024 || (n & 1)) return fail(HW_EINVAL, "need an even n >= 1024 and an output pointer");
    double *a = nullptr, *b = nullptr, *c = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hw_status r = HW_OK;
    const size_t bytes = (size_t)n * sizeof(double);
    if (hipMalloc((void**)&a, bytes) != hipSuccess || hipMalloc((void**)&b, bytes) != hipSuccess ||
        hipMalloc((void**)&c, bytes) != hipSuccess) {
        r = fail(HW_ENOMEM, "triad arrays allocation failed");
    } else if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
               hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        r = fail(HW_EHIP, "triad stream setup failed");
    } else {
        const int reps = 10;
        bool ok = hipMemsetAsync(b, 0, bytes, st) == hipSuccess && hipMemsetAsync(c, 0, bytes, st) == hipSuccess;
        for (int k = 0; ok && k < 2; ++k) ok = hw_probe_triad_launch(a, b, c, n, st) == hipSuccess;
        ok = ok && hipEventRecord(e0, st) == hipSuccess;
        for (int k = 0; ok && k < reps; ++k) ok = hw_probe_triad_launch(a, b, c, n, st) == hipSuccess;
        ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f)
            *gbs_out = 24.0 * (double)n * reps / (ms * 1e-3) / 1e9;
        else
            r = fail(HW_EHIP, "triad probe failed");
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (c) (void)hipFree(c);
    return r;
}

hw_status hw_probe_mfma(int precision, double* tflops_out)
{
    if (!tflops_out || (precision != HW_FP64 && precision != HW_FP32))
        return fail(HW_EINVAL, "precision must be HW_FP64 or HW_FP32, output non-null");
    const bool fp64 = precision == HW_FP64;
    const int groups = 256 * 8, iters = 4096, chains = 8;
    void* sink = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hw_status r = HW_OK;
    if (hipMalloc(&sink, (size_t)groups * 256 * 8) != hipSuccess) {
        r = fail(HW_ENOMEM, "probe sink allocation failed");
    } else if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
               hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        r = fail(HW_EHIP, "probe stream setup failed");
    } else {
        bool ok = hw_probe_mfma_launch(fp64, sink, groups, iters, st) == hipSuccess;
        ok = ok && hipEventRecord(e0, st) == hipSuccess;
        ok = ok && hw_probe_mfma_launch(fp64, sink, groups, iters, st) == hipSuccess;
        ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
        float ms = 0.0f;
        if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f) {
            const double flops = (double)groups * 4 * iters * chains * 2048.0;
            *tflops_out = flops / (ms * 1e-3) / 1e12;
        } else {
            r = fail(HW_EHIP, "MFMA probe failed");
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (sink) (void)hipFree(sink);
    return r;
}

hw_status hw_probe_coexec(double ms_out[3])
{
    if (!ms_out) return fail(HW_EINVAL, "output pointer is null");
    const int groups = 4096, iters = 4096;
    float* sink = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hw_status r = HW_OK;
    if (hipMalloc((void**)&sink, (size_t)groups * 256 * sizeof(float)) != hipSuccess) {
        r = fail(HW_ENOMEM, "probe sink allocation failed");
    } else if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
               hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        r = fail(HW_EHIP, "probe stream setup failed");
    } else {
        for (int mode = 0; mode < 3 && r == HW_OK; ++mode) {
            bool ok = hw_probe_coexec_launch(mode, sink, groups, iters, st) == hipSuccess;
            ok = ok && hipEventRecord(e0, st) == hipSuccess;
            ok = ok && hw_probe_coexec_launch(mode, sink, groups, iters, st) == hipSuccess;
            ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f)
                ms_out[mode] = ms;
            else
                r = fail(HW_EHIP, "co-execution probe failed");
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (sink) (void)hipFree(sink);
    return r;
}

} // extern "C"
