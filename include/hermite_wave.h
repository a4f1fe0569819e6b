/*
 * hermite_wave.h -- C ABI of libhermite_wave.so: the staggered half-step of the
 * dissipative (order 2m-1) and conservative (order 2m) Hermite methods for
 * u_tt = c^2 Lap u (Appelo, Hagstrom & Vargas, "Hermite Methods for the Scalar
 * Wave Equation"), on one AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Sec. 2.1, Sec. 3, Sec. 4):
 *   domain prod_i [xl_i, xr_i], n_i cells, h_i = (xr_i - xl_i)/n_i;
 *   constant speed c, time step dt with c dt <= min_i h_i (Sec. 1);
 *   walls per dimension: periodic, Dirichlet or Neumann (Sec. 3.1.3: ghost polynomials
 *   by odd / even extension; homogeneous, or with wall data through hw_half_step_ext);
 *   nodal degree m: (m+1)^d coefficients of u per node, m^d of v (dissipative).
 *
 * Grids (Sec. 2.1).  Primal nodes x_i = xl + i h, dual nodes x_{i+1/2}.  Periodic
 * dimensions carry n_i nodes on both grids; other dimensions carry n_i + 1 primal
 * nodes (i = 0..n_i) and n_i dual nodes.  A half step maps the data of one grid at
 * time t to the other grid at t + dt/2 (dissipative), or updates one grid from
 * t - dt/2 to t + dt/2 using the other grid at t (conservative, Sec. 4.1).
 *
 * Array layout at this boundary.  Every state array is FP64, node-major with the
 * node index i0 + n0*(i1 + n1*i2) (x fastest), coefficient-minor with the
 * coefficient index l0 + M*(l1 + M*l2) (l_x fastest), M = m+1 for u and M = m for
 * v.  Values are the scaled Taylor coefficients h^l/l! d^l f of Sec. 2.2 (v is
 * scaled in space only).  All array pointers passed in are DEVICE pointers owned
 * by the caller; the library copies from / into them on the given stream and
 * keeps no reference after the call returns.  Internally the state may be held in
 * FP32 (HW_FP32); conversion happens at set/get time.
 *
 * Errors.  Every call returns a status; none aborts or throws across the ABI.
 * hw_last_error() gives a thread-local message for the last failure.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Calls are
 * asynchronous on that stream except hw_energy, which synchronises it.
 */
#ifndef HERMITE_WAVE_H
#define HERMITE_WAVE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HW_OK = 0,
    HW_EINVAL = -1,       /* bad argument (null pointer, d, m, n, bc, method...) */
    HW_ECFL = -2,         /* c dt > min_i h_i (1 + 1e-12): outside the stability bound */
    HW_ENOMEM = -3,       /* device allocation failed */
    HW_EUNSUPPORTED = -4, /* no kernel for this (d, m, method, precision, kernel) */
    HW_EHIP = -5,         /* a HIP runtime call failed */
    HW_ESTATE = -6        /* call out of order (e.g. stepping before set_state) */
} hw_status;

typedef enum {
    HW_DISS_FULL = 0,    /* dissipative, modified first step for d >= 2 (Sec. 3.3) */
    HW_DISS_SIMPLE = 1,  /* dissipative, straightforward tensor extension (Sec. 3.3) */
    HW_CONSERVATIVE = 2  /* conservative (Sec. 4.1, Sec. 4.3) */
} hw_method;

typedef enum { HW_PERIODIC = 0, HW_DIRICHLET = 1, HW_NEUMANN = 2 } hw_bc;

typedef enum {
    HW_FP64 = 0, /* FP64 storage and arithmetic */
    HW_FP32 = 1, /* FP32 storage; FP32 MFMA contractions where a tiled kernel exists */
    HW_BF16 = 2  /* FP32 storage, BF16 MFMA operands with FP32 accumulation (tiled only) */
} hw_precision;

typedef enum {
    HW_KERNEL_AUTO = 0,    /* 3-D m = 3 (either method): composed in FP64 and FP32, tiled
                              for BF16 operands; 2-D batches: batched; single problems with
                              d <= 2: dense where it exists; else generic */
    HW_KERNEL_GENERIC = 1, /* one workgroup per cell, any d <= 3, any supported m */
    HW_KERNEL_TILED = 2,   /* LDS-tiled MFMA kernel (3-D dissipative full, m = 3) */
    HW_KERNEL_SPLIT = 3,   /* two kernels per half step, as in the paper's two-kernel GPU
                              design (Sec. 6.1): the first writes each cell's interpolants
                              (p0, Q, R) to a device workspace, the second reads them and
                              sums the Taylor series; single dissipative problems only
                              (HW_EUNSUPPORTED otherwise); for comparison with the fused
                              kernels */
    HW_KERNEL_DENSE = 4,   /* one lane per cell, d <= 2: the cell's half step as one dense
                              matrix (built once per problem from the same operators and
                              time-sum weights) applied to its corner nodes, one launch per
                              problem of a batch; d = 1 (any m), d = 2 dissipative (any m),
                              d = 2 conservative m <= 5, FP64 or FP32 (HW_EUNSUPPORTED
                              otherwise; with HW_KERNEL_AUTO the other problems of a batch
                              share one generic launch) */
    HW_KERNEL_COMPOSED = 5, /* 3-D, m = 3, dissipative (full or simple variant, any
                              truncation) or conservative, FP64 or FP32, single problems: each
                              cell's half step as its composed matrix (conservative: the even
                              time sum S, then u_new = 2 S - u_old), corners combined by the
                              reflection symmetry of the Hermite operators, applied per output
                              parity class to 16 cells at a time on the matrix cores
                              (HW_EUNSUPPORTED otherwise) */
    HW_KERNEL_BATCH = 6    /* 2-D, FP64 or FP32, any m and method, batches or single problems:
                              the problems grouped by (m, method); per group and half step one
                              launch of the dense kernel runs one workgroup per item of a work
                              list of tiles (or strips) of every problem of the group (at most
                              one launch per group, all of them in the captured graph); form
                              and tile shape chosen by the autotuner (HW_EUNSUPPORTED
                              otherwise; the default for 2-D batches) */
} hw_kernel;

typedef enum { HW_PRIMAL = 0, HW_DUAL = 1 } hw_grid;

typedef struct {
    int d;            /* space dimension, 1..3 */
    int m;            /* nodal degree: dissipative 1..6, conservative 0..6 */
    int n[3];         /* cells per dimension (>= 2); entries beyond d ignored */
    double xl[3];     /* lower domain bound per dimension */
    double xr[3];     /* upper domain bound per dimension (> xl) */
    double c;         /* wave speed (> 0) */
    double dt;        /* time step (> 0), c dt <= min h_i */
    int bc[3];        /* hw_bc per dimension */
    int method;       /* hw_method */
    int precision;    /* hw_precision */
    int taylor_stages;/* 0: exact (terminating) Taylor series in time; s > 0: keep
                         stages 0..s only (the truncated series of Sec. 6.1), dissipative */
    int kernel;       /* hw_kernel */
} hw_problem;

typedef struct hw_solver hw_solver;

/* Validate the problem and allocate the state buffers on the current device.
 * Sec. 2.1 (grids), Sec. 1 (c dt <= h).  *out is set only on HW_OK. */
hw_status hw_create(const hw_problem* p, hw_solver** out);

/* Free everything the solver owns (NULL is accepted). */
void hw_destroy(hw_solver* s);

/* Node count of `grid` and the number of u and v coefficients per node
 * (v count is 0 for the conservative method).  Any output pointer may be NULL.
 * Sec. 2.1 (primal and dual grids), Sec. 2.2 ((m+1)^d Taylor coefficients of u and
 * m^d of v per node, Sec. 3.1.1). */
hw_status hw_layout(const hw_solver* s, int grid, int64_t* n_nodes, int* n_u_coef,
                    int* n_v_coef);

/* Set the state at time t0 = 0.
 * Dissipative: u_primal, v_or_u_dual = u and v on the primal grid (Sec. 3.1.1).
 * Conservative: u_primal = u on the primal grid at t0, v_or_u_dual = u on the dual
 * grid at t0 + dt/2 (the two time levels of Sec. 4.1). */
hw_status hw_set_state(hw_solver* s, const double* u_primal, const double* v_or_u_dual,
                       void* stream);

/* Conservative only: build both levels from u0 (and v0, or NULL for v0 = 0), both
 * primal arrays of (m+1)^d coefficients; the dual level at t0 + dt/2 is the exact
 * Taylor evolution of the degree-m cell interpolants (start-up step). */
hw_status hw_cons_startup(hw_solver* s, const double* u0, const double* v0_or_null,
                          void* stream);

/* Advance n full steps (2n half steps, Sec. 3.1.2 / Sec. 4.1).  The step loop is
 * captured once per (n, buffer parity) in a hipGraph and replayed on `stream`; for a
 * single 1-D problem of at most 512 cells the graph is one single-workgroup launch that
 * runs all 2n half steps (the same per-cell arithmetic as one launch per half step).
 * Dissipative: requires the state on the primal grid. */
hw_status hw_advance(hw_solver* s, int n_full_steps, void* stream);

/* Capture and instantiate the hipGraph that hw_advance(s, n) replays from the
 * current step parity, without launching it, so that a later hw_advance(s, n) does
 * no capture work.  Batches: use it with the batch solver as well. */
hw_status hw_prepare_advance(hw_solver* s, int n_full_steps);

/* Advance n half steps with plain kernel launches (no graph). */
hw_status hw_half_steps(hw_solver* s, int n_half, void* stream);

/* One half step of a single problem with a forcing term and / or inhomogeneous,
 * time-dependent wall data (plain launches, no graph).
 *
 * Forcing, u_tt = c^2 Lap u + f.  Dissipative method: Sec. 3.1.2 eq.
 * (recursion_diss_1d_2), stage s of the Taylor series in time receives dt^s/s! times the
 * (s-1)-th time derivative of f.  Conservative method: eq. (wavequ) with f in the even
 * Taylor sum of eq. (update), d^2r u/dt^2r = c^2 Lap d^(2r-2) u/dt^(2r-2) +
 * d^(2r-2) f/dt^(2r-2).  Both in closed form, exact for f polynomial in time up to the
 * orders given.  f_coef: device pointer (FP64, caller-owned, read during the call's
 * kernels on `stream`) to [n_out][n_orders][K^d] values phi[r][k] = h^k/k! d^k/dx^k
 * d^r/dt^r f (k a multi-index, k_x fastest, 0 <= k_i < K) at every node of the grid this
 * half step writes (the grid opposite hw_state_grid for the dissipative method; node
 * order as in hw_layout), with K = 2m at the time at the start of the half step
 * (dissipative) and K = 2m+2 at the middle time, the time of the other grid's level
 * (conservative; only the even orders r enter).  n_orders: 0..16 (0 = no forcing; f_coef
 * may then be NULL).  A taylor_stages truncation drops the forcing terms of later stages
 * as well.  With forcing the whole half step runs in the generic kernel.
 *
 * Wall data (Sec. 3.1.3).  On a half step that writes the primal grid the cells at a
 * non-periodic wall have ghost corners.  With wall_u (and, dissipative, wall_v) NULL they
 * are the homogeneous odd (Dirichlet) / even (Neumann) mirror images of the interior
 * nodes.  Otherwise the ghost data are R(interior) + 2 W(ghost): R the homogeneous mirror,
 * W the solution's prescribed-parity part about the wall (Dirichlet: its even normal part,
 * whose constant term is the wall value g(t) and whose higher even terms follow from g
 * through the PDE, e.g. u_xx = (g_tt - c^2 Lap_tangential g)/c^2; Neumann: its odd normal
 * part), taken at the ghost node half a cell beyond the wall; at corners the walls are
 * applied dimension by dimension in increasing order.  The records (FP64 device arrays,
 * caller-owned) give W at wall points:
 *   faces: for every non-periodic dimension i in increasing order, the low wall
 *     (x_i = xl_i) then the high wall (x_i = xr_i);
 *   wall points of face i: the positions of the input grid's nodes (the dual grid,
 *     hw_layout) in the other dimensions t, extended by one ghost position at each end
 *     when t is non-periodic (index 0 = half a cell below xl_t, n_t + 1 = half a cell above
 *     xr_t; periodic t: the n_t dual nodes), x fastest;
 *   one record per wall point: M^d values (M = m+1 for wall_u, m for wall_v), coefficient
 *     index l_x fastest; in dimension i the index j stands for the normal degree k = 2j
 *     (Dirichlet) or 2j+1 (Neumann); each entry is h_i^k/k! d_i^k prod_{t != i}
 *     h_t^l_t/l_t! d_t^l_t of the solution (u, resp. v = u_t) at the wall point and at the
 *     time of the half step's input data.
 * The records are read only on half steps that write the primal grid (else ignored) and
 * only at the wall points some ghost corner needs.  Without forcing the problem's own
 * kernel runs the half step with homogeneous walls and a second launch adds the wall
 * data's contribution to the cells at the walls (the half step is linear in the ghost
 * data).
 *
 * HW_EINVAL for batches, n_orders out of range, a NULL f_coef with n_orders > 0, a
 * dissipative call with only one of wall_u / wall_v, or a conservative one with wall_v;
 * HW_ESTATE if no state is set. */
hw_status hw_half_step_ext(hw_solver* s, const double* f_coef, int n_orders, const double* wall_u,
                           const double* wall_v, void* stream);

/* hw_half_step_ext with homogeneous walls. */
hw_status hw_half_step_forced(hw_solver* s, const double* f_coef, int n_orders, void* stream);

/* Copy the state out (device pointers, FP64, layouts as above; the data of Sec. 3.1.1
 * for the dissipative method, the two staggered levels of Sec. 4.1 for the
 * conservative one).
 * Dissipative: u and v of the grid that holds the state (hw_state_grid).
 * Conservative: u on the primal grid and u on the dual grid (newest levels). */
hw_status hw_get_state(const hw_solver* s, double* u, double* v_or_u_dual, void* stream);

/* Grid that holds the dissipative state (HW_PRIMAL after whole steps); for the
 * conservative method, the grid updated last.  -1 on a NULL solver. */
int hw_state_grid(const hw_solver* s);

/* Conservative only: the discrete energy 2(|p_A|^2 - <p_B^new, p_B^old>) in the
 * |.|_{m+1} seminorm (Sec. 4.2 eq. (Vconst), Sec. 5.2), A = the grid not updated
 * last, B = the grid updated last with its new and previous levels.  Cells
 * straddling a non-periodic wall weigh 1/2 per such dimension.  FP64 accumulation,
 * deterministic order.  Synchronises `stream`.  HW_ESTATE before the first step. */
hw_status hw_energy(hw_solver* s, double* e_out, void* stream);

/* The same energy without any allocation, for callers that cannot allocate memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * writes E to e_out_device (a caller-owned DEVICE double) asynchronously on `stream`;
 * no host synchronisation, no host-side buffer.  The per-workgroup partial sums of both
 * passes go to a fixed device array of the library, 2 x 2048 doubles (32 KiB) on each GPU
 * it runs on, held until the process ends: calls that overlap on one GPU (concurrent
 * streams or threads) race on it and must be serialised by the caller.  Any grid size is
 * served (at most 2048 workgroups per pass, grid-stride over cells); HW_EINVAL if a pass
 * would need more partial sums than the array holds.  The two passes' partials are
 * summed on the GPU in a fixed order, so the result agrees with hw_energy to rounding
 * (a different summation order), not bit for bit.  Other errors as hw_energy. */
hw_status hw_energy_noalloc(hw_solver* s, double* e_out_device, void* stream);

/* Simulated time of the primal level: t0 + (half steps applied)/2 * dt for the
 * dissipative method; the primal level's time for the conservative method
 * (Sec. 3.1.2: a full step advances both grids by dt; Sec. 4.1: the conservative
 * levels are staggered by dt/2). */
double hw_time(const hw_solver* s);

/* Thread-local message describing the last failure ("" if none). */
const char* hw_last_error(void);

/* The autotuner's choices so far in this process, one line per key (kernel, d, m,
 * method, precision, size class -> chosen launch shape, its time).  Launch shapes are
 * timed on the problem itself when a solver is created (HW_AUTOTUNE=0 in the environment
 * turns this off; HW_TUNE_CACHE=<file> keeps the choices across processes;
 * HW_TUNE_FORCE=<kernel>=<choice>[,...] imposes a choice, e.g. "dense=-64,dense_list=16").
 * For the 2-D dense kernels ("dense", "dense_list") a choice c > 0 is the per-lane gather
 * form with tiles of c x (256 / c) cells, c = -32 or -64 the LDS-staged form (whole node
 * records in LDS) with tiles of |c| x (256 / |c|) cells, c = -1032 or -1064 the row-chunked
 * staged form (one coefficient row of the tile's nodes in LDS at a time) with tiles 32 or
 * 64 cells wide, c = -2016 (m = 3..6 only) the composed-map form on the matrix cores
 * (strips of 16 cells walking their cell rows; the four corner sums of each cell formed
 * in LDS, the cell matrix applied as 16x16x4 products).  HW_TUNE_LOG=1 prints every
 * candidate's time to stderr while it is measured; "cmap3d_offsets=64" makes the 3-D
 * composed-map kernel use 64-bit per-lane offsets, the form otherwise taken only for layers
 * over 4 GB.  The text is
 * thread-local and valid until the next call from the same thread.  This is about the
 * implementation's launch configuration, not the method of the paper. */
const char* hw_tuning_report(void);

/* ---- peak probes -------------------------------------------------------------------
 * Measured attainable peaks of the current GPU, against which the rooflines are set (the
 * paper times a DAXPY on its GPU for its attainable bandwidth, Sec. 6).  Both allocate
 * their own buffers, run on a private stream and synchronise it.
 * hw_probe_stream_triad: a = b + s c over three FP64 arrays of n elements (n even, >= 1024;
 *   choose them far larger than the caches), 10 timed passes after 2 untimed;
 *   *gbs_out = 24 n bytes per pass / time, in GB/s.
 * hw_probe_mfma: 2048 workgroups of 4 waves, each wave 4096 rounds of 8 independent
 *   16x16x4 matrix-core products (2048 flops each) in HW_FP32 or HW_FP64, no memory
 *   traffic; *tflops_out in TFLOP/s.
 * hw_probe_coexec: whether matrix-core and vector work overlap on a SIMD.  4096
 *   workgroups of 4 waves, each wave 4096 rounds; a round is 4 independent FP32 16x16x4
 *   products and/or 32 independent FP32 vector FMAs.  ms_out[0]: products only, [1]: FMAs
 *   only, [2]: both in every wave (milliseconds per launch).  [2] near max([0], [1]) means
 *   the two overlap, near [0] + [1] that they take turns. */
hw_status hw_probe_stream_triad(int64_t n, double* gbs_out);
hw_status hw_probe_mfma(int precision, double* tflops_out);
hw_status hw_probe_coexec(double ms_out[3]);

/* ---- batches: independent problems advanced together --------------------------
 * Many independent problems of the kind above (each one the problem statement of
 * Sec. 2.1 with its own grid, m, c, dt, walls and method, Sec. 3 / Sec. 4) stepped
 * together.  All problems of a batch share d and precision.  hw_batch_advance captures
 * the step loop in a hipGraph.  How a half step of the batch is launched depends on
 * the kernel selector: HW_KERNEL_GENERIC runs one grid-stride launch over a work list
 * of (problem, cell); HW_KERNEL_AUTO / HW_KERNEL_BATCH for 2-D batches run one dense
 * launch per (m, method) group, one workgroup per tile (or strip) of all its problems, in
 * the form the autotuner chose for the group (in the captured graph each group's chain of
 * launches is a branch of its own, so the groups may run concurrently); HW_KERNEL_DENSE
 * runs one dense launch per problem the dense kernel serves and one generic launch over
 * the remaining problems.
 * hw_batch_layout, hw_batch_set_state, hw_batch_cons_startup and hw_batch_get_state
 * are hw_layout, hw_set_state, hw_cons_startup and hw_get_state for problem i. */
hw_status hw_batch_create(const hw_problem* ps, int count, hw_solver** out);
hw_status hw_batch_layout(const hw_solver* b, int i, int grid, int64_t* n_nodes, int* n_u_coef,
                          int* n_v_coef);
hw_status hw_batch_set_state(hw_solver* b, int i, const double* u_primal,
                             const double* v_or_u_dual, void* stream);
hw_status hw_batch_cons_startup(hw_solver* b, int i, const double* u0, const double* v0_or_null,
                                void* stream);
hw_status hw_batch_advance(hw_solver* b, int n_full_steps, void* stream);
hw_status hw_batch_get_state(const hw_solver* b, int i, double* u, double* v_or_u_dual,
                             void* stream);

#ifdef __cplusplus
}
#endif
#endif
