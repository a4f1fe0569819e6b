// Internal structures shared by the host side and the kernels of libhermite_wave.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define HW_MAXD 3
#define HW_MAXM 6            // largest nodal degree served by the generic kernel
#define HW_MAXJ 24           // largest Laplacian power in the time sums (d*(m)+1)

enum HwVariant { HWV_DISS_FULL = 0, HWV_DISS_SIMPLE = 1, HWV_CONS = 2, HWV_CONS_STARTUP = 3 };

// Operator set of one nodal degree m, stored as T (float or double), row-major.
// All u operators act on the per-dimension index j = s*(m+1) + l (s = 0 left, 1 right).
//   full : H_m, P x 2M (P = 2m+2, M = m+1)
//   d2   : rows 2..P-1 of H_m scaled by (k+2)(k+1) (the scaled second derivative), 2m x 2M
//   trunc: H_{m-1} on the same 2M inputs with zero columns for l = m, 2m x 2M
//   vop  : H_{m-1}, 2m x 2m (acts on v data, j = s*m + l)
struct OpOffsets {
    int full, d2, trunc, vop;
};

// One problem as seen by a half-step launch in one direction.
struct ProblemDesc {
    int d, m, variant;
    int bc[3];
    int ext_from[3];     // node extents of the grid read
    int ext_to[3];       // node extents of the grid written
    int to_grid;         // 0 primal, 1 dual
    int n_out;           // output nodes (cells) of this half step
    const void* u_in;    // u on the grid read (dissipative, conservative)
    const void* v_in;    // v on the grid read (dissipative) / v0 (start-up) or null
    const void* u_old;   // conservative: old level on the grid written
    void* u_out;
    void* v_out;
    OpOffsets op;        // into the operator pool of matching precision
    double tau;          // dt/2
    double lam2[3];      // (lambda_i/2)^2, lambda_i = c dt / h_i
    // time-sum weights: g(alpha,beta) = j! prod_i F[i][alpha_i][beta_i], j = |beta|
    //   F[i][a][b] = (a+2b)!/a! (lambda_i/2)^(2b) / b!
    double F[3][HW_MAXM + 2][HW_MAXM + 2];
    // per-j coefficients (j! folded in), zero beyond a stage truncation:
    //   dissipative: uQ = tau j!/(2j+1)!, uR = j!/(2j+2)!, vQ = j!/(2j)!, vR = j!/(tau (2j+1)!)
    //   conservative: uQ = j!/(2j)! (even sum), uR = tau j!/(2j+1)! (start-up odd sum)
    double cuQ[HW_MAXJ], cuR[HW_MAXJ], cvQ[HW_MAXJ], cvR[HW_MAXJ];
    // two-kernel form (dissipative): 0 = fused; 1 = interpolate only, writing the
    // cell's p0 | Q | R blocks to work + cell * work_stride; 2 = time evolution only,
    // reading them back
    int split;
    int work_stride;
    void* work;
};

// Forcing and inhomogeneous wall data of one half step of the generic kernel.
// Forcing (u_tt = c^2 Lap u + f): for every output node, `orders` blocks of scaled
// space-time Taylor coefficients h^k/k! d^k/dx^k d^r/dt^r f at the node (FP64), (2m)^d per
// block for the dissipative method (at the start of the half step), (2m+2)^d for the
// conservative one (at the middle time).  w[0][r][j] = tau^(r+2) j!/(2j+r+2)! (u),
// w[1][r][j] = tau^(r+1) j!/(2j+r+1)! (v), zero beyond a stage truncation; the
// conservative update adds twice the u weights of the even orders.
// Walls (half steps onto the primal grid): the wall records of every face (FP64, the
// layout of hw_half_step_ext), u with (m+1)^d and v with m^d values per record; a ghost
// corner gets R(interior) + 2 W(ghost).  correction != 0: the interior data count as zero
// and the outputs are accumulated (+=), so the launch adds the walls' contribution to a
// half step computed with homogeneous walls; `cells` (or null) lists the output nodes
// of the work list.
#define HW_MAXF 16
struct ForcingArgs {
    const double* coef = nullptr; // null: no forcing
    int orders = 0;
    const double* w = nullptr;    // [2][HW_MAXF][HW_MAXJ]
    const double* wall_u = nullptr;
    const double* wall_v = nullptr;
    const int64_t* cells = nullptr;
    int correction = 0;
};

// Energy (conservative): sum over the cells centred at the nodes of `center_grid`
// of w_cell * <I f, I g>_{m+1} (f, g data on the other grid).
struct EnergyDesc {
    int d, m;
    int bc[3];
    int ext_from[3], ext_to[3];
    int center_grid;
    int n_cells;
    const void* f;
    const void* g;
    double hfac;          // prod_i h_i^(1-2(m+1))
    int hi_off;           // offset of the high-row interpolation operator (M x 2M, double)
    int gram_off;         // offset of the Gram block (M x M, double)
};
