// LDS-tiled half-step kernel for the 3-D dissipative method with the modified first
// step (Sec. 3.3, d = 3), nodal degree m = 3, element type T = float or double, and a
// BF16-operand form (FP32 storage and accumulation, BF16 operands of the matrix-core
// stages).
//
// A workgroup owns a column of 4 x TY cells (TY = 8 for float, 4 for double) and walks
// it upwards in z, one node layer of the input grid at a time.  Per layer:
//   1. the (4+1) x (TY+1) nodes of the layer (u: 64, v: 27 coefficients), loaded into
//      registers during the previous layer, are stashed in LDS; ghost nodes outside
//      non-periodic walls are mirrored with the odd / even coefficient signs of
//      Sec. 3.1.3; the cell layer finished in the previous pass is stored and the loads
//      of the next node layer are issued;
//   2. x-pass, once per x-edge of the layer (shared by the cells on both sides), on
//      the matrix cores: the 16 stacked rows [H_3 rows 0..3 | rows 2..7 of H_3 times
//      (k+2)(k+1) | H_{m-1} on l <= 2] times the 8 inputs (side s, l_x) of the 16
//      (l_y, l_z) lines of the edge, one 16x16x8 product per edge; v lines meet
//      H_{m-1} on the vector units;
//   3. y- and z-passes per (cell, k_x, half of the k_y range): the y-pass of this
//      layer is combined with the previous layer's (kept in registers) into the
//      z-pass, giving for the cell between the two layers p0 (centre rows),
//      Q = I_{m-1}^3 v and R = sum_i (lambda_i/2)^2 d_i^2 c^(i) (modified first step),
//      the latter divided by (lambda_z/2)^2;
//   4. the Taylor series in time is summed in closed form (Sec. 3.1.2).  With
//      S(k) = prod_i ((lambda_i/2)^2)^floor(k_i/2), k = a + 2b and j = |b|,
//        u' = p0 + sum_b W(a,b) S(k)/S(a) [tau Q/(2j+1)! + R/(2j+2)!]
//        v' =      sum_b W(a,b) S(k)/S(a) [Q/(2j)! + R/(tau (2j+1)!)]
//      W(a,b) = j!/prod b_i! prod (a_i+2b_i)!/a_i!.  For a given lambda and tau every
//      factor is a constant, so each input's weight is one table entry built on the
//      host.  Only k with the parity of a enter, so the sums split into 8 parity
//      classes, each a dense (<= 16 outputs) x (27 Q + 27 R inputs) block applied to
//      16 cells at a time on the matrix cores; the outputs are staged in LDS for the
//      coalesced 16-byte stores of step 1 of the next pass.
// Every node of the input grid is read from HBM once per column (plus the one-node
// halo shared with the neighbouring columns), every output node written once.
#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>

#include "hermite_tables.h"
#include "hw_kernels.h"

namespace {

constexpr int TX = 4;

constexpr double kFact[20] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0, 5040.0, 40320.0,
                              362880.0, 3628800.0, 39916800.0, 479001600.0, 6227020800.0,
                              87178291200.0, 1307674368000.0, 20922789888000.0,
                              355687428096000.0, 6402373705728000.0, 121645100408832000.0};

// 1-D operators (compile-time tables; device uses need compile-time indices)
__host__ __device__ constexpr double opH3(int r, int c) { return kH3c[r * 8 + c]; } // c = s*4 + l
__host__ __device__ constexpr double opD2(int r, int c)                               // r = 0..5
{
    return kH3c[(r + 2) * 8 + c] * (double)((r + 2) * (r + 1));
}
__host__ __device__ constexpr double opH2(int r, int c) { return kH2c[r * 6 + c]; } // c = s*3 + l
__host__ __device__ constexpr double opH2t(int r, int c)                              // c = s*4 + l
{
    return (c % 4 == 3) ? 0.0 : kH2c[r * 6 + (c / 4) * 3 + (c % 4)];
}
// x-pass stacked rows: 0..3 H_3 centre rows, 4..9 second-derivative rows, 10..15 H_2t
__host__ __device__ constexpr double opX(int r, int c)
{
    return r < 4 ? opH3(r, c) : (r < 10 ? opD2(r - 4, c) : opH2t(r - 10, c));
}

// LDS strides are odd numbers of 4-byte words so that the lanes of a wave, which
// index neighbouring nodes, edges or cells, fall into different banks.
constexpr int NUP = 65;  // node stride of u
constexpr int NVP = 29;  // node stride of v
constexpr int XUR = 20;  // row stride of an edge's u x-pass results (rows 4 apart: 80 words)
constexpr int XUE = 16 * XUR + 1; // x-edge stride of the u x-pass results: [row][l_y + 4 l_z]
constexpr int XVE = 55;  // x-edge stride of the v x-pass results: [row][l_y + 3 l_z] + 1
constexpr int P0S = 65;  // cell stride of p0: [kx + 4 ky + 16 kz]
constexpr int ZS = 433;  // cell stride of [tau S Q (216) | S R (216) | 0]
constexpr int OUS = 68;  // cell stride of the staged u outputs (16-byte rows for the stores;
                         // word 64 takes the writes of unused time-sum rows)

// time-sum blocks: 8 classes x 14 K-steps of 4 (54 inputs padded to 56)
constexpr int TS_KSTEPS = 14;

template <typename T, int TY>
struct Shared {
    static constexpr int NXL = TX + 1, NYL = TY + 1;
    static constexpr int NNODE = NXL * NYL;
    static constexpr int NEDGE = TX * NYL;
    static constexpr int NC = TX * TY;
    T nu[NNODE * NUP];
    T nv[NNODE * NVP];
    T xu[NEDGE * XUE];
    T xv[NEDGE * XVE];
    T p0[NC * P0S];
    T z[NC * ZS];
    alignas(32) T out[NC * (OUS + 27)]; // staged outputs of a cell layer: u (stride OUS), then v (27)
    static_assert(NC % 16 == 0, "cells come in groups of 16 for the time-sum products");
};

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float vec __attribute__((ext_vector_type(4)));
    static __device__ inline vec mac(float a, float b, vec c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // row of the 16x16 result held in element r of lane l (column = l % 16)
    static __device__ inline int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct Mfma<double> {
    typedef double vec __attribute__((ext_vector_type(4)));
    static __device__ inline vec mac(double a, double b, vec c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int l, int r) { return (l >> 4) + 4 * r; }
};

// Device tables (per element type and per lambda, tau: the class-block weights carry the
// scalings), built on the host:
//   xa[2][64]          A operand of the x-pass (K-step, lane): opX[l%16][4 ks + l/16]
//   ta[8][14][64]      A operand of the class blocks (class, K-step, lane)
//   tk[8][56]          LDS offset in the cell block [Q|R|0] of input kk of a class
//   tr[8][16]          output of (class, row): -1 unused, else
//                      is_v << 12 | scale mask (alpha_i >= 2) << 8 | flat alpha index
template <typename T>
struct Tables {
    T xa[2][64];
    T ta[8][TS_KSTEPS][64];
    int tk[8][TS_KSTEPS * 4];
    int tr[8][16];
    // BF16-operand form (16x16x32 products, 8 operands per lane, k = 8 (lane / 16) + e):
    //   xb[64][8]        x-pass A operand: opX[l % 16][k] for k < 8, else 0
    //   tb[8][2][64][8]  class-block A operand, K-block kb: W[l % 16][32 kb + k] without the
//                    lambda and tau factors (the BF16 form scales in the kernel)
    //   kb8[8][2][4][8]  LDS offset of input 32 kb + 8 g + e of a class (padding: zero slot)
    unsigned short xb[64][8];
    unsigned short tb[8][2][64][8];
    int kb8[8][2][4][8];
};

// bf16 bit pattern of x, rounded to nearest even
inline unsigned short to_bf16(double x)
{
    float f = (float)x;
    unsigned int u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

struct Map1 {
    int j, ghost;
};

__device__ inline Map1 map_node(int gi, int ext, int bc)
{
    Map1 m;
    m.ghost = 0;
    if (bc == 0) {
        int j = gi;
        while (j < 0) j += ext;
        while (j >= ext) j -= ext;
        m.j = j;
    } else if (gi < 0) {
        m.j = 0;
        m.ghost = 1;
    } else if (gi >= ext) {
        m.j = ext - 1;
        m.ghost = 1;
    } else {
        m.j = gi;
    }
    return m;
}

// sign of coefficient l of a node mirrored across a wall of type bc
__device__ inline bool flips(int bc, int l) { return (bc == 1) ? ((l & 1) == 0) : ((l & 1) == 1); }

// One output row of a 1-D Hermite operator from the sums E[l] = left + right and
// differences O[l] = left - right of the two nodes' data.  The operators satisfy
// H[k][right, l] = (-1)^(k+l) H[k][left, l] (reflection of the cell about its centre),
// so row k needs only the left-node column and E or O by the parity of k + l; `parity`
// is the derivative order k of the row (row + 2 for the second-derivative rows).
template <int NL, typename T, typename Op>
__device__ inline T sym(Op op, int row, int parity, const T* E, const T* O, T acc = T(0))
{
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        const double w = op(row, l);
        if (w != 0.0) acc += T(w) * (((parity + l) & 1) ? O[l] : E[l]);
    }
    return acc;
}

// y- and z-passes of the R and Q paths for rows k_y = KH .. KH+2 of one (cell, k_x).
// Unscaled form (the factors S(k), (lambda_z/2)^2 and tau are part of the time-sum weights):
//   Ay[ky][lz <= 2] = gx H2t_y d2_x + gy d2_y H2t_x,  gx,y = (l_x,y/2)^2 / (l_z/2)^2   (z operator H_2),
//   By[ky][lz <= 3] = H2t_y H2t_x                                                    (z operator d2),
//   Cy[ky][lz <= 2] = H2_y H2_x v,
// so that the z-pass gives Q = I_{m-1}^3 v and R / (l_z/2)^2 (scaled form: below).  yz_y computes this
// layer's y-pass (cA: 9 of its 16 entries, cB, cC); yz_z combines the previous layer
// (pA, pB, pC, side s = 0) with this one (side s = 1), stores Q and R / (l_z/2)^2 of
// the cell and moves this layer's results into pA, pB, pC.
// Scalings of the y/z-passes.  Unscaled form: gx, gy only.  Scaled form (BF16 operands,
// whose weights must stay free of lambda and tau, see the table builder): the row
// factors f = S_x(k_x) S_y(k_y) times l_x, l_y, l_z (the (lambda/2)^2) and tau, the
// z-factors S_z applied at the end, as Q and R are then stored pre-scaled by S(k)
// (tau S Q and S R).
template <typename T>
struct YzScale {
    T gx, gy, l2x, l2y, l2z, tau;
};

template <int KH, bool SC, typename T>
__device__ inline void yz_y(const T* xu0, const T* xu1, const T* xv0, const T* xv1, int kx,
                            T (&cA)[16], T (&cB)[12], T (&cC)[9], const YzScale<T>& sc)
{
    T fx[3], fy[3], fb[3], fc[3];
    const T skx = kx < 2 ? T(1) : (kx < 4 ? sc.l2x : sc.l2x * sc.l2x);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int ky = KH + j;
        const T f = (ky / 2 == 0) ? skx : ((ky / 2 == 1) ? skx * sc.l2y : skx * (sc.l2y * sc.l2y));
        fx[j] = SC ? f * sc.l2x : sc.gx;
        fy[j] = SC ? f * sc.l2y : sc.gy;
        fb[j] = f * sc.l2z;
        fc[j] = f * sc.tau;
    }
#pragma unroll
    for (int lz = 0; lz < 4; ++lz) {
        T Eh[4], Oh[4];
#pragma unroll
        for (int ly = 0; ly < 4; ++ly) {
            const T a0 = xu0[(10 + kx) * XUR + ly + 4 * lz], a1 = xu1[(10 + kx) * XUR + ly + 4 * lz];
            Eh[ly] = a0 + a1;
            Oh[ly] = a0 - a1;
        }
        if (lz < 3) {
            T Ed[3], Od[3], Eq[3], Oq[3];
#pragma unroll
            for (int ly = 0; ly < 3; ++ly) {
                const T d0 = xu0[(4 + kx) * XUR + ly + 4 * lz], d1 = xu1[(4 + kx) * XUR + ly + 4 * lz];
                const T q0 = xv0[kx * 9 + ly + 3 * lz], q1 = xv1[kx * 9 + ly + 3 * lz];
                Ed[ly] = d0 + d1;
                Od[ly] = d0 - d1;
                Eq[ly] = q0 + q1;
                Oq[ly] = q0 - q1;
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int ky = KH + j;
                cA[j + 3 * lz] = fx[j] * sym<3>(opH2, ky, ky, Ed, Od) + fy[j] * sym<4>(opD2, ky, ky + 2, Eh, Oh);
                const T c = sym<3>(opH2, ky, ky, Eq, Oq);
                cC[j + 3 * lz] = SC ? fc[j] * c : c;
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const T b = sym<3>(opH2, KH + j, KH + j, Eh, Oh);
            cB[j + 3 * lz] = SC ? fb[j] * b : b;
        }
    }
}

template <int KH, bool SC, typename T>
__device__ inline void yz_z(bool emit, int kx, T (&pA)[16], T (&pB)[12], T (&pC)[9], const T (&cA)[16],
                            const T (&cB)[12], const T (&cC)[9], T* zc, T l2z)
{
    const T sz[3] = {T(1), l2z, l2z * l2z};
    if (emit) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int ky = KH + j;
            T EA[3], OA[3], EC[3], OC[3], EB[4], OB[4];
#pragma unroll
            for (int lz = 0; lz < 3; ++lz) {
                EA[lz] = pA[j + 3 * lz] + cA[j + 3 * lz];
                OA[lz] = pA[j + 3 * lz] - cA[j + 3 * lz];
                EC[lz] = pC[j + 3 * lz] + cC[j + 3 * lz];
                OC[lz] = pC[j + 3 * lz] - cC[j + 3 * lz];
            }
#pragma unroll
            for (int lz = 0; lz < 4; ++lz) {
                EB[lz] = pB[j + 3 * lz] + cB[j + 3 * lz];
                OB[lz] = pB[j + 3 * lz] - cB[j + 3 * lz];
            }
#pragma unroll
            for (int kz = 0; kz < 6; ++kz) {
                const int k = kx + 6 * ky + 36 * kz;
                const T q = sym<3>(opH2, kz, kz, EC, OC);
                const T r = sym<4>(opD2, kz, kz + 2, EB, OB, sym<3>(opH2, kz, kz, EA, OA));
                zc[k] = (SC && kz >= 2) ? q * sz[kz / 2] : q;
                zc[216 + k] = (SC && kz >= 2) ? r * sz[kz / 2] : r;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        pA[i] = cA[i];
        pC[i] = cC[i];
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) pB[i] = cB[i];
}

// p0 (centre rows) of one (cell, k_x): y-pass Y[ky][lz] = sum_{s,ly} H3[ky][s,ly]
// xu[e_s][kx][ly + 4 lz] of this layer, z-pass with the previous layer's (pA)
template <typename T>
__device__ inline void p0_y(const T* xu0, const T* xu1, int kx, T (&cur)[16])
{
#pragma unroll
    for (int lz = 0; lz < 4; ++lz) {
        T E[4], O[4];
#pragma unroll
        for (int ly = 0; ly < 4; ++ly) {
            const T a0 = xu0[kx * XUR + ly + 4 * lz], a1 = xu1[kx * XUR + ly + 4 * lz];
            E[ly] = a0 + a1;
            O[ly] = a0 - a1;
        }
#pragma unroll
        for (int ky = 0; ky < 4; ++ky) cur[ky + 4 * lz] = sym<4>(opH3, ky, ky, E, O);
    }
}

template <typename T>
__device__ inline void p0_z(bool emit, T (&pA)[16], const T (&cur)[16], T* dst)
{
    if (emit) {
#pragma unroll
        for (int ky = 0; ky < 4; ++ky) {
            T E[4], O[4];
#pragma unroll
            for (int lz = 0; lz < 4; ++lz) {
                E[lz] = pA[ky + 4 * lz] + cur[ky + 4 * lz];
                O[lz] = pA[ky + 4 * lz] - cur[ky + 4 * lz];
            }
#pragma unroll
            for (int kz = 0; kz < 4; ++kz) dst[4 * ky + 16 * kz] = sym<4>(opH3, kz, kz, E, O);
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) pA[i] = cur[i];
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// one 16x16x32 product with BF16 operands, FP32 accumulation (same result layout as the
// FP32 16x16x4 product)
__device__ inline Mfma<float>::vec mac_bf16(bf16x8 a, bf16x8 b, Mfma<float>::vec c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// BF (float only): the matrix-core stages (x-pass, time sums) take BF16 operands
template <typename T, int TY, bool BF>
__global__ void __launch_bounds__(16 * TX * TY)
k_tiled3d_m3(TiledArgs a, int tz, const Tables<T>* __restrict__ tabs)
{
    static_assert(!BF || sizeof(T) == 4, "BF16 operands with FP32 storage only");
    using S = Shared<T, TY>;
    using MF = Mfma<T>;
    constexpr int NT = 16 * TX * TY;
    constexpr int NW = NT / 64;
    constexpr int NC = S::NC, NXL = S::NXL, NNODE = S::NNODE, NEDGE = S::NEDGE;
    extern __shared__ __align__(32) unsigned char smem_raw[];
    S& sh = *reinterpret_cast<S*>(smem_raw);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;

    const int tiles_x = (a.ext_to[0] + TX - 1) / TX;
    const int x0 = (blockIdx.x % tiles_x) * TX;
    const int y0 = (blockIdx.x / tiles_x) * TY;
    const int cz0 = blockIdx.y * tz;
    const int cz1 = min(cz0 + tz, a.ext_to[2]);
    const int off = (a.to_grid == 1) ? 0 : -1; // input node of corner s = cell + off + s

    // BF16 operands: the scalings stay in FP32 arithmetic (SC), see the table builder
    constexpr bool SC = BF;
    const YzScale<T> ysc{T(a.lam2[0] / a.lam2[2]), T(a.lam2[1] / a.lam2[2]), T(a.lam2[0]),
                         T(a.lam2[1]), T(a.lam2[2]), T(a.tau)};
    const T* __restrict__ gu = (const T*)a.u_in;
    const T* __restrict__ gv = (const T*)a.v_in;

    // the padding slot of every cell block reads as zero in the class products
    for (int c = tid; c < NC; c += NT) sh.z[c * ZS + 432] = T(0);
    const T xa0 = tabs->xa[0][lane], xa1 = tabs->xa[1][lane];
    bf16x8 xb, tb[2];
    int kb8[2][8];
    if constexpr (BF) {
        xb = *(const bf16x8*)tabs->xb[lane];
        const int p = wave % 8;
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
            tb[kb] = *(const bf16x8*)tabs->tb[p][kb][lane];
#pragma unroll
            for (int e = 0; e < 8; ++e) kb8[kb][e] = tabs->kb8[p][kb][lane >> 4][e];
        }
    }
    // every wave keeps CPW parity classes for the whole run, holds their operands in
    // registers (no table loads in the loop) and applies each to GPW groups of 16 cells
    static_assert(NW % 8 == 0 || 8 % NW == 0, "waves and parity classes must tile");
    constexpr int CPW = NW >= 8 ? 1 : 8 / NW;
    constexpr int GPW = NW >= 8 ? (NC / 16) / (NW / 8) : NC / 16;
    static_assert(NW < 8 || (NC / 16) % (NW / 8) == 0, "cell groups must tile the waves");
    auto cls_of = [&](int c) { return NW >= 8 ? wave % 8 : wave + c * NW; };
    auto grp_of = [&](int k) { return NW >= 8 ? wave / 8 + k * (NW / 8) : k; };
    // output target of each result row: LDS offset in the staged outputs (u rows relative
    // to the cell's u block, v rows flagged by 1 << 16), -1 for an unused row; in the
    // scaled form (SC) also the output scale 1/S(alpha), times 1/tau for v
    int tkv[CPW][TS_KSTEPS], rdst[CPW][4];
    T tav[CPW][TS_KSTEPS], rsc[CPW][4];
    const T inv_tau = T(1.0 / a.tau);
    const T inv_l2[3] = {T(1.0 / a.lam2[0]), T(1.0 / a.lam2[1]), T(1.0 / a.lam2[2])};
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int p = cls_of(c);
#pragma unroll
        for (int ks = 0; ks < TS_KSTEPS; ++ks) {
            tav[c][ks] = tabs->ta[p][ks][lane];
            tkv[c][ks] = tabs->tk[p][4 * ks + (lane >> 4)];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int info = tabs->tr[p][MF::row(lane, r)];
            const bool isv = info >= 0 && (info & 0x1000);
            rdst[c][r] = info < 0 ? -1 : (isv ? (1 << 16) | (info & 0xff) : (info & 0xff));
            T sc = isv ? inv_tau : T(1);
#pragma unroll
            for (int i = 0; i < 3; ++i)
                if (info >= 0 && (info & (0x100 << i))) sc *= inv_l2[i];
            rsc[c][r] = sc;
        }
    }

    // ---- 1. node layers: fetched into registers one layer ahead, then stashed in
    //         LDS; ghosts mirrored with signs ----
    const long long plane = (long long)a.ext_from[0] * a.ext_from[1];
    constexpr int NUC = (NNODE * 16 + NT - 1) / NT; // u chunks (4 coefficients) per thread
    constexpr int NVE = (NNODE * 27 + NT - 1) / NT; // v coefficients per thread
    T ru[NUC][4], rv[NVE];
    // per-thread load slots: the xy part of the source node and the ghost signs are
    // fixed for the column; only the layer (z) changes
    int us_off[NUC], us_msk[NUC], vs_off[NVE], vs_msk[NVE];
#pragma unroll
    for (int i = 0; i < NUC; ++i) {
        const int e = tid + i * NT;
        us_off[i] = 0;
        us_msk[i] = 0;
        if (e >= NNODE * 16) continue;
        const int node = e >> 4, qq = e & 15;
        const Map1 mx = map_node(x0 + off + node % NXL, a.ext_from[0], a.bc[0]);
        const Map1 my = map_node(y0 + off + node / NXL, a.ext_from[1], a.bc[1]);
        us_off[i] = mx.j + a.ext_from[0] * my.j;
        int m = 1;
#pragma unroll
        for (int lx = 0; lx < 4; ++lx)
            if (mx.ghost && flips(a.bc[0], lx)) m |= 2 << lx;
        if (my.ghost && flips(a.bc[1], qq & 3)) m |= 32;
        us_msk[i] = m;
    }
#pragma unroll
    for (int i = 0; i < NVE; ++i) {
        const int e = tid + i * NT;
        vs_off[i] = 0;
        vs_msk[i] = 0;
        if (e >= NNODE * 27) continue;
        const int node = e / 27, cc = e % 27;
        const Map1 mx = map_node(x0 + off + node % NXL, a.ext_from[0], a.bc[0]);
        const Map1 my = map_node(y0 + off + node / NXL, a.ext_from[1], a.bc[1]);
        vs_off[i] = mx.j + a.ext_from[0] * my.j;
        bool neg = false;
        if (mx.ghost && flips(a.bc[0], cc % 3)) neg = !neg;
        if (my.ghost && flips(a.bc[1], (cc / 3) % 3)) neg = !neg;
        vs_msk[i] = 1 | (neg ? 2 : 0);
    }
    // fetch() only issues the loads (every slot loads, idle slots from node 0) and
    // records the z-ghost state of the layer; the signs are applied in stash(), so
    // the loads stay in flight while the previous layer is being processed.
    int zghost = 0;
    auto fetch = [&](int layer_gz) {
        const Map1 mz = map_node(layer_gz, a.ext_from[2], a.bc[2]);
        const long long zoff = plane * mz.j;
        zghost = mz.ghost;
#pragma unroll
        for (int i = 0; i < NUC; ++i) {
            const int qq = (tid + i * NT) & 15;
            const long long node = (us_msk[i] & 1) ? zoff + us_off[i] : 0;
            const T* src = gu + node * 64 + 4 * qq;
#pragma unroll
            for (int lx = 0; lx < 4; ++lx) ru[i][lx] = src[lx];
        }
#pragma unroll
        for (int i = 0; i < NVE; ++i) {
            const int cc = (tid + i * NT) % 27;
            const long long node = (vs_msk[i] & 1) ? zoff + vs_off[i] : 0;
            rv[i] = gv[node * 27 + cc];
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int i = 0; i < NUC; ++i) {
            const int e = tid + i * NT;
            if (e >= NNODE * 16) break;
            const int qq = e & 15;
            const bool zneg = zghost && flips(a.bc[2], qq >> 2);
            const bool yz = ((us_msk[i] & 32) != 0) != zneg;
            T* dst = sh.nu + (e >> 4) * NUP + 4 * qq;
#pragma unroll
            for (int lx = 0; lx < 4; ++lx) {
                const bool ng = yz != ((us_msk[i] >> (lx + 1)) & 1);
                dst[lx] = ng ? -ru[i][lx] : ru[i][lx];
            }
        }
#pragma unroll
        for (int i = 0; i < NVE; ++i) {
            const int e = tid + i * NT;
            if (e >= NNODE * 27) break;
            const int cc = e % 27;
            const bool ng = ((vs_msk[i] & 2) != 0) != (zghost && flips(a.bc[2], cc / 9));
            sh.nv[(e / 27) * NVP + cc] = ng ? -rv[i] : rv[i];
        }
    };

    // ---- stage-3 task: [R and Q: 6 kx x 2 ky halves | p0: 4 kx] x NC cells ----
    // task ids: 0..5 lower half of the k_y range (k_x = id), 6..11 upper half, 12..15 p0.
    // A wave holds 64 / NC consecutive slots; the order keeps the two halves in different
    // waves (with 4 slots per wave, the last two waves pair two half tasks with two p0
    // tasks, the light path)
    const int slot = tid / NC, cell3 = tid % NC;
    constexpr int kOrder4[16] = {0, 1, 2, 3, 6, 7, 8, 9, 4, 5, 12, 13, 10, 11, 14, 15};
    const int t3 = (64 / NC == 4) ? kOrder4[slot] : slot;
    const bool is_p0 = t3 >= 12;
    const int kx = is_p0 ? t3 - 12 : t3 % 6;
    const bool hi = !is_p0 && t3 >= 6; // upper half of the k_y range (3..5)
    const int ccx = cell3 % TX, ccy = cell3 / TX;
    const int e0 = ccx + TX * ccy, e1 = ccx + TX * (ccy + 1); // x-edges below / above in y
    T pA[16], pB[12], pC[9];                                   // previous layer's y-results

    const int nlayers = cz1 - cz0 + 1;
    T* const ou_base = sh.out;
    T* const ov_base = sh.out + NC * OUS;
    // ---- 5. store a staged cell layer.  Full tiles: one group of 4 coefficients
    //         per thread for u (NT = 16 NC groups); the v outputs of a tile row of
    //         TX = 4 cells are contiguous in memory, TY rows x 27 groups.  Partial
    //         tiles (and v rows whose pitch breaks the group alignment): one value per
    //         thread and step ----
    typedef T vec4 __attribute__((ext_vector_type(4)));
    const bool full_x = x0 + TX <= a.ext_to[0];
    const bool vec_v = full_x && (a.ext_to[0] % 4 == 0);
    const long long plane_to = (long long)a.ext_to[0] * a.ext_to[1];
    const int su_c = tid >> 4, su_q = tid & 15;
    const bool su_ok = y0 + su_c / TX < a.ext_to[1];
    const long long su_g = ((long long)(x0 + su_c % TX) + (long long)a.ext_to[0] * (y0 + su_c / TX)) * 64 + 4 * su_q;
    const int sv_r = tid / 27, sv_q = tid % 27;
    const bool sv_ok = tid < TY * 27 && y0 + sv_r < a.ext_to[1];
    const long long sv_g = ((long long)x0 + (long long)a.ext_to[0] * (y0 + sv_r)) * 27 + 4 * sv_q;
    auto store_layer = [&](int cz) {
        T* __restrict__ out_u = (T*)a.u_out;
        T* __restrict__ out_v = (T*)a.v_out;
        if (full_x) {
            if (su_ok)
                *(vec4*)(out_u + cz * plane_to * 64 + su_g) = *(const vec4*)(ou_base + su_c * OUS + 4 * su_q);
        } else {
            for (int i = tid; i < NC * 64; i += NT) {
                const int c = i >> 6, coef = i & 63;
                const int gx = x0 + c % TX, gy = y0 + c / TX;
                if (gx >= a.ext_to[0] || gy >= a.ext_to[1]) continue;
                out_u[(gx + (long long)a.ext_to[0] * gy + plane_to * cz) * 64 + coef] = ou_base[c * OUS + coef];
            }
        }
        if (vec_v) {
            if (sv_ok)
                *(vec4*)(out_v + cz * plane_to * 27 + sv_g) = *(const vec4*)(ov_base + sv_r * (TX * 27) + 4 * sv_q);
        } else {
            for (int i = tid; i < NC * 27; i += NT) {
                const int c = i / 27, coef = i % 27;
                const int gx = x0 + c % TX, gy = y0 + c / TX;
                if (gx >= a.ext_to[0] || gy >= a.ext_to[1]) continue;
                out_v[(gx + (long long)a.ext_to[0] * gy + plane_to * cz) * 27 + coef] = ov_base[c * 27 + coef];
            }
        }
    };

    // ---- 4. time sums: class blocks on the matrix cores, 16 cells per product.  The
    //         wave's CPW x GPW products run as interleaved independent chains, all B
    //         operands read first.  Lanes 0-31 hold u rows and lanes 32-63 v rows of a
    //         class block: the target and the p0 term are selected per lane, so both
    //         kinds share one instruction stream ----
    using Acc = typename MF::vec;
    using BOp = typename std::conditional<BF, bf16x8, T>::type;
    constexpr int NB = BF ? 2 : TS_KSTEPS; // operand registers per (class, cell group)
    auto ts_load = [&](BOp (&bv)[CPW][GPW][NB]) {
#pragma unroll
        for (int c = 0; c < CPW; ++c)
#pragma unroll
            for (int k = 0; k < GPW; ++k) {
                const T* zc = sh.z + (16 * grp_of(k) + (lane & 15)) * ZS;
                if constexpr (BF) {
#pragma unroll
                    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                        for (int e = 0; e < 8; ++e) bv[c][k][kb][e] = (__bf16)zc[kb8[kb][e]];
                } else {
#pragma unroll
                    for (int ks = 0; ks < TS_KSTEPS; ++ks) bv[c][k][ks] = zc[tkv[c][ks]];
                }
            }
    };
    auto ts_mac = [&](const BOp (&bv)[CPW][GPW][NB], Acc (&acc)[CPW][GPW]) {
#pragma unroll
        for (int c = 0; c < CPW; ++c)
#pragma unroll
            for (int k = 0; k < GPW; ++k) acc[c][k] = Acc{T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int ks = 0; ks < NB; ++ks)
#pragma unroll
            for (int c = 0; c < CPW; ++c)
#pragma unroll
                for (int k = 0; k < GPW; ++k) {
                    if constexpr (BF)
                        acc[c][k] = mac_bf16(tb[ks], bv[c][k][ks], acc[c][k]);
                    else
                        acc[c][k] = MF::mac(tav[c][ks], bv[c][k][ks], acc[c][k]);
                }
    };
    auto ts_out = [&](const Acc (&acc)[CPW][GPW]) {
#pragma unroll
        for (int c = 0; c < CPW; ++c)
#pragma unroll
            for (int k = 0; k < GPW; ++k) {
                const int cell = 16 * grp_of(k) + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    // unused rows write to the padding word 64 of the cell's u block (never
                    // stored), so every lane stores and the epilogue has no branches: its
                    // p0 reads and stores are issued back to back
                    const int dst = rdst[c][r];
                    const bool used = dst >= 0, isv = dst >= (1 << 16);
                    const int ai = used ? (dst & 0xffff) : 64;
                    const T pz = sh.p0[cell * P0S + (isv || !used ? 0 : ai)];
                    const T val = (SC ? rsc[c][r] * acc[c][k][r] : acc[c][k][r]) + (isv ? T(0) : pz);
                    const int o = isv ? NC * OUS + cell * 27 + ai : cell * OUS + ai;
                    ou_base[o] = val;
                }
            }
    };
    // Per node layer: stash it, store the cell layer finished in the previous pass,
    // issue the loads of the next node layer, then the x-, y/z- and time passes.  The
    // stores go out before the loads, so the in-order memory counter that the next
    // stash waits on covers stores issued a whole pass earlier.
    fetch(cz0 + off);
    for (int step = 0; step < nlayers; ++step) {
        stash();
        __syncthreads();
        if (step >= 2) store_layer(cz0 + step - 2);
        if (step + 1 < nlayers) fetch(cz0 + off + step + 1);

        // ---- 2. x-pass: u on the matrix cores (one edge per wave), v on the VALU ----
        if constexpr (BF) {
            // one 16x16x32 product per edge: lanes 0-15 hold the 8 inputs (s, l_x) of
            // line j = lane, the other lanes the zero padding of K
            constexpr int EPW = (NEDGE + NW - 1) / NW;
            bf16x8 bb[EPW];
#pragma unroll
            for (int i = 0; i < EPW; ++i) {
                const int e = wave + i * NW;
#pragma unroll
                for (int q = 0; q < 8; ++q) bb[i][q] = (__bf16)0.0f;
                if (e < NEDGE && lane < 16) {
                    const int n0 = e % TX + NXL * (e / TX);
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        bb[i][q] = (__bf16)sh.nu[(n0 + q / 4) * NUP + (q % 4) + 4 * lane];
                }
            }
#pragma unroll
            for (int i = 0; i < EPW; ++i) {
                const int e = wave + i * NW;
                if (e < NEDGE) {
                    typename MF::vec acc = {T(0), T(0), T(0), T(0)};
                    acc = mac_bf16(xb, bb[i], acc);
                    T* dst = sh.xu + e * XUE + (lane & 15);
#pragma unroll
                    for (int r = 0; r < 4; ++r) dst[MF::row(lane, r) * XUR] = acc[r];
                }
            }
        } else {
            // B[k][j] = input (s, l_x = k) of line j = l_y + 4 l_z: nu[node][l_x + 4 j];
            // the operands of all of the wave's edges are read before the products
            constexpr int EPW = (NEDGE + NW - 1) / NW;
            T b0[EPW], b1[EPW];
#pragma unroll
            for (int i = 0; i < EPW; ++i) {
                const int e = wave + i * NW;
                if (e < NEDGE) {
                    const int n0 = e % TX + NXL * (e / TX);
                    b0[i] = sh.nu[n0 * NUP + (lane >> 4) + 4 * (lane & 15)];
                    b1[i] = sh.nu[(n0 + 1) * NUP + (lane >> 4) + 4 * (lane & 15)];
                }
            }
#pragma unroll
            for (int i = 0; i < EPW; ++i) {
                const int e = wave + i * NW;
                if (e < NEDGE) {
                    typename MF::vec acc = {T(0), T(0), T(0), T(0)};
                    acc = MF::mac(xa0, b0[i], acc);
                    acc = MF::mac(xa1, b1[i], acc);
                    T* dst = sh.xu + e * XUE + (lane & 15);
#pragma unroll
                    for (int r = 0; r < 4; ++r) dst[MF::row(lane, r) * XUR] = acc[r];
                }
            }
        }
        for (int task = tid; task < NEDGE * 9; task += NT) {
            const int e = task % NEDGE, line = task / NEDGE;
            const int cx = e % TX, b = e / TX;
            const int n0 = cx + NXL * b;
            const int ly = line % 3, lz = line / 3;
            T E[3], O[3];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const T a0 = sh.nv[n0 * NVP + l + 3 * ly + 9 * lz];
                const T a1 = sh.nv[(n0 + 1) * NVP + l + 3 * ly + 9 * lz];
                E[l] = a0 + a1;
                O[l] = a0 - a1;
            }
            T* dst = sh.xv + e * XVE + line;
#pragma unroll
            for (int r = 0; r < 6; ++r) dst[r * 9] = sym<3>(opH2, r, r, E, O);
        }
        __syncthreads();

        // ---- 3. y-pass of this layer, z-pass with the previous one ----
        const bool emit = step > 0;
        const T* xu0 = sh.xu + e0 * XUE;
        const T* xu1 = sh.xu + e1 * XUE;
        const T* xv0 = sh.xv + e0 * XVE;
        const T* xv1 = sh.xv + e1 * XVE;
        T cA[16], cB[12], cC[9];
        if (is_p0) {
            p0_y(xu0, xu1, kx, cA);
            p0_z(emit, pA, cA, sh.p0 + cell3 * P0S + kx);
        } else if (!hi) {
            yz_y<0, SC>(xu0, xu1, xv0, xv1, kx, cA, cB, cC, ysc);
            yz_z<0, SC>(emit, kx, pA, pB, pC, cA, cB, cC, sh.z + cell3 * ZS, ysc.l2z);
        } else {
            yz_y<3, SC>(xu0, xu1, xv0, xv1, kx, cA, cB, cC, ysc);
            yz_z<3, SC>(emit, kx, pA, pB, pC, cA, cB, cC, sh.z + cell3 * ZS, ysc.l2z);
        }
        if (!emit) continue; // the first layer only primes the registers
        __syncthreads();

        // ---- 4. time sums of the cell layer just emitted ----
        BOp bv[CPW][GPW][NB];
        Acc acc[CPW][GPW];
        ts_load(bv);
        if constexpr (!BF) __builtin_amdgcn_sched_barrier(0); // FP32/FP64: every operand read before the products
        ts_mac(bv, acc);
        ts_out(acc);
    }
    if (nlayers >= 2) {
        __syncthreads();
        store_layer(cz1 - 1);
    }
}

// ---------------------------------------------------------------------------
// host: constant tables and launch
// ---------------------------------------------------------------------------
double weight(int ax, int ay, int az, int bx, int by, int bz)
{
    return kFact[bx + by + bz] / (kFact[bx] * kFact[by] * kFact[bz]) * kFact[ax + 2 * bx] /
           kFact[ax] * kFact[ay + 2 * by] / kFact[ay] * kFact[az + 2 * bz] / kFact[az];
}

// S(k) = prod_i ((lambda_i/2)^2)^floor(k_i/2)
double scale_s(const int k[3], const double lam2[3])
{
    double s = 1.0;
    for (int i = 0; i < 3; ++i)
        for (int e = 0; e < k[i] / 2; ++e) s *= lam2[i];
    return s;
}

template <typename T>
void build_tables(Tables<T>& t, const double lam2[3], double tau)
{
    std::memset(&t, 0, sizeof t);
    for (int ks = 0; ks < 2; ++ks)
        for (int l = 0; l < 64; ++l) t.xa[ks][l] = (T)opX(l % 16, 4 * ks + l / 16);
    for (int p = 0; p < 8; ++p) {
        const int px = p & 1, py = (p >> 1) & 1, pz = (p >> 2) & 1;
        // rows: 8 u outputs, then the v outputs of the class
        int ra[16][3], nrow = 0;
        bool rv[16];
        for (int o = 0; o < 8; ++o) {
            ra[nrow][0] = px + 2 * (o & 1);
            ra[nrow][1] = py + 2 * ((o >> 1) & 1);
            ra[nrow][2] = pz + 2 * (o >> 2);
            rv[nrow++] = false;
        }
        for (int az = pz; az <= 2; az += 2)
            for (int ay = py; ay <= 2; ay += 2)
                for (int ax = px; ax <= 2; ax += 2) {
                    ra[nrow][0] = ax;
                    ra[nrow][1] = ay;
                    ra[nrow][2] = az;
                    rv[nrow++] = true;
                }
        for (int row = 0; row < 16; ++row) {
            if (row >= nrow) {
                t.tr[p][row] = -1;
                continue;
            }
            const int* al = ra[row];
            const int flat = rv[row] ? al[0] + 3 * al[1] + 9 * al[2] : al[0] + 4 * al[1] + 16 * al[2];
            int mask = 0;
            for (int i = 0; i < 3; ++i)
                if (al[i] >= 2) mask |= 1 << i;
            t.tr[p][row] = (rv[row] ? 0x1000 : 0) | (mask << 8) | flat;
        }
        // inputs kk: 0..26 Q, 27..53 R, 54..55 padding (zero slot)
        // W: weights of the unscaled form (FP32 and FP64 operands); W0: without the
        // scalings, for the BF16 operands, whose rounding of lambda- and tau-dependent
        // weights would perturb the scheme itself (a time-step error that accumulates
        // over the steps), so the BF16 form applies the scalings in FP32 instead
        double W[16][TS_KSTEPS * 4] = {}, W0[16][TS_KSTEPS * 4] = {};
        for (int kk = 0; kk < TS_KSTEPS * 4; ++kk) {
            if (kk >= 54) {
                t.tk[p][kk] = 432;
                continue;
            }
            const bool isr = kk >= 27;
            const int tt = kk % 27;
            const int k[3] = {px + 2 * (tt % 3), py + 2 * ((tt / 3) % 3), pz + 2 * (tt / 9)};
            t.tk[p][kk] = (isr ? 216 : 0) + k[0] + 6 * k[1] + 36 * k[2];
            for (int row = 0; row < nrow; ++row) {
                const int* al = ra[row];
                if (k[0] < al[0] || k[1] < al[1] || k[2] < al[2]) continue;
                const int bx = (k[0] - al[0]) / 2, by = (k[1] - al[1]) / 2, bz = (k[2] - al[2]) / 2;
                const int j = bx + by + bz;
                const double w = weight(al[0], al[1], al[2], bx, by, bz);
                // u: tau Q/(2j+1)!, R/(2j+2)!;  v: Q/(2j)!, R/(2j+1)! / tau.  The inputs
                // arrive unscaled (Q, R / (l_z/2)^2), the outputs as they are stored,
                // so the weight carries S(k) / S(alpha), (l_z/2)^2 for R, tau for Q
                const int fq = rv[row] ? 2 * j : 2 * j + 1;
                const double sc = scale_s(k, lam2) / scale_s(al, lam2) * (isr ? lam2[2] : tau) /
                                  (rv[row] ? tau : 1.0);
                W0[row][kk] = w / kFact[isr ? fq + 1 : fq];
                W[row][kk] = W0[row][kk] * sc;
            }
        }
        for (int ks = 0; ks < TS_KSTEPS; ++ks)
            for (int l = 0; l < 64; ++l) t.ta[p][ks][l] = (T)W[l % 16][4 * ks + l / 16];
        for (int kb = 0; kb < 2; ++kb)
            for (int l = 0; l < 64; ++l)
                for (int e = 0; e < 8; ++e) {
                    const int k = 32 * kb + 8 * (l / 16) + e;
                    t.tb[p][kb][l][e] = to_bf16(k < TS_KSTEPS * 4 ? W0[l % 16][k] : 0.0);
                    if (l < 4 * 16 && l % 16 == 0)
                        t.kb8[p][kb][l / 16][e] = k < TS_KSTEPS * 4 ? t.tk[p][k] : 432;
                }
    }
    for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e) {
            const int k = 8 * (l / 16) + e;
            t.xb[l][e] = to_bf16(k < 8 ? opX(l % 16, k) : 0.0);
        }
}

template <typename T>
hipError_t create_tables(const double lam2[3], double tau, void** out)
{
    Tables<T>* h = new Tables<T>();
    build_tables(*h, lam2, tau);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(Tables<T>));
    if (e == hipSuccess) e = hipMemcpy(p, h, sizeof(Tables<T>), hipMemcpyHostToDevice);
    delete h;
    if (e != hipSuccess) {
        if (p) (void)hipFree(p);
        return e;
    }
    *out = p;
    return hipSuccess;
}

template <typename T, int TY, bool BF = false>
hipError_t launch(const TiledArgs& a, hipStream_t st)
{
    constexpr int NT = 16 * TX * TY;
    const Tables<T>* tabs = static_cast<const Tables<T>*>(a.tables);
    const size_t lds = sizeof(Shared<T, TY>);
    auto kern = k_tiled3d_m3<T, TY, BF>;
    hipError_t e = hw_lds_limit<k_tiled3d_m3<T, TY, BF>>(lds);
    if (e != hipSuccess) return e;
    const int tz = 64;
    const int tiles = ((a.ext_to[0] + TX - 1) / TX) * ((a.ext_to[1] + TY - 1) / TY);
    const int chunks = (a.ext_to[2] + tz - 1) / tz;
    hipLaunchKernelGGL(kern, dim3(tiles, chunks), dim3(NT), lds, st, a, tz, tabs);
    return hipGetLastError();
}

} // namespace

bool hw_tiled_supported(int d, int m, int method, int precision)
{
    return d == 3 && m == 3 && method == 0 && (precision == 0 || precision == 1 || precision == 2);
}

hipError_t hw_tiled_tables_create(int precision, const double lam2[3], double tau, void** out)
{
    *out = nullptr;
    for (int i = 0; i < 3; ++i)
        if (!(lam2[i] >= 2.5e-7)) return hipErrorInvalidValue;
    if (!(tau > 0.0)) return hipErrorInvalidValue;
    return precision == 0 ? create_tables<double>(lam2, tau, out) : create_tables<float>(lam2, tau, out);
}

void hw_tiled_tables_destroy(void* tables)
{
    if (tables) (void)hipFree(tables);
}

hipError_t hw_launch_tiled(const TiledArgs& a, int precision, hipStream_t st)
{
    if (!a.tables) return hipErrorInvalidValue;
    for (int i = 0; i < 3; ++i)
        if (!(a.lam2[i] >= 2.5e-7) || a.ext_to[i] < 1 || a.ext_from[i] < 1) return hipErrorInvalidValue;
    if (precision == 0) return launch<double, 4>(a, st);
    if (precision == 2) return launch<float, 8, true>(a, st);
    return launch<float, 8>(a, st);
}
