// Composed-map half-step kernel for 2-D problems on the matrix cores, nodal degree
// m = 3..6, both methods (dissipative: u and v; conservative, Sec. 4.1: the even time sum
// S of the other grid's u, u_new = 2 S - u_old), element type T = float or double.
//
// The half step of a cell is a linear map of its 4 corner nodes (NI = n_u [+ n_v]
// coefficients each) to its output node, composed on the host (cellmap.cpp).  By the
// reflection symmetry of the Hermite operators about the cell centre (kept by the time
// sums), corner s = (s_x, s_y) enters output a with (-1)^(sum_i s_i (a_i + l_i)) times
// corner 0's entry, so the corners are combined into the four sums
// S_p[l] = sum_s (-1)^(p . s) x_s[l] (p = p_x + 2 p_y), and output a needs, for each input
// l, only S_{pi(a) xor pi(l)}[l] (pi: the parity vector).  Grouped by the output parity
// class q = pi(a), each class is a dense (rows of the class) x NI product with the
// class's column of selected sums; its rows are cut into tiles of 16 ("chains", one or
// two per class), each applied to 16 cells at a time as a chain of 16x16x4 products.
//
// A workgroup of 8 waves owns a strip of 16 cells along x and walks a chunk of its cell
// rows upwards in y, one node row of the input grid at a time; wave 2 q + h runs every
// chain of class q over half h of the K range (the two halves' partial outputs are added
// when the row is stored, so that the waves of a class share their B operands and the
// chains are half as long):
//   1. the row's 17 nodes, loaded into registers during the previous row, are stashed in
//      LDS (ghost nodes outside non-periodic walls mirrored with the odd / even signs of
//      Sec. 3.1.3); the cell row finished two rows ago is stored and the loads of the
//      next node row are issued (loads and stores through buffer resources built per row
//      from its wave-uniform base, each lane adding a 32-bit offset fixed per strip);
//   2. butterflies: per cell and input l, T_px[l] = x(left)[l] +- x(right)[l] of this
//      row, combined with those of the row below (kept in registers since the previous
//      pass) into S_{px + 2 py}[l] = T_px(lower)[l] +- T_px(upper)[l], written to LDS in
//      class order: the cell's block holds, for class q and K position k, the sum that
//      class selects for input l_k, S_{q xor pi(l_k)}[l_k], so that a wave's B operands
//      are read at affine offsets;
//   3. the chains' products (A: the chains' rows of the composed map, registers; B: the
//      selected sums read from LDS), partial outputs staged in LDS for the coalesced
//      stores.
// LDS strides follow the 32 banks of 4 bytes served 32 lanes (b32) or 16 lanes (b64) at a
// time: node stride = 2 (mod 32) in FP32 (the 16 cells of a butterfly pass on the 16 even
// banks, the pass's second K position -- whose input index has the other parity -- on the
// odd ones), 1 (mod 16) in FP64; sums' cell stride = 2 (mod 32) in FP32, odd in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "buffer_io.h"
#include "hw_kernels.h"

namespace {

constexpr int CX = 16;      // cells of a strip
constexpr int NXN = CX + 1; // nodes of a row of a strip
constexpr int NT2 = 512;    // threads of a workgroup: 4 classes x 2 K halves

// smallest v >= x with v = r (mod m)
constexpr int up_to_residue(int x, int m, int r) { return x + ((r - x % m) % m + m) % m; }

template <typename T, int MU, bool CONS>
struct Shape2 {
    static constexpr int MV = CONS ? 0 : MU - 1;
    static constexpr int NU = MU * MU, NV = MV * MV, NI = NU + NV; // inputs = outputs per node
    static constexpr int TL = (NI + 3) / 4 * 4;                    // K positions (padded)
    static constexpr int KS = TL / 4;                              // K-steps of 4
    static constexpr int KH = (KS + 1) / 2;                        // K-steps of the first half
    static constexpr bool PAD = TL > NI;                           // padding reads slot NI or NI+1 (zero)
    static constexpr int SX0 = NI + (PAD ? 2 : 0);                 // minimum node stride
    static constexpr int SX = sizeof(T) == 4 ? up_to_residue(SX0, 32, 2) : up_to_residue(SX0, 16, 1);
    static constexpr int TSZ0 = 4 * TL;
    static constexpr int TSZ = sizeof(T) == 4 ? up_to_residue(TSZ0, 32, 2) : (TSZ0 | 1);
    static constexpr int OS = (NI + 1) | 1; // cell stride of the staged outputs (slot NI: unused rows)
    // rows of the largest parity class (u: ceil(MU/2)^2, v: ceil(MV/2)^2): one or two chains
    static constexpr int RMAX = ((MU + 1) / 2) * ((MU + 1) / 2) + ((MV + 1) / 2) * ((MV + 1) / 2);
    static constexpr int CPC = (RMAX + 15) / 16; // chains per class at most
    static_assert(CPC <= 2, "at most two chains per class");
    static_assert(SX >= SX0 && TSZ >= TSZ0 && OS > NI, "strides");
    static_assert(TL < 256 && NI + 2 < 256, "packed butterfly slots");
    static_assert(sizeof(T) == 8 || (SX % 32 == 2 && TSZ % 32 == 2), "FP32 strides");
    static_assert(sizeof(T) == 4 || (SX % 16 == 1 && TSZ % 2 == 1), "FP64 strides");
};

template <typename T>
struct Mf2;
template <>
struct Mf2<float> {
    typedef float vec __attribute__((ext_vector_type(4)));
    static __device__ inline vec mac(float a, float b, vec c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __host__ __device__ inline int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct Mf2<double> {
    typedef double vec __attribute__((ext_vector_type(4)));
    static __device__ inline vec mac(double a, double b, vec c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __host__ __device__ inline int row(int l, int r) { return (l >> 4) + 4 * r; }
};

// Tables of one problem:
//   ta[q][c][KS][64] A operand of chain c of class q: entry (row i = lane % 16 of the
//                    chain's tile, K position 4 ks + lane / 16)
//   tr[q][c][16]     output of the chain's row (index into the node's u | v block), -1 unused
//   ncl[q]           chains of class q (1 or 2)
//   kl[TL]           input at K position k (padding positions: the zero slots NI, NI + 1,
//                    whichever index parity keeps the butterfly pairs below complete)
//   pk[TL]           parity vector pi of that input (0 for the padding positions)
//   bk[TL]           K positions of the butterfly passes, pairs (even, odd) whose inputs
//                    have indices of opposite parity
template <typename T, int MU, bool CONS>
struct C2Tables {
    using S = Shape2<T, MU, CONS>;
    T ta[4][S::CPC][S::KS][64];
    int tr[4][S::CPC][16];
    int ncl[4];
    int kl[S::TL];
    int pk[S::TL];
    int bk[S::TL];
};

template <typename T, int MU, bool CONS>
struct C2Shared {
    using S = Shape2<T, MU, CONS>;
    alignas(16) T tsum[CX * S::TSZ];
    alignas(16) T out[2][CX * S::OS]; // partial outputs of the two K halves
    T nd[NXN * S::SX];
};

struct Map1 {
    int j, ghost;
};

// node gi of a grid of ext nodes along a direction with wall type bc (0 periodic: wrapped,
// gi in [-ext, 2 ext) -- the rows a strip reads lie in [-1, ext]; else clamped to the wall
// node, a ghost image)
__device__ inline Map1 map_node(int gi, int ext, int bc)
{
    Map1 m;
    m.ghost = 0;
    if (bc == 0) {
        m.j = gi < 0 ? gi + ext : (gi >= ext ? gi - ext : gi);
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

// sign of coefficient l of a node mirrored across a wall of type bc (1: Dirichlet, odd
// extension: (-1)^(l+1); 2: Neumann, even extension: (-1)^l)
__host__ __device__ inline bool flips(int bc, int l) { return (bc == 1) ? ((l & 1) == 0) : ((l & 1) == 1); }

// (l_x, l_y) of input c of a node (u block: MU x MU, then v block: MV x MV)
template <int MU>
__host__ __device__ inline void coef2(int c, int& lx, int& ly)
{
    if (c < MU * MU) {
        lx = c % MU;
        ly = c / MU;
    } else {
        const int v = c - MU * MU;
        lx = v % (MU - 1);
        ly = v / (MU - 1);
    }
}

// One strip of 16 cells (x0 .. x0 + 15) over cell rows cy0 .. cy1 - 1 of problem a.
template <typename T, int MU, bool CONS, int NT>
__device__ void strip(const DenseArgs& a, const C2Tables<T, MU, CONS>* __restrict__ tabs, int x0, int cy0, int cy1,
                      unsigned char* smem_raw)
{
    using S = Shape2<T, MU, CONS>;
    using SH = C2Shared<T, MU, CONS>;
    using MF = Mf2<T>;
    constexpr int NI = S::NI, NU = S::NU, NV = S::NV, KS = S::KS, KH = S::KH, TL = S::TL, CPC = S::CPC;
    constexpr int SX = S::SX, TSZ = S::TSZ, OS = S::OS;
    constexpr int UE = (NXN * NU + 63) / 64 * 64; // u elements of a row, padded to whole waves
    constexpr int NVD = NV > 0 ? NV : 1;          // (divisor; no v records in the conservative method)
    constexpr int NE = UE + NXN * NV;
    constexpr int NLOAD = (NE + NT - 1) / NT;
    constexpr int NBF = (CX * TL + NT - 1) / NT;
    SH& sh = *reinterpret_cast<SH*>(smem_raw);
    static_assert(NT == NT2, "one wave per (class, K half)");
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int off = a.to_grid == 1 ? 0 : -1; // input node of corner s = cell + off + s
    typedef const __attribute__((address_space(1))) T* GIn;
    typedef __attribute__((address_space(1))) T* GOut;
    const GIn gu = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.u_in));
    const GIn gv = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.v_in));

    // the zero slots NI, NI + 1 of every node (padding inputs); never written by the stash
    if constexpr (S::PAD)
        for (int i = tid; i < 2 * NXN; i += NT) sh.nd[(i >> 1) * SX + NI + (i & 1)] = T(0);

    // the wave's class q and K half h: A operands of the class's chains over that half
    // (K-steps h KH ..), output targets
    const int q = wave >> 1, h = wave & 1;
    const int two = CPC > 1 ? tabs->ncl[q] > 1 : 0;
    T ta[CPC][KH];
    int rdst[CPC][2]; // output slots of rows r and r + 2 packed as r | r + 2 << 16
#pragma unroll
    for (int c = 0; c < CPC; ++c) {
#pragma unroll
        for (int j = 0; j < KH; ++j) {
            const int ks = h * KH + j;
            ta[c][j] = ks < KS ? tabs->ta[q][c][ks][lane] : T(0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = tabs->tr[q][c][MF::row(lane, r)];
            // unused rows write the spare slot NI of the cell
            const int slot = o < 0 ? NI : o;
            if (r < 2) rdst[c][r] = slot;
            else rdst[c][r - 2] |= slot << 16;
        }
    }

    // node loads: slot i = element tid + i NT of the row's block of the 17 u records,
    // padded to whole waves, followed by the 17 v records, so that every wave's slot reads
    // one array through a buffer resource made per row from its wave-uniform base; the byte
    // offset within the row, the x ghost sign and the LDS slot are fixed per strip (x
    // positions past the periodic wrap of a narrow grid are mapped with the modulo)
    const int ex0 = a.ext_from[0], ex1 = a.ext_from[1];
    uint32_t ld_off[NLOAD];
    int ld_msk[NLOAD]; // -1: idle; bit 1: negate (x ghost), bit 3: l_y odd, bits 4..: LDS slot
    // node rows in flight: PD ahead of the row being stashed (two ahead, with the registers
    // to hold them, measured no faster)
    constexpr int PD = 1;
    T rl[PD][NLOAD];
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
        const int e = tid + i * NT;
        ld_off[i] = 0;
        ld_msk[i] = -1; // idle slot: reads the row's first element, never stashed
        int node, c;
        if (e < NXN * NU) {
            node = e / NU;
            c = e % NU;
        } else if (e >= UE && e < NE) {
            node = (e - UE) / NVD;
            c = NU + (e - UE) % NVD;
        } else {
            continue;
        }
        int lx, ly;
        coef2<MU>(c, lx, ly);
        int gx = x0 + off + node;
        if (a.bc[0] == 0) gx = ((gx % ex0) + ex0) % ex0;
        const Map1 mx = map_node(gx, ex0, a.bc[0]);
        ld_off[i] = (uint32_t)((c < NU ? (int64_t)mx.j * NU + c : (int64_t)mx.j * NV + (c - NU)) * (int64_t)sizeof(T));
        const bool neg = mx.ghost && flips(a.bc[0], lx);
        ld_msk[i] = (neg ? 2 : 0) | ((ly & 1) << 3) | ((node * SX + c) << 4);
    }
    const uint32_t ubytes = (uint32_t)((int64_t)ex0 * NU * sizeof(T)), vbytes = (uint32_t)((int64_t)ex0 * NV * sizeof(T));
    int yghost[PD] = {};
    auto fetch = [&](auto B, int gy) {
        const Map1 my = map_node(gy, ex1, a.bc[1]);
        yghost[B] = my.ghost;
        const int64_t rn = (int64_t)ex0 * my.j;
        const __amdgpu_buffer_rsrc_t ru = make_rsrc((const void*)(gu + rn * NU), ubytes);
        const __amdgpu_buffer_rsrc_t rv = CONS ? ru : make_rsrc((const void*)(gv + rn * NV), vbytes);
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) {
            const bool isu = CONS || i * NT + 64 * wave < UE; // wave-uniform
            rl[B][i] = BufIO<T>::load(isu ? ru : rv, ld_off[i]);
        }
    };
    auto stash = [&](auto B) {
        // the y flip of a ghost row: Dirichlet flips even l_y, Neumann odd l_y
        const bool yflip_odd = a.bc[1] != 1;
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) {
            const int m = ld_msk[i];
            if (m < 0) continue;
            bool neg = (m & 2) != 0;
            if (yghost[B] && (((m >> 3) & 1) != 0) == yflip_odd) neg = !neg;
            sh.nd[m >> 4] = neg ? -rl[B][i] : rl[B][i];
        }
    };

    // staged outputs of a cell row, stored coalesced (a strip's row of cells is contiguous)
    const int nrows = cy1 - cy0 + 1; // node rows
    // output slots: element tid + k NT of the strip's 16 u (v) records, its byte offset
    // within the output row fixed per strip; bit k (16 + k) of s_ok: the u (v) slot has an
    // output inside the grid
    constexpr int NSU = (CX * NU + NT - 1) / NT, NSV = CONS ? 1 : (CX * NV + NT - 1) / NT;
    // (the FP64 dissipative m = 6 kernel, short of registers, recomputes them per row)
    constexpr bool LEAN = sizeof(T) == 8 && !CONS && MU == 7;
    constexpr int NSUK = LEAN ? 1 : NSU, NSVK = LEAN ? 1 : NSV;
    uint32_t su_keep[NSUK], sv_keep[NSVK];
    int s_keep = 0;
    auto slot_u = [&](int k, bool& ok) {
        const int i = tid + k * NT, c = i / NU, o = i % NU;
        ok = i < CX * NU && x0 + c < a.ext_to[0];
        return (uint32_t)(((int64_t)(x0 + c) * NU + o) * (int64_t)sizeof(T));
    };
    auto slot_v = [&](int k, bool& ok) {
        const int i = tid + k * NT, c = i / NVD, o = i % NVD;
        ok = !CONS && i < CX * NV && x0 + c < a.ext_to[0];
        return (uint32_t)(((int64_t)(x0 + c) * NV + o) * (int64_t)sizeof(T));
    };
    if constexpr (!LEAN) {
#pragma unroll
        for (int k = 0; k < NSU; ++k) {
            bool ok;
            su_keep[k] = slot_u(k, ok);
            if (ok) s_keep |= 1 << k;
        }
#pragma unroll
        for (int k = 0; k < NSV; ++k) {
            bool ok;
            sv_keep[k] = slot_v(k, ok);
            if (ok) s_keep |= 1 << (16 + k);
        }
    }
    // byte offset of u (v) output slot k within the row; whether it has an output
    auto su_off = [&](int k, bool& ok) {
        if constexpr (LEAN) return slot_u(k, ok);
        ok = (s_keep >> k) & 1;
        return su_keep[k];
    };
    auto sv_off = [&](int k, bool& ok) {
        if constexpr (LEAN) return slot_v(k, ok);
        ok = (s_keep >> (16 + k)) & 1;
        return sv_keep[k];
    };
    const uint32_t uobytes = (uint32_t)((int64_t)a.ext_to[0] * NU * sizeof(T));
    const uint32_t vobytes = (uint32_t)((int64_t)a.ext_to[0] * NV * sizeof(T));
    T ov[CONS ? NSU : 1];
    auto old_fetch = [&](int cy) {
        if constexpr (CONS) {
            const GIn old_u = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.u_old)) + (int64_t)a.ext_to[0] * cy * NU;
            const __amdgpu_buffer_rsrc_t r = make_rsrc((const void*)old_u, uobytes);
#pragma unroll
            for (int k = 0; k < NSU; ++k) {
                bool ok;
                const uint32_t o = su_off(k, ok);
                if (ok) ov[k] = BufIO<T>::load(r, o);
            }
        }
    };
    auto store_row = [&](int cy) {
        const GOut out_u = reinterpret_cast<GOut>(reinterpret_cast<uintptr_t>(a.u_out)) + (int64_t)a.ext_to[0] * cy * NU;
        const __amdgpu_buffer_rsrc_t ru = make_rsrc((const void*)out_u, uobytes);
#pragma unroll
        for (int k = 0; k < NSU; ++k) {
            bool ok;
            const uint32_t o = su_off(k, ok);
            if (!ok) continue;
            const int i = tid + k * NT, li = (i / NU) * OS + i % NU;
            const T s2 = sh.out[0][li] + sh.out[1][li];
            // conservative: u_new = 2 S - u_old, the old values loaded one pass earlier
            if constexpr (CONS) BufIO<T>::store(T(2) * s2 - ov[k], ru, o);
            else BufIO<T>::store(s2, ru, o);
        }
        if constexpr (!CONS) {
            const GOut out_v = reinterpret_cast<GOut>(reinterpret_cast<uintptr_t>(a.v_out)) + (int64_t)a.ext_to[0] * cy * NV;
            const __amdgpu_buffer_rsrc_t rv = make_rsrc((const void*)out_v, vobytes);
#pragma unroll
            for (int k = 0; k < NSV; ++k) {
                bool ok;
                const uint32_t o = sv_off(k, ok);
                if (!ok) continue;
                const int i = tid + k * NT, li = (i / NVD) * OS + NU + i % NVD;
                BufIO<T>::store(sh.out[0][li] + sh.out[1][li], rv, o);
            }
        }
    };

    // butterfly slots: 32 lanes cover 16 cells x a pair of K positions; a thread keeps the
    // same (cell, kp) slots in every pass
    // slot k: K position kp, its input l and parity vector pl, packed kp | l << 8 | pl << 16
    T prev[NBF][2];
    int bslot[NBF];
#pragma unroll
    for (int k = 0; k < NBF; ++k) {
        const int t = tid + k * NT;
        const int kp = t < CX * TL ? tabs->bk[2 * (t >> 5) + ((t >> 4) & 1)] : 0;
        bslot[k] = kp | tabs->kl[kp] << 8 | tabs->pk[kp] << 16;
    }

    // one pass per node row `step`, held in register buffer B (the buffers alternate; the
    // row PD ahead is loaded into B once it has been stashed)
    auto pass = [&](auto B, int step) {
        stash(B);
        __syncthreads();
        // (the stores go out before the next row's loads: issuing the loads first, even
        // before the barrier, measured slower)
        if (step >= 2) store_row(cy0 + step - 2);
        if (step + PD < nrows) fetch(B, cy0 + off + step + PD);
        if (step >= 1) old_fetch(cy0 + step - 1); // the cell row computed in this pass

        // butterflies of node row `step`: T_px of this row, combined with the lower row's
        // into S_{px + 2 py} of cell row step - 1
#pragma unroll
        for (int k = 0; k < NBF; ++k) {
            const int t = tid + k * NT;
            if (t >= CX * TL) break;
            const int cell = t & 15, kp = bslot[k] & 255, l = (bslot[k] >> 8) & 255, pl = bslot[k] >> 16;
            const T xl = sh.nd[cell * SX + l], xr = sh.nd[(cell + 1) * SX + l];
            const T cur[2] = {xl + xr, xl - xr};
            if (step > 0) {
                // S_p goes to the block of class q = p xor pi(l)
                T* dst = sh.tsum + cell * TSZ + kp;
                dst[pl * TL] = prev[k][0] + cur[0];
                dst[(pl ^ 1) * TL] = prev[k][1] + cur[1];
                dst[(pl ^ 2) * TL] = prev[k][0] - cur[0];
                dst[(pl ^ 3) * TL] = prev[k][1] - cur[1];
            }
            prev[k][0] = cur[0];
            prev[k][1] = cur[1];
        }
        __syncthreads();
        if (step == 0) return;

        // (the products run at a raised wave priority: the product chains of one
        // workgroup go ahead of the other workgroups' vector and LDS work on the SIMD;
        // about 1% on the batch, where raising the butterflies instead, as the 3-D kernel
        // does, measured nothing)
        __builtin_amdgcn_s_setprio(1);
        // the class's products for cell row step - 1 over this wave's K half, partial
        // outputs staged for the next pass
        const int cell = lane & 15;
        const T* bsrc = sh.tsum + cell * TSZ + q * TL + 4 * h * KH + (lane >> 4);
        T* odst = sh.out[h] + cell * OS;
        // (with KS odd the second half has one K-step fewer: h and the bound are uniform).
        // Where registers are short (FP64, two chains of 22 K-steps) the B operands are read
        // in chunks of 2 K-steps, the next chunk's reads issued before the current chunk's
        // products; the empty asm keeps the reads from being hoisted further.
        constexpr int BC = (sizeof(T) == 8 && KH > 8) ? 2 : KH, NCH = (KH + BC - 1) / BC;
        T bv[KH];
        auto bload = [&](int c) {
#pragma unroll
            for (int j = c * BC; j < (c + 1) * BC && j < KH; ++j)
                if (h * KH + j < KS) bv[j] = bsrc[4 * j];
        };
        typename MF::vec acc0 = {T(0), T(0), T(0), T(0)};
        bload(0);
        if (CPC > 1 && two) {
            typename MF::vec acc1 = {T(0), T(0), T(0), T(0)};
#pragma unroll
            for (int c = 0; c < NCH; ++c) {
                if constexpr (NCH > 1) {
                    if (c + 1 < NCH) bload(c + 1);
                    asm volatile("" ::: "memory");
                }
#pragma unroll
                for (int j = c * BC; j < (c + 1) * BC && j < KH; ++j) {
                    if (h * KH + j < KS) {
                        acc0 = MF::mac(ta[0][j], bv[j], acc0);
                        acc1 = MF::mac(ta[CPC - 1][j], bv[j], acc1);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) odst[(rdst[CPC - 1][r & 1] >> (16 * (r >> 1))) & 0xffff] = acc1[r];
        } else {
#pragma unroll
            for (int c = 1; c < NCH; ++c) bload(c);
#pragma unroll
            for (int j = 0; j < KH; ++j)
                if (h * KH + j < KS) acc0 = MF::mac(ta[0][j], bv[j], acc0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) odst[(rdst[0][r & 1] >> (16 * (r >> 1))) & 0xffff] = acc0[r];
        __builtin_amdgcn_s_setprio(0);
    };
    fetch(std::integral_constant<int, 0>{}, cy0 + off);
    if constexpr (PD == 2) {
        fetch(std::integral_constant<int, PD - 1>{}, cy0 + off + 1); // nrows >= 2
        for (int step = 0; step < nrows; step += 2) {
            pass(std::integral_constant<int, 0>{}, step);
            if (step + 1 < nrows) pass(std::integral_constant<int, PD - 1>{}, step + 1);
        }
    } else {
        for (int step = 0; step < nrows; ++step) pass(std::integral_constant<int, 0>{}, step);
    }
    __syncthreads();
    store_row(cy0 + nrows - 2);
}

// (at least 4 waves per SIMD: two workgroups of 8 waves per CU)
template <typename T, int MU, bool CONS, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_cmap2d(DenseArgs a, int ry)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int x0 = blockIdx.x * CX, cy0 = blockIdx.y * ry, cy1 = min(cy0 + ry, a.ext_to[1]);
    strip<T, MU, CONS, NT>(a, static_cast<const C2Tables<T, MU, CONS>*>(a.cm2), x0, cy0, cy1, smem_raw);
}

// many problems of one (m, method): one workgroup per item of a work list of strips
// {problem, x0, cy0, cy1} (a persistent loop over items costs registers: the loop-invariant
// values of a strip are then held across items); workgroup b runs on XCD b mod 8, and the
// workgroups of one XCD take a contiguous part of the list (neighbouring strips share
// their edge nodes in that XCD's L2)
template <typename T, int MU, bool CONS, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) k_cmap2d_list(const DenseArgs* __restrict__ probs, const int4* __restrict__ items,
                                                    int n_items)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = blockIdx.x;
    const int per_xcd = (n_items + 7) / 8;
    const int t = (b % 8) * per_xcd + b / 8;
    if (t >= n_items) return; // whole workgroup
    const int4 it = items[t];
    const int pi = __builtin_amdgcn_readfirstlane(it.x), x0 = __builtin_amdgcn_readfirstlane(it.y);
    const int cy0 = __builtin_amdgcn_readfirstlane(it.z), cy1 = __builtin_amdgcn_readfirstlane(it.w);
    const DenseArgs a = probs[pi];
    strip<T, MU, CONS, NT>(a, static_cast<const C2Tables<T, MU, CONS>*>(a.cm2), x0, cy0, cy1, smem_raw);
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
template <typename T, int MU, bool CONS>
hipError_t create(const std::vector<double>& G0, void** out)
{
    using S = Shape2<T, MU, CONS>;
    using Tab = C2Tables<T, MU, CONS>;
    constexpr int NI = S::NI, NU = S::NU, KS = S::KS, TL = S::TL, MV = S::MV;
    if (G0.size() != (size_t)NI * NI) return hipErrorInvalidValue;
    Tab* h = new Tab();
    std::memset(h, 0, sizeof *h);
    // K order: the natural input order, padding positions last.  The butterfly passes pair
    // an even K position with an odd one whose inputs have indices of opposite parity (their
    // LDS reads and writes then fall on the even and the odd banks); the padding positions
    // read the zero slot NI or NI + 1, chosen to keep the four (position, input) parity
    // classes balanced so that every position finds its partner.
    {
        int cnt[4] = {0, 0, 0, 0}; // [2 * position parity + input parity]
        for (int k = 0; k < NI; ++k) {
            h->kl[k] = k;
            ++cnt[2 * (k & 1) + (k & 1)];
        }
        for (int k = NI; k < TL; ++k) {
            const int pk = k & 1;
            // even position: (0, even input) pairs with (1, odd), (0, odd) with (1, even)
            const int want_in = pk == 0 ? (cnt[0] < cnt[3] ? 0 : 1) : (cnt[3] < cnt[0] ? 1 : 0);
            h->kl[k] = (NI & 1) == want_in ? NI : NI + 1;
            ++cnt[2 * pk + want_in];
        }
        std::vector<int> cls[4]; // [position parity][input parity]
        for (int k = 0; k < TL; ++k) cls[2 * (k & 1) + (h->kl[k] & 1)].push_back(k);
        // complete pairs first, then whatever remains (correct either way, only slower)
        std::vector<int> ev, od;
        int j = 0;
        const size_t n03 = std::min(cls[0].size(), cls[3].size()), n12 = std::min(cls[1].size(), cls[2].size());
        for (size_t i = 0; i < n03; ++i, ++j) {
            h->bk[2 * j] = cls[0][i];
            h->bk[2 * j + 1] = cls[3][i];
        }
        for (size_t i = 0; i < n12; ++i, ++j) {
            h->bk[2 * j] = cls[1][i];
            h->bk[2 * j + 1] = cls[2][i];
        }
        for (size_t i = n03; i < cls[0].size(); ++i) ev.push_back(cls[0][i]);
        for (size_t i = n12; i < cls[1].size(); ++i) ev.push_back(cls[1][i]);
        for (size_t i = n12; i < cls[2].size(); ++i) od.push_back(cls[2][i]);
        for (size_t i = n03; i < cls[3].size(); ++i) od.push_back(cls[3][i]);
        for (size_t i = 0; i < ev.size(); ++i, ++j) {
            h->bk[2 * j] = ev[i];
            h->bk[2 * j + 1] = od[i];
        }
        if (2 * j != TL) {
            delete h;
            return hipErrorInvalidValue;
        }
    }
    for (int k = 0; k < TL; ++k) {
        const int l = h->kl[k];
        int lx = 0, ly = 0;
        if (l < NI) coef2<MU>(l, lx, ly);
        h->pk[k] = l < NI ? (lx & 1) + 2 * (ly & 1) : 0;
    }
    for (int q = 0; q < 4; ++q) {
        const int qx = q & 1, qy = q >> 1;
        std::vector<int> rows; // outputs of the class: u block, then v block
        for (int ay = qy; ay < MU; ay += 2)
            for (int ax = qx; ax < MU; ax += 2) rows.push_back(ax + MU * ay);
        if (!CONS)
            for (int ay = qy; ay < MV; ay += 2)
                for (int ax = qx; ax < MV; ax += 2) rows.push_back(NU + ax + MV * ay);
        const int ncl = (int)(rows.size() + 15) / 16;
        if (ncl < 1 || ncl > S::CPC) {
            delete h;
            return hipErrorInvalidValue;
        }
        h->ncl[q] = ncl;
        for (int c = 0; c < S::CPC; ++c) {
            const int r0 = 16 * c, nr = std::max(0, std::min(16, (int)rows.size() - r0));
            for (int i = 0; i < 16; ++i) h->tr[q][c][i] = i < nr ? rows[r0 + i] : -1;
            // the selected sum of input l for class q sits at K position k of the class's
            // block (the butterflies write S_{q xor pi(l)} there), so A holds G0 itself
            for (int ks = 0; ks < KS; ++ks)
                for (int lanei = 0; lanei < 64; ++lanei) {
                    const int i = lanei & 15, k = 4 * ks + (lanei >> 4), l = h->kl[k];
                    h->ta[q][c][ks][lanei] = (i < nr && l < NI) ? (T)G0[(size_t)l * NI + rows[r0 + i]] : T(0);
                }
        }
    }

    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(Tab));
    if (e == hipSuccess) e = hipMemcpy(p, h, sizeof(Tab), hipMemcpyHostToDevice);
    delete h;
    if (e != hipSuccess) {
        if (p) (void)hipFree(p);
        return e;
    }
    *out = p;
    return hipSuccess;
}

template <typename T, int MU, bool CONS>
hipError_t launch1(const DenseArgs& a, int ry, hipStream_t st)
{
    constexpr int NT = NT2;
    const size_t lds = sizeof(C2Shared<T, MU, CONS>);
    auto kern = k_cmap2d<T, MU, CONS, NT>;
    hipError_t e = hw_lds_limit<k_cmap2d<T, MU, CONS, NT>>(lds);
    if (e != hipSuccess) return e;
    const dim3 grid((a.ext_to[0] + CX - 1) / CX, (a.ext_to[1] + ry - 1) / ry);
    hipLaunchKernelGGL(kern, grid, dim3(NT), lds, st, a, ry);
    return hipGetLastError();
}

template <typename T, int MU, bool CONS>
hipError_t launch_list(const DenseArgs* probs, const int4* items, int n_items, hipStream_t st)
{
    constexpr int NT = NT2;
    const size_t lds = sizeof(C2Shared<T, MU, CONS>);
    auto kern = k_cmap2d_list<T, MU, CONS, NT>;
    hipError_t e = hw_lds_limit<k_cmap2d_list<T, MU, CONS, NT>>(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(8 * ((n_items + 7) / 8)), dim3(NT), lds, st, probs, items, n_items);
    return hipGetLastError();
}

template <typename T, bool CONS, typename F>
hipError_t by_m(int m, F f)
{
    switch (m) {
    case 3: return f(std::integral_constant<int, 4>{});
    case 4: return f(std::integral_constant<int, 5>{});
    case 5: return f(std::integral_constant<int, 6>{});
    case 6: return f(std::integral_constant<int, 7>{});
    }
    return hipErrorInvalidValue;
}

} // namespace

bool hw_cmap2d_supported(int m) { return m >= 3 && m <= 6; }

bool hw_cmap2d_rows_fit(int m, bool cons, bool fp64, int64_t ext)
{
    const int64_t nu = (int64_t)(m + 1) * (m + 1);
    (void)cons; // the u records are the larger ones in both methods
    return ext >= 0 && ext * nu * (fp64 ? 8 : 4) < ((int64_t)1 << 32);
}

hipError_t hw_cmap2d_tables_create(const std::vector<double>& G0, int m, bool cons, bool fp64, void** out)
{
    *out = nullptr;
    if (!hw_cmap2d_supported(m)) return hipErrorInvalidValue;
    auto mk = [&](auto T_tag, auto c_tag) {
        using T = decltype(T_tag);
        constexpr bool C = decltype(c_tag)::value;
        return by_m<T, C>(m, [&](auto mu) { return create<T, decltype(mu)::value, C>(G0, out); });
    };
    if (fp64)
        return cons ? mk(double(), std::true_type{}) : mk(double(), std::false_type{});
    return cons ? mk(float(), std::true_type{}) : mk(float(), std::false_type{});
}

hipError_t hw_launch_cmap2d(const DenseArgs& a, int m, bool cons, bool fp64, int ry, hipStream_t st)
{
    if (!a.cm2 || ry < 1) return hipErrorInvalidValue;
    if (!hw_cmap2d_rows_fit(m, cons, fp64, std::max(a.ext_from[0], a.ext_to[0]))) return hipErrorInvalidValue;
    if (a.ext_to[0] < 1 || a.ext_to[1] < 1 || a.ext_from[0] < 1 || a.ext_from[1] < 1) return hipErrorInvalidValue;
    auto go = [&](auto T_tag, auto c_tag) {
        using T = decltype(T_tag);
        constexpr bool C = decltype(c_tag)::value;
        return by_m<T, C>(m, [&](auto mu) { return launch1<T, decltype(mu)::value, C>(a, ry, st); });
    };
    if (fp64) return cons ? go(double(), std::true_type{}) : go(double(), std::false_type{});
    return cons ? go(float(), std::true_type{}) : go(float(), std::false_type{});
}

hipError_t hw_launch_cmap2d_list(const DenseArgs* probs, const int4* items, int n_items, int m, bool cons, bool fp64,
                                 hipStream_t st)
{
    if (n_items <= 0) return hipSuccess;
    if (n_items > INT32_MAX - 7) return hipErrorInvalidValue;
    auto go = [&](auto T_tag, auto c_tag) {
        using T = decltype(T_tag);
        constexpr bool C = decltype(c_tag)::value;
        return by_m<T, C>(m, [&](auto mu) { return launch_list<T, decltype(mu)::value, C>(probs, items, n_items, st); });
    };
    if (fp64) return cons ? go(double(), std::true_type{}) : go(double(), std::false_type{});
    return cons ? go(float(), std::true_type{}) : go(float(), std::false_type{});
}
