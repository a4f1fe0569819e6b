// Composed-map half-step kernel for 3-D problems of nodal degree m = 3, element type
// T = float or double: the dissipative method (Sec. 3.3; the modified first step or the
// straightforward variant, exact or truncated series) and the conservative method
// (Sec. 4.1: the even time sum S of the other grid's u, then u_new = 2 S - u_old).
//
// One half step maps a cell's 8 corner nodes (u: 64, v: 27 coefficients each; the
// conservative method u only) linearly to its output node (Sec. 3.1: interpolate, sum the
// Taylor series in time, evaluate at the centre).  The host composes that map into a matrix (cellmap.cpp).  Because the
// Hermite operators are symmetric under reflection about the cell centre and the time
// sums keep the parity of every index, corner s = (s_x, s_y, s_z) enters output a with
// (-1)^(sum_i s_i (a_i + l_i)) times corner 0's entry.  So the corners are first combined
// into the eight sums S_p[l] = sum_s (-1)^(p . s) x_s[l], and output a needs, for each
// input l, only S_{pi(a) xor pi(l)}[l] (pi: the parity vector).  Grouped by the output
// parity class q = pi(a), the outputs of a class (8 of u, <= 8 of v) are one dense
// (<= 16) x 91 product with the class's column of selected sums, applied to 16 cells at a
// time on the matrix cores.
//
// A workgroup (512 threads) owns a column of 4 x CY cells (CY = 4) and walks it upwards
// in z, one node layer of the input grid at a time.  Per layer:
//   1. the layer's 5 x (CY+1) nodes, loaded into registers during the previous layer, are
//      stashed in LDS (ghost nodes outside non-periodic walls mirrored with the odd /
//      even signs of Sec. 3.1.3); the cell layer finished in the previous pass is stored
//      and the loads of the next node layer are issued;
//   2. butterflies: per cell and input l, the four sums over the cell's corners of this
//      layer, T_{pxy}[l], combined with those of the layer below (kept in registers
//      since the previous pass) into the eight sums S_p[l] = T_{pxy}(lower)[l] +-
//      T_{pxy}(upper)[l], written to LDS;
//   3. the class products: the selected sums S_p[l] read as the B operand, the class
//      block of the composed map as the A operand (registers), one 16x16x4 product
//      chain of 23 steps per class and group of 16 cells, one chain per wave;
//      the outputs are staged in LDS for the coalesced stores of step 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "buffer_io.h"
#include "hw_kernels.h"

namespace {

constexpr int CX = 4;                         // cells along x of a workgroup's column
constexpr int NXL = CX + 1;
// LDS strides, chosen for its 32 banks of 4 bytes, which serve a 32-bit access of a wave
// 32 lanes at a time and a 64-bit access 16 lanes at a time.  Every LDS pass of the
// kernel puts the 16 cells of a product group (4 x 4 in x, y) on distinct banks:
//   * nodes: node (x, y) of a layer at x SX + y SY (its inputs contiguous); FP32:
//     SX = 2, SY = 8 (mod 32), so that a corner's 16 nodes fall on the 16 even banks
//     (2 (x + 4 y) mod 32) and the second input of the pass, whose index has the other
//     parity, on the odd ones; FP64: SX = 1, SY = 4 (mod 16), one input per pass;
//   * butterfly sums [cell][ks][p][k mod 4] (k = 4 ks + k mod 4: the K position of the
//     input), so that the 8 sums of one input lie within 29 words of each other (one base
//     address for the butterfly's writes): cell stride = 2 (mod 32) in FP32 (K positions
//     4 ks and 4 ks + 1 of a product's operand pass on the even and odd banks), odd in FP64
// Dissipative method: 91 inputs per node (u 64, v 27) in 23 K-steps (K position 91 reads
// a zero slot of every node), 91 outputs; conservative method (Sec. 4.1): the even time
// sum S of the u inputs, 64 inputs in 16 K-steps, 64 outputs, u_new = 2 S - u_old.
template <typename T, bool CONS>
struct Shape {
    static constexpr int NI = CONS ? 64 : 91;                 // inputs per node
    static constexpr int KS = CONS ? 16 : 23;                 // K-steps of 4
    static constexpr int TL = 4 * KS;                         // K positions
    static constexpr int NV = CONS ? 0 : 27;                  // v outputs per cell
    static constexpr int SX = CONS ? (sizeof(T) == 4 ? 66 : 65) : (sizeof(T) == 4 ? 98 : 97);
    static constexpr int SY = CONS ? (sizeof(T) == 4 ? 360 : 340) : (sizeof(T) == 4 ? 520 : 500);
    static constexpr int TSZ = CONS ? (sizeof(T) == 4 ? 514 : 513) : (sizeof(T) == 4 ? 738 : 737);
    static_assert(SX >= TL && SY >= (CX + 1) * SX && TSZ >= 8 * TL, "strides too small");
};
constexpr int OUS = 68;                       // cell stride of the staged u outputs


template <typename T>
struct Mf;
template <>
struct Mf<float> {
    typedef float vec __attribute__((ext_vector_type(4)));
    static __device__ inline vec mac(float a, float b, vec c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <>
struct Mf<double> {
    typedef double vec __attribute__((ext_vector_type(4)));
    static __device__ inline vec mac(double a, double b, vec c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int l, int r) { return (l >> 4) + 4 * r; }
};

// Tables per problem (lambda and tau are inside the composed map):
//   ta[8][KS][64]  A operand of class q: entry (row i = lane % 16, K position 4 ks + lane / 16,
//                  which holds input perm[4 ks + lane / 16], see create())
//   tb[8][KS][4]   per (class, K-step, lane / 16): offset of the selected butterfly sum in a
//                  cell's block, 32 ks + 4 p + lane / 16 with p = p_x + 2 p_y + 4 p_z of the
//                  input at K position k = 4 ks + lane / 16; the padding position k = 91
//                  reads the zero sums of the zero node slot 91
//   kl[4 KS]       input at K position k (91 for the padding position)
//   bk[4 KS]       K positions of the butterfly passes, two per pass of 16 cells: an even
//                  and an odd position whose inputs have indices of opposite parity
//   tr[8][16]      output of (class, row): -1 unused, else is_v << 12 | flat alpha index
template <typename T, bool CONS>
struct CTables {
    static constexpr int KS = Shape<T, CONS>::KS;
    T ta[8][KS][64];
    int tb[8][KS][4];
    int tr[8][16];
    int kl[4 * KS];
    int bk[4 * KS];
};

// column of CX x CY cells: NC cells per layer
template <typename T, int CY, bool CONS>
struct CShared {
    using S = Shape<T, CONS>;
    static constexpr int NC = CX * CY, NNODE = NXL * (CY + 1);
    // the node layer first: its reads then take the per-thread slot address with small
    // immediate offsets
    alignas(16) T nd[(CY * S::SY + NXL * S::SX + 3) / 4 * 4];
    alignas(16) T tsum[NC * S::TSZ];
    alignas(16) T out[NC * (OUS + S::NV)];
};

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

__device__ inline bool flips(int bc, int l) { return (bc == 1) ? ((l & 1) == 0) : ((l & 1) == 1); }

// coefficient (l_x, l_y, l_z) of input c of a node (u: 4^3, then v: 3^3)
__host__ __device__ inline void coef3(int c, int& lx, int& ly, int& lz)
{
    if (c < 64) {
        lx = c & 3;
        ly = (c >> 2) & 3;
        lz = c >> 4;
    } else {
        const int v = c - 64;
        lx = v % 3;
        ly = (v / 3) % 3;
        lz = v / 9;
    }
}

// The second launch bound is the minimum number of waves per SIMD.  FP32: two
// workgroups of 8 waves per CU, i.e. 4 waves per SIMD, which caps the registers at 128
// per lane (the LDS footprint allows two workgroups); FP64: one workgroup, 2 waves per
// SIMD (at most 256 registers)
// OFF: type of the per-thread byte offsets within a layer of the node arrays -- uint32_t
// when a layer of u fits 4 GB (the loads and stores then go through buffer resources made
// per layer from its wave-uniform base: no per-layer vector address arithmetic), else
// int64_t (global loads and stores at base + offset)
template <typename T, int CY, int NT, bool CONS, typename OFF>
__global__ void __launch_bounds__(NT, sizeof(T) == 4 ? 4 : 2) k_cmap3d(TiledArgs a, int tz, const CTables<T, CONS>* __restrict__ tabs)
{
    using MF = Mf<T>;
    using SH = CShared<T, CY, CONS>;
    using S = Shape<T, CONS>;
    constexpr int NI = S::NI, KS = S::KS, TL = S::TL;
    constexpr int NC = SH::NC, NNODE = SH::NNODE, NW = NT / 64;
    // the 8 classes x NC/16 cell groups of a layer's products over the waves: a wave
    // keeps CPW classes (A operands in registers) and applies each to GPW groups
    constexpr int CPW = NW >= 8 ? 1 : 8 / NW;
    constexpr int GPW = NW >= 8 ? (NC / 16) / (NW / 8) : NC / 16;
    constexpr int NLOAD = (NNODE * NI + NT - 1) / NT;
    static_assert(NW == 4 || (NW % 8 == 0 && (NC / 16) % (NW / 8) == 0), "waves must tile the products");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SH& sh = *reinterpret_cast<SH*>(smem_raw);
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    const int tiles_x = (a.ext_to[0] + CX - 1) / CX;
    const int x0 = (blockIdx.x % tiles_x) * CX, y0 = (blockIdx.x / tiles_x) * CY;
    const int cz0 = blockIdx.y * tz, cz1 = min(cz0 + tz, a.ext_to[2]);
    const int off = (a.to_grid == 1) ? 0 : -1; // input node of corner s = cell + off + s
    typedef const __attribute__((address_space(1))) T* GIn;
    typedef __attribute__((address_space(1))) T* GOut;
    const GIn gu = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.u_in));
    const GIn gv = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.v_in));
    // element at byte offset o from a (wave-uniform) base
    auto at = [](auto base, OFF o) {
        using P = decltype(base);
        typedef typename std::conditional<std::is_const<typename std::remove_pointer<P>::type>::value,
                                          const __attribute__((address_space(1))) char*,
                                          __attribute__((address_space(1))) char*>::type C;
        return reinterpret_cast<P>(reinterpret_cast<C>(base) + o);
    };

    constexpr int TSZ = S::TSZ, SX = S::SX, SY = S::SY;
    // dissipative: slot 91 of every node (the padding input) holds zero, so the
    // butterflies write zero sums for it; the stash never writes it
    if constexpr (!CONS)
        for (int i = tid; i < NNODE; i += NT) sh.nd[(i % NXL) * SX + (i / NXL) * SY + 91] = T(0);

    auto grp_of = [&](int g) { return NW >= 8 ? wave / 8 + (NW / 8) * g : g; };
    // the wave's classes: A operands, B offsets, output targets (registers)
    T ta[CPW][KS];
    int tb[CPW][KS], rdst[CPW][4];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
        const int q = NW >= 8 ? wave % 8 : wave + NW * c;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            ta[c][ks] = tabs->ta[q][ks][lane];
            tb[c][ks] = tabs->tb[q][ks][lane >> 4];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int info = tabs->tr[q][MF::row(lane, r)];
            // unused rows write to the padding word 64 of the cell's u block (never stored)
            rdst[c][r] = info < 0 ? 64 : ((info & 0x1000) ? (1 << 16) | (info & 0xff) : (info & 0xff));
        }
    }

    // ---- node loads: slot i of this thread = element tid + i NT of the layer's block of
    //      the NNODE u records (64 each) followed by the NNODE v records (27 each); NNODE x
    //      64 is a multiple of 64, so every wave's slot reads one of the two arrays, whose
    //      layer base is then wave-uniform.  The xy part, the xy ghost signs and the LDS
    //      slot are fixed per column ----
    const long long plane = (long long)a.ext_from[0] * a.ext_from[1];
    constexpr int NUE = NNODE * 64; // u elements of a layer
    OFF ld_off[NLOAD];              // byte offset within the layer of u or v
    int ld_msk[NLOAD];              // bit 1: negate (xy ghost), bit 3: l_z odd, bits 4..: LDS slot
    T rl[NLOAD];
#pragma unroll
    for (int i = 0; i < NLOAD; ++i) {
        const int e = tid + i * NT;
        ld_off[i] = 0;
        ld_msk[i] = -1; // idle slot: reads node 0 of the layer, never stashed
        if (e >= NNODE * NI) continue;
        const bool isu = e < NUE;
        const int node = isu ? e >> 6 : (e - NUE) / 27, c = isu ? e & 63 : 64 + (e - NUE) % 27;
        int lx, ly, lz;
        coef3(c, lx, ly, lz);
        const Map1 mx = map_node(x0 + off + node % NXL, a.ext_from[0], a.bc[0]);
        const Map1 my = map_node(y0 + off + node / NXL, a.ext_from[1], a.bc[1]);
        const long long nxy = mx.j + (long long)a.ext_from[0] * my.j;
        ld_off[i] = (OFF)((isu ? nxy * 64 + c : nxy * 27 + (c - 64)) * (long long)sizeof(T));
        bool neg = false;
        if (mx.ghost && flips(a.bc[0], lx)) neg = !neg;
        if (my.ghost && flips(a.bc[1], ly)) neg = !neg;
        const int slot = (node % NXL) * SX + (node / NXL) * SY + c;
        ld_msk[i] = (neg ? 2 : 0) | ((lz & 1) << 3) | (slot << 4);
    }
    constexpr bool BUF = std::is_same<OFF, uint32_t>::value;
    const uint32_t ubytes = (uint32_t)(plane * 64 * sizeof(T)), vbytes = (uint32_t)(plane * 27 * sizeof(T));
    int zghost = 0;
    auto fetch = [&](int layer_gz) {
        const Map1 mz = map_node(layer_gz, a.ext_from[2], a.bc[2]);
        zghost = mz.ghost;
        const long long zn = plane * mz.j;
        const GIn lu = gu + zn * 64, lv = CONS ? lu : gv + zn * 27;
        // every slot loads (idle slots from node 0): no branches, so the loads stay in
        // flight until the stash of the next pass
        if constexpr (BUF) {
            const __amdgpu_buffer_rsrc_t ru = make_rsrc((const void*)lu, ubytes);
            const __amdgpu_buffer_rsrc_t rv = CONS ? ru : make_rsrc((const void*)lv, vbytes);
#pragma unroll
            for (int i = 0; i < NLOAD; ++i) {
                const bool isu = CONS || i * NT + 64 * wave < NUE; // wave-uniform
                rl[i] = BufIO<T>::load(isu ? ru : rv, (uint32_t)ld_off[i]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < NLOAD; ++i) {
                const bool isu = CONS || i * NT + 64 * wave < NUE; // wave-uniform
                rl[i] = *at(isu ? lu : lv, ld_off[i]);
            }
        }
    };
    auto stash = [&]() {
        // the z flip of a ghost layer: Dirichlet flips even l_z, Neumann odd l_z
        const bool zflip_odd = a.bc[2] != 1;
#pragma unroll
        for (int i = 0; i < NLOAD; ++i) {
            const int e = tid + i * NT;
            if (e >= NNODE * NI) break;
            const int m = ld_msk[i];
            bool neg = (m & 2) != 0;
            if (zghost && (((m >> 3) & 1) != 0) == zflip_odd) neg = !neg;
            sh.nd[m >> 4] = neg ? -rl[i] : rl[i];
        }
    };

    // ---- staged outputs of a cell layer, stored coalesced: per thread, output slot k
    //      (element tid + k NT of the layer's NC u or v records) at a byte offset within
    //      the output layer fixed per column; bit k of s_ok: the cell is inside the grid ----
    const int nlayers = cz1 - cz0 + 1;
    constexpr int NSU = (NC * 64 + NT - 1) / NT, NSV = CONS ? 1 : (NC * 27 + NT - 1) / NT;
    OFF su_off[NSU], sv_off[NSV];
    int s_ok = 0;
#pragma unroll
    for (int k = 0; k < NSU; ++k) {
        const int i = tid + k * NT, c = (i >> 6) % NC, coef = i & 63;
        const int gx = x0 + c % CX, gy = y0 + c / CX;
        su_off[k] = (OFF)(((gx + (long long)a.ext_to[0] * gy) * 64 + coef) * (long long)sizeof(T));
        if (i < NC * 64 && gx < a.ext_to[0] && gy < a.ext_to[1]) s_ok |= 1 << k;
    }
#pragma unroll
    for (int k = 0; k < NSV; ++k) {
        const int i = tid + k * NT, c = (i / 27) % NC, coef = i % 27;
        const int gx = x0 + c % CX, gy = y0 + c / CX;
        sv_off[k] = (OFF)(((gx + (long long)a.ext_to[0] * gy) * 27 + coef) * (long long)sizeof(T));
        if (!CONS && i < NC * 27 && gx < a.ext_to[0] && gy < a.ext_to[1]) s_ok |= 1 << (16 + k);
    }
    const long long plane_to = (long long)a.ext_to[0] * a.ext_to[1];
    // conservative: the old level of the cell layer stored in the next pass, loaded at the
    // end of this pass's loads so that its latency overlaps the layer's work
    T ov[CONS ? NSU : 1];
    const uint32_t uobytes = (uint32_t)(plane_to * 64 * sizeof(T)), vobytes = (uint32_t)(plane_to * 27 * sizeof(T));
    auto old_fetch = [&](int cz) {
        if constexpr (CONS) {
            const GIn old_l = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.u_old)) + plane_to * cz * 64;
            if constexpr (BUF) {
                const __amdgpu_buffer_rsrc_t r = make_rsrc((const void*)old_l, uobytes);
#pragma unroll
                for (int k = 0; k < NSU; ++k)
                    if (s_ok & (1 << k)) ov[k] = BufIO<T>::load(r, (uint32_t)su_off[k]);
            } else {
#pragma unroll
                for (int k = 0; k < NSU; ++k)
                    if (s_ok & (1 << k)) ov[k] = *at(old_l, su_off[k]);
            }
        }
    };
    T* const ou_base = sh.out;
    T* const ov_base = sh.out + NC * OUS;
    auto store_layer = [&](int cz) {
        const GOut out_u = reinterpret_cast<GOut>(reinterpret_cast<uintptr_t>(a.u_out)) + plane_to * cz * 64;
        const GOut out_v = reinterpret_cast<GOut>(reinterpret_cast<uintptr_t>(a.v_out)) + plane_to * cz * 27;
        // (unused where BUF is false)
        const __amdgpu_buffer_rsrc_t ru = make_rsrc((const void*)out_u, uobytes);
        const __amdgpu_buffer_rsrc_t rv = make_rsrc((const void*)out_v, vobytes);
        auto put = [&](GOut base, __amdgpu_buffer_rsrc_t r, OFF o, T v) {
            if constexpr (BUF) BufIO<T>::store(v, r, (uint32_t)o);
            else *at(base, o) = v;
        };
        if constexpr (sizeof(T) == 8) {
            // FP64 (one workgroup per CU): every slot's staged value read first, indices
            // clamped into the staging area, so that one wait covers the reads (the empty asm
            // statements keep the compiler from sinking the reads into the stores' branches);
            // in FP32 the same order measured slower
            T su[NSU], sv[NSV];
#pragma unroll
            for (int k = 0; k < NSU; ++k) {
                const int i = min(tid + k * NT, NC * 64 - 1);
                su[k] = ou_base[(i >> 6) * OUS + (i & 63)];
            }
            if constexpr (!CONS) {
#pragma unroll
                for (int k = 0; k < NSV; ++k) sv[k] = ov_base[min(tid + k * NT, NC * 27 - 1)];
            }
#pragma unroll
            for (int k = 0; k < NSU; ++k) asm volatile("" ::"v"(su[k]));
#pragma unroll
            for (int k = 0; k < NSU; ++k) {
                if (!(s_ok & (1 << k))) continue;
                // conservative: u_new = 2 S - u_old, the old values loaded one pass earlier
                if constexpr (CONS) put(out_u, ru, su_off[k], T(2) * su[k] - ov[k]);
                else put(out_u, ru, su_off[k], su[k]);
            }
            if constexpr (!CONS) {
#pragma unroll
                for (int k = 0; k < NSV; ++k)
                    if (s_ok & (1 << (16 + k))) put(out_v, rv, sv_off[k], sv[k]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < NSU; ++k) {
                const int i = tid + k * NT, c = i >> 6, coef = i & 63;
                if (!(s_ok & (1 << k))) continue;
                // conservative: u_new = 2 S - u_old, the old values loaded one pass earlier
                if constexpr (CONS) put(out_u, ru, su_off[k], T(2) * ou_base[c * OUS + coef] - ov[k]);
                else put(out_u, ru, su_off[k], ou_base[c * OUS + coef]);
            }
            if constexpr (!CONS) {
#pragma unroll
                for (int k = 0; k < NSV; ++k) {
                    const int i = tid + k * NT;
                    if (s_ok & (1 << (16 + k))) put(out_v, rv, sv_off[k], ov_base[i]);
                }
            }
        }
    };

    constexpr int NBF = (NC * TL + NT - 1) / NT; // butterfly slots per thread
    // T_pxy of the lower node layer: with two sets (where the registers allow: not in the
    // FP32 dissipative kernel with 64-bit offsets, which would spill), the pass over layer
    // `step` writes its own into set step & 1 and reads the lower layer's from the other
    // (no copies)
    constexpr int NPS = (sizeof(T) == 8 || CONS || BUF) ? 2 : 1;
    T prev[NPS][NBF][4];
    int bkp[NBF], bl[NBF];                       // K position and input of each slot
#pragma unroll
    for (int k = 0; k < NBF; ++k) {
        const int t = tid + k * NT;
        bkp[k] = t < NC * TL ? tabs->bk[2 * ((t >> 5) / (NC / 16)) + ((t >> 4) & 1)] : 0;
        bl[k] = tabs->kl[bkp[k]];
    }
    auto pass = [&](auto B, int step) {
        constexpr int CUR = NPS == 2 ? decltype(B)::value : 0, LO = NPS == 2 ? 1 - CUR : 0;
        // The stash, stores, loads and butterflies run at a raised wave priority, the class
        // products at the normal one: on a SIMD shared by the two workgroups of a CU, the
        // instructions of a workgroup heading for its next barrier are issued first and the
        // other workgroup's product chains fill the gaps (matrix-core and vector
        // instructions do not execute together; FP32 launch 5.32 -> 5.0 ms).
        __builtin_amdgcn_s_setprio(1);
        stash();
        __syncthreads();
        if (step >= 2) store_layer(cz0 + step - 2);
        if (step + 1 < nlayers) fetch(cz0 + off + step + 1);
        if constexpr (CONS)
            if (step >= 1) old_fetch(cz0 + step - 1); // the cell layer computed in this pass

        // ---- 2. butterflies: T_pxy[l] of this layer (pxy = px + 2 py), combined with
        //      the lower layer's into S_p[l], stored at the input's K position kp; 32
        //      lanes cover 16 cells x the two positions of a pair, and a thread keeps the
        //      same (cell, kp) slots in every pass ----
#pragma unroll
        for (int k = 0; k < NBF; ++k) {
            const int t = tid + k * NT;
            if (t >= NC * TL) break;
            const int cell = (t & 15) + 16 * ((t >> 5) % (NC / 16)), kp = bkp[k];
            const int l = bl[k];
            const int nb = (cell % CX) * SX + (cell / CX) * SY + l;
            const T x00 = sh.nd[nb], x10 = sh.nd[nb + SX];
            const T x01 = sh.nd[nb + SY], x11 = sh.nd[nb + SX + SY];
            const T p = x00 + x10, q = x00 - x10, r = x01 + x11, s = x01 - x11;
            const T cur[4] = {p + r, q + s, p - r, q - s};
            if (step > 0) {
                T* dst = sh.tsum + cell * TSZ + 32 * (kp >> 2) + (kp & 3);
#pragma unroll
                for (int pxy = 0; pxy < 4; ++pxy) {
                    dst[4 * pxy] = prev[LO][k][pxy] + cur[pxy];
                    dst[4 * (4 + pxy)] = prev[LO][k][pxy] - cur[pxy];
                }
            }
#pragma unroll
            for (int pxy = 0; pxy < 4; ++pxy) prev[CUR][k][pxy] = cur[pxy];
        }
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        if (step == 0) return; // the first layer only primes the sums

        // ---- 3. class products for the cell layer between the two node layers ----
        T bv[CPW][GPW][KS];
        auto load_b = [&](int ks0, int ks1) {
#pragma unroll
            for (int c = 0; c < CPW; ++c)
#pragma unroll
                for (int g = 0; g < GPW; ++g)
#pragma unroll
                    for (int ks = ks0; ks < ks1; ++ks)
                        bv[c][g][ks] = sh.tsum[(16 * grp_of(g) + (lane & 15)) * TSZ + tb[c][ks]];
        };
        typename MF::vec acc[CPW][GPW];
#pragma unroll
        for (int c = 0; c < CPW; ++c)
#pragma unroll
            for (int g = 0; g < GPW; ++g) acc[c][g] = typename MF::vec{T(0), T(0), T(0), T(0)};
        auto products = [&](int ks0, int ks1) {
#pragma unroll
            for (int ks = ks0; ks < ks1; ++ks)
#pragma unroll
                for (int c = 0; c < CPW; ++c)
#pragma unroll
                    for (int g = 0; g < GPW; ++g) acc[c][g] = MF::mac(ta[c][ks], bv[c][g][ks], acc[c][g]);
        };
        // the first half of the operands is read before any product; the second half is
        // read while the first half's products run
        constexpr int KH = KS / 2;
        load_b(0, KH);
        __builtin_amdgcn_sched_barrier(0);
        load_b(KH, KS);
        products(0, KH);
        __builtin_amdgcn_sched_barrier(0);
        products(KH, KS);
#pragma unroll
        for (int c = 0; c < CPW; ++c)
#pragma unroll
            for (int g = 0; g < GPW; ++g) {
                const int cell = 16 * grp_of(g) + (lane & 15);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int dst = rdst[c][r];
                    const int ai = dst & 0xffff;
                    const int o = dst >= (1 << 16) ? NC * OUS + cell * 27 + ai : cell * OUS + ai;
                    ou_base[o] = acc[c][g][r];
                }
            }
    };
    fetch(cz0 + off);
    for (int step = 0; step < nlayers; step += 2) {
        pass(std::integral_constant<int, 0>{}, step);
        if (step + 1 < nlayers) pass(std::integral_constant<int, 1>{}, step + 1);
    }
    if (nlayers >= 2) {
        __syncthreads();
        store_layer(cz1 - 1);
    }
}

// ---------------------------------------------------------------------------
// host: tables and launch
// ---------------------------------------------------------------------------
template <typename T, bool CONS>
hipError_t create(const ProblemDesc& D, void** out)
{
    using S = Shape<T, CONS>;
    constexpr int NI = S::NI, KS = S::KS;
    using Tab = CTables<T, CONS>;
    std::vector<double> G;
    int n_in = 0, n_out = 0;
    hw_cell_map(D, G, n_in, n_out); // [8 * NI][NI], corner 0's rows first
    if (n_out != NI || n_in != 8 * NI) return hipErrorInvalidValue;
    // K order of the inputs (the products accumulate in it, in the element type):
    // higher-degree coefficients first.  On smooth data those are the smaller terms, so
    // the running sums stay small until the large low-degree terms enter; in FP32 that
    // order leaves several times less rounding error than the natural one.  Dissipative:
    // position 91 is the padding input.
    int perm[4 * KS];
    {
        int k = 0;
        for (int dg = 9; dg >= 0; --dg)
            for (int l = 0; l < NI; ++l) {
                int lx, ly, lz;
                coef3(l, lx, ly, lz);
                if (lx + ly + lz == dg) perm[k++] = l;
            }
        while (k < 4 * KS) perm[k++] = -1;
    }
    Tab* h = new Tab();
    std::memset(h, 0, sizeof *h);
    for (int k = 0; k < 4 * KS; ++k) h->kl[k] = perm[k] < 0 ? 91 : perm[k];
    // butterfly pairs: (even K position, odd K position) with inputs of opposite index
    // parity.  There are as many even positions holding even inputs as odd positions
    // holding odd ones (half the positions hold inputs of each parity), so the pairs
    // always exist.
    {
        std::vector<int> cls[4]; // [position parity][input parity]
        for (int k = 0; k < 4 * KS; ++k) cls[2 * (k & 1) + (h->kl[k] & 1)].push_back(k);
        if (cls[0].size() != cls[3].size() || cls[1].size() != cls[2].size()) {
            delete h;
            return hipErrorInvalidValue;
        }
        int j = 0;
        for (size_t i = 0; i < cls[0].size(); ++i, ++j) {
            h->bk[2 * j] = cls[0][i];
            h->bk[2 * j + 1] = cls[3][i];
        }
        for (size_t i = 0; i < cls[1].size(); ++i, ++j) {
            h->bk[2 * j] = cls[1][i];
            h->bk[2 * j + 1] = cls[2][i];
        }
    }
    for (int q = 0; q < 8; ++q) {
        const int qx = q & 1, qy = (q >> 1) & 1, qz = (q >> 2) & 1;
        // rows: the 8 u outputs of the class, then (dissipative) its v outputs
        int rows[16], nrow = 0;
        for (int o = 0; o < 8; ++o)
            rows[nrow++] = (qx + 2 * (o & 1)) + 4 * (qy + 2 * ((o >> 1) & 1)) + 16 * (qz + 2 * (o >> 2));
        if (!CONS)
            for (int az = qz; az <= 2; az += 2)
                for (int ay = qy; ay <= 2; ay += 2)
                    for (int ax = qx; ax <= 2; ax += 2) rows[nrow++] = 64 + ax + 3 * ay + 9 * az;
        for (int r = 0; r < 16; ++r)
            h->tr[q][r] = r < nrow ? (rows[r] >= 64 ? 0x1000 | (rows[r] - 64) : rows[r]) : -1;
        for (int ks = 0; ks < KS; ++ks) {
            for (int g = 0; g < 4; ++g) {
                const int l = perm[4 * ks + g];
                if (l < 0) {
                    h->tb[q][ks][g] = 32 * ks + g; // p = 0: the sums of the zero node slot
                    continue;
                }
                int lx, ly, lz;
                coef3(l, lx, ly, lz);
                const int px = (qx + lx) & 1, py = (qy + ly) & 1, pz = (qz + lz) & 1;
                h->tb[q][ks][g] = 32 * ks + 4 * (px + 2 * py + 4 * pz) + g;
            }
            for (int lanei = 0; lanei < 64; ++lanei) {
                const int i = lanei & 15, l = perm[4 * ks + (lanei >> 4)];
                h->ta[q][ks][lanei] = (i < nrow && l >= 0) ? (T)G[(size_t)l * NI + rows[i]] : T(0);
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

template <typename T, int CY, int NT, bool CONS, typename OFF>
hipError_t launch(const TiledArgs& a, hipStream_t st)
{
    const size_t lds = sizeof(CShared<T, CY, CONS>);
    auto kern = k_cmap3d<T, CY, NT, CONS, OFF>;
    hipError_t e = hw_lds_limit<k_cmap3d<T, CY, NT, CONS, OFF>>(lds);
    if (e != hipSuccess) return e;
    // z-chunks of 64 cell layers, doubled while at least 2048 workgroups remain (each
    // chunk re-reads one node layer below it: longer chunks waste less)
    const int tiles = ((a.ext_to[0] + CX - 1) / CX) * ((a.ext_to[1] + CY - 1) / CY);
    int tz = 64;
    while (tz < a.ext_to[2] && (int64_t)tiles * ((a.ext_to[2] + 2 * tz - 1) / (2 * tz)) >= 2048) tz *= 2;
    const int chunks = (a.ext_to[2] + tz - 1) / tz;
    hipLaunchKernelGGL(kern, dim3(tiles, chunks), dim3(NT), lds, st, a, tz,
                       static_cast<const CTables<T, CONS>*>(a.tables));
    return hipGetLastError();
}

} // namespace

hipError_t hw_cmap3d_tables_create(const ProblemDesc& D, bool fp64, void** out)
{
    *out = nullptr;
    if (D.d != 3 || D.m != 3) return hipErrorInvalidValue;
    if (D.variant == HWV_CONS) return fp64 ? create<double, true>(D, out) : create<float, true>(D, out);
    if (D.variant != HWV_DISS_FULL && D.variant != HWV_DISS_SIMPLE) return hipErrorInvalidValue;
    return fp64 ? create<double, false>(D, out) : create<float, false>(D, out);
}

hipError_t hw_launch_cmap3d(const TiledArgs& a, bool fp64, hipStream_t st)
{
    if (!a.tables) return hipErrorInvalidValue;
    if (a.cons && !a.u_old) return hipErrorInvalidValue;
    for (int i = 0; i < 3; ++i)
        if (a.ext_to[i] < 1 || a.ext_from[i] < 1) return hipErrorInvalidValue;
    // 4 x 4-cell columns, 512 threads: one class and one group of 16 cells per wave.
    // FP32: 62 KB (dissipative) / 46 KB (conservative) of LDS and at most 128 registers:
    // two workgroups per CU, four waves per SIMD; FP64: 123 / 92 KB, one workgroup per CU
    // (two waves per SIMD)
    // 32-bit offsets within a layer where a layer of u (64 coefficients per node) of either
    // grid fits 4 GB (HW_TUNE_FORCE="cmap3d_offsets=64" imposes the 64-bit form, so that
    // tests reach it on small grids)
    const double layer = 64.0 * (fp64 ? 8 : 4) * std::max((double)a.ext_from[0] * a.ext_from[1],
                                                           (double)a.ext_to[0] * a.ext_to[1]);
    int forced = 0;
    const bool wide = hw_tune_forced("cmap3d_offsets", forced) && forced == 64;
    if (layer < 4294967296.0 && !wide) {
        if (a.cons) return fp64 ? launch<double, 4, 512, true, uint32_t>(a, st) : launch<float, 4, 512, true, uint32_t>(a, st);
        return fp64 ? launch<double, 4, 512, false, uint32_t>(a, st) : launch<float, 4, 512, false, uint32_t>(a, st);
    }
    if (a.cons) return fp64 ? launch<double, 4, 512, true, int64_t>(a, st) : launch<float, 4, 512, true, int64_t>(a, st);
    return fp64 ? launch<double, 4, 512, false, int64_t>(a, st) : launch<float, 4, 512, false, int64_t>(a, st);
}
