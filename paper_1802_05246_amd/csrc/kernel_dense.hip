// Per-lane dense half-step kernel for d <= 2: one lane per output node ("cell").
//
// The half step of one cell is a fixed linear map of its 2^d corner nodes (composed on
// the host into the matrix G, see cellmap.cpp); every lane gathers its corners from
// global memory, mirrors ghost corners outside non-periodic walls with the odd / even
// signs of Sec. 3.1.3, and accumulates the product with G in registers, one input at a
// time against all outputs (corners first combined by the reflection symmetry, so that
// G holds one corner's rows).  G is the same for every lane, so its entries are read
// through the scalar unit and enter the FMAs as scalar operands.  Dissipative: the
// outputs are u' and v' of the node; conservative (Sec. 4.1): the even time sum S,
// and u_new = 2 S - u_old.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hw_kernels.h"

namespace {

constexpr int DENSE_BLOCK = 256;

constexpr int cpow(int b, int e) { return e == 0 ? 1 : b * cpow(b, e - 1); }

// sign of coefficient l of a node mirrored across a wall of type bc (1: Dirichlet,
// odd extension: (-1)^(l+1); 2: Neumann, even extension: (-1)^l)
__device__ inline bool flips(int bc, int l) { return (bc == 1) ? ((l & 1) == 0) : ((l & 1) == 1); }

template <typename T, int D, int MU, bool CONS>
__device__ void dense_cell(const DenseArgs& a, int64_t cell)
{
    constexpr int MV = CONS ? 0 : MU - 1;
    constexpr int NU = cpow(MU, D), NV = CONS ? 0 : cpow(MV, D);
    constexpr int NO = CONS ? NU : NU + NV;
    // the old level is read before the products (its latency overlaps them) unless the
    // registers it would hold are needed more by the accumulators (conservative m = 6)
    constexpr bool EARLY_OLD = CONS && NU <= 36;

    // corners: input node per dimension and side, and whether it is a ghost image
    int node[2][2];
    bool ghost[2][2];
    int64_t rem = cell;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const int oi = (int)(rem % a.ext_to[i]);
        rem /= a.ext_to[i];
        const int ext = a.ext_from[i];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            int j;
            bool gh = false;
            if (a.to_grid == 1) { // dual node i+1/2: primal nodes i, i+1
                j = oi + s;
                if (a.bc[i] == 0 && j >= ext) j -= ext;
            } else {              // primal node i: dual nodes i-1/2, i+1/2
                j = oi - 1 + s;
                if (a.bc[i] == 0) {
                    if (j < 0) j += ext;
                } else if (j < 0) {
                    j = 0;
                    gh = true;
                } else if (j >= ext) {
                    j = ext - 1;
                    gh = true;
                }
            }
            node[i][s] = j;
            ghost[i][s] = gh;
        }
    }

    // G holds the rows of corner 0 only: by the reflection symmetry of the Hermite
    // operators about the cell centre (which the time sums keep, as they preserve the
    // parity of every index), corner c = (s_0, s_1) enters output a with
    // (-1)^(sum_i s_i (a_i + l_i)) times corner 0's entry, so the corners are first
    // combined into the 2^d sums S_p = sum_c (-1)^(p . s) x_c and each entry of G
    // multiplies the one S_p whose parities p = a + l (mod 2) it needs
    // G is read through the constant address space: its loads are wave-uniform and the
    // kernel never writes it, so they go through the scalar unit also where the pointer
    // itself comes from memory (the batch kernel's per-problem descriptors), not only
    // from a kernel argument
    typedef const __attribute__((address_space(4))) T* ConstPtr;
    const ConstPtr G = reinterpret_cast<ConstPtr>(reinterpret_cast<uintptr_t>(a.G));
    // the node arrays are global memory: said explicitly, so that pointers read from
    // memory (batch descriptors) load and store as global, not generic, accesses
    typedef const __attribute__((address_space(1))) T* GIn;
    typedef __attribute__((address_space(1))) T* GOut;
    const GIn __restrict__ uin = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.u_in));
    const GIn __restrict__ vin = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.v_in));
    const GIn __restrict__ uold_in = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.u_old));
    // conservative: the old level is read first, so that its latency overlaps the products
    T uold[EARLY_OLD ? NU : 1];
    if constexpr (EARLY_OLD) {
#pragma unroll
        for (int o = 0; o < NU; ++o) uold[o] = uold_in[cell * NU + o];
    }
    T acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = T(0);

    int64_t nd[1 << D];
    bool gx[1 << D][2];
#pragma unroll
    for (int c = 0; c < (1 << D); ++c) {
        int64_t st = 1;
        nd[c] = 0;
        gx[c][1] = false;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            const int s = (c >> i) & 1;
            nd[c] += node[i][s] * st;
            st *= a.ext_from[i];
            gx[c][i] = ghost[i][s];
        }
    }
    // parity of output o along dimension i
    auto opar = [](int o, int i) {
        const int md = o < NU ? MU : MV, oo = o < NU ? o : o - NU;
        return (i == 0 ? oo % md : (oo / md) % md) & 1;
    };
    // one block (u: extent MU per dimension, v: MV) of the corners against G
    auto block = [&](const GIn base, auto md_tag, int in0) {
        constexpr int MD = decltype(md_tag)::value;
        constexpr int NB = cpow(MD, D);
        // input l = lx + MD ly; ly_odd: the y parity of l when it is not known at compile time
        auto one = [&](int l, int lx, int ly, bool ly_odd) {
            T x[1 << D];
#pragma unroll
            for (int c = 0; c < (1 << D); ++c) {
                bool neg = false;
                if (gx[c][0] && flips(a.bc[0], lx)) neg = !neg;
                if (D > 1 && gx[c][1] && flips(a.bc[1], ly)) neg = !neg;
                const T v = base[nd[c] * NB + l];
                x[c] = neg ? -v : v;
            }
            T S[1 << D];
            if constexpr (D == 1) {
                S[0] = x[0] + x[1];
                S[1] = x[0] - x[1];
            } else {
                const T p = x[0] + x[1], q = x[0] - x[1], r = x[2] + x[3], t = x[2] - x[3];
                // S[px + 2 py]; with ly odd the roles of py = 0 and 1 swap
                S[0] = ly_odd ? p - r : p + r;
                S[1] = ly_odd ? q - t : q + t;
                S[2] = ly_odd ? p + r : p - r;
                S[3] = ly_odd ? q + t : q - t;
            }
            const ConstPtr g = G + (int64_t)(in0 + l) * NO;
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                const int px = (opar(o, 0) + lx) & 1;
                const int py = D > 1 ? opar(o, 1) : 0;
                acc[o] += g[o] * S[px + 2 * py];
            }
        };
        if constexpr (D == 1) {
#pragma unroll
            for (int l = 0; l < NB; ++l) one(l, l, 0, false);
        } else {
            // a loop over the rows l_y: keeps the loads of one row in flight at a time (few
            // registers, many waves) and the code within the instruction cache
#pragma unroll 1
            for (int ly = 0; ly < MD; ++ly)
#pragma unroll
                for (int lx = 0; lx < MD; ++lx) one(lx + MD * ly, lx, ly, (ly & 1) != 0);
        }
    };
    block(uin, std::integral_constant<int, MU>{}, 0);
    if constexpr (!CONS) block(vin, std::integral_constant<int, MV>{}, NU);

    const GOut __restrict__ uo = reinterpret_cast<GOut>(reinterpret_cast<uintptr_t>(a.u_out)) + cell * NU;
    if constexpr (EARLY_OLD) {
#pragma unroll
        for (int o = 0; o < NU; ++o) uo[o] = T(2) * acc[o] - uold[o];
    } else if constexpr (CONS) {
        // the old level in chunks of 16, each chunk's loads issued before its stores (the
        // compiler cannot tell that the old and new levels do not overlap, and would
        // otherwise wait for every load after the previous store)
        const GIn __restrict__ old = uold_in + cell * NU;
        constexpr int CH = 16;
#pragma unroll
        for (int o0 = 0; o0 < NU; o0 += CH) {
            T ov[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j)
                if (o0 + j < NU) ov[j] = old[o0 + j];
#pragma unroll
            for (int j = 0; j < CH; ++j)
                if (o0 + j < NU) uo[o0 + j] = T(2) * acc[o0 + j] - ov[j];
        }
    } else {
        const GOut __restrict__ vo = reinterpret_cast<GOut>(reinterpret_cast<uintptr_t>(a.v_out)) + cell * NV;
#pragma unroll
        for (int o = 0; o < NU; ++o) uo[o] = acc[o];
#pragma unroll
        for (int o = 0; o < NV; ++o) vo[o] = acc[NU + o];
    }
}

// one problem: 1-D consecutive cells per workgroup; 2-D tiles of TX x (256 / TX) cells
// (TX = a.tile_x), so that the rows of corner nodes a workgroup reads are shared by its
// own cells
template <typename T, int D, int MU, bool CONS>
__global__ void __launch_bounds__(DENSE_BLOCK) k_dense(DenseArgs a)
{
    int64_t cell;
    if constexpr (D == 1) {
        cell = (int64_t)blockIdx.x * DENSE_BLOCK + threadIdx.x;
        if (cell >= a.n_cells) return;
    } else {
        const int tx = a.tile_x;
        const int tiles_x = (a.ext_to[0] + tx - 1) / tx;
        const int x = (blockIdx.x % tiles_x) * tx + (int)threadIdx.x % tx;
        const int y = (blockIdx.x / tiles_x) * (DENSE_BLOCK / tx) + (int)threadIdx.x / tx;
        if (x >= a.ext_to[0] || y >= a.ext_to[1]) return;
        cell = x + (int64_t)a.ext_to[0] * y;
    }
    dense_cell<T, D, MU, CONS>(a, cell);
}

// Many half steps of one small 1-D problem in one launch of one workgroup (a launch per half
// step of a few dozen cells costs more than the cells' work): half step k takes its arguments
// from args[(k & 1) * 2 + ((k >> 1) & 1)] (direction, conservative slot parity), its lanes loop
// over the cells, and a barrier separates it from the next, whose inputs are this one's
// outputs.  The waves of a workgroup share one CU and its vector L1, so the barrier (which
// waits for the stores) is all the visibility the next half step's loads need.
template <typename T, int MU, bool CONS>
__global__ void __launch_bounds__(DENSE_BLOCK) k_dense1d_steps(const DenseArgs* __restrict__ args, int k0, int n_half)
{
    for (int k = k0; k < k0 + n_half; ++k) {
        const DenseArgs a = args[(k & 1) * 2 + ((k >> 1) & 1)];
        for (int64_t cell = threadIdx.x; cell < a.n_cells; cell += DENSE_BLOCK) dense_cell<T, 1, MU, CONS>(a, cell);
        __syncthreads();
    }
}

template <typename T, int MU, bool CONS>
hipError_t launch_1d_steps(const DenseArgs* args, int k0, int n_half, hipStream_t st)
{
    hipLaunchKernelGGL((k_dense1d_steps<T, MU, CONS>), dim3(1), dim3(DENSE_BLOCK), 0, st, args, k0, n_half);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_1d_steps(const DenseArgs* args, int k0, int n_half, int m, bool cons, hipStream_t st)
{
    if (cons) {
        switch (m) {
        case 0: return launch_1d_steps<T, 1, true>(args, k0, n_half, st);
        case 1: return launch_1d_steps<T, 2, true>(args, k0, n_half, st);
        case 2: return launch_1d_steps<T, 3, true>(args, k0, n_half, st);
        case 3: return launch_1d_steps<T, 4, true>(args, k0, n_half, st);
        case 4: return launch_1d_steps<T, 5, true>(args, k0, n_half, st);
        case 5: return launch_1d_steps<T, 6, true>(args, k0, n_half, st);
        case 6: return launch_1d_steps<T, 7, true>(args, k0, n_half, st);
        }
    } else {
        switch (m) {
        case 1: return launch_1d_steps<T, 2, false>(args, k0, n_half, st);
        case 2: return launch_1d_steps<T, 3, false>(args, k0, n_half, st);
        case 3: return launch_1d_steps<T, 4, false>(args, k0, n_half, st);
        case 4: return launch_1d_steps<T, 5, false>(args, k0, n_half, st);
        case 5: return launch_1d_steps<T, 6, false>(args, k0, n_half, st);
        case 6: return launch_1d_steps<T, 7, false>(args, k0, n_half, st);
        }
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------
// LDS-staged 2-D form: a workgroup's tile of TX x TY cells (TX TY = 256) first copies the
// (TX+1) x (TY+1) input nodes it needs into LDS with coalesced loads (a row of nodes is
// contiguous in memory), ghost nodes mirrored there; the lanes then read their corners
// from LDS, and the outputs go back through LDS so that they too are stored (and the
// conservative old level read) with coalesced accesses.  Per cell the arithmetic is the
// per-lane dense form above.
template <typename T, int MU, bool CONS>
struct StagedShape {
    static constexpr int MV = CONS ? 0 : MU - 1;
    static constexpr int NU = MU * MU, NV = MV * MV, NI = NU + NV, NO = NI;
    // odd strides: a lane per cell (or node) at this stride touches distinct banks
    static constexpr int NIP = NI | 1, NOP = NO | 1;
    static constexpr size_t lds_words(int tx)
    {
        const size_t in = (size_t)(tx + 1) * (DENSE_BLOCK / tx + 1) * NIP, out = (size_t)DENSE_BLOCK * NOP;
        return in > out ? in : out;
    }
};

__device__ inline int wrap_node(int j, int ext, int bc, bool& ghost)
{
    ghost = false;
    if (bc == 0) {
        j %= ext;
        return j < 0 ? j + ext : j;
    }
    if (j < 0) {
        ghost = true;
        return 0;
    }
    if (j >= ext) {
        ghost = true;
        return ext - 1;
    }
    return j;
}

template <typename T, int MU, bool CONS, int TX>
__device__ void dense_tile_staged(const DenseArgs& a, int x0, int y0, T* __restrict__ sm)
{
    using S = StagedShape<T, MU, CONS>;
    constexpr int TY = DENSE_BLOCK / TX, NXT = TX + 1, NYT = TY + 1;
    constexpr int MV = S::MV, NU = S::NU, NV = S::NV, NO = S::NO, NIP = S::NIP, NOP = S::NOP;
    typedef const __attribute__((address_space(1))) T* GIn;
    typedef __attribute__((address_space(1))) T* GOut;
    typedef const __attribute__((address_space(4))) T* ConstPtr;
    const int tid = threadIdx.x;
    const int off = a.to_grid == 1 ? 0 : -1; // input node of corner s = cell + off + s
    const int ex0 = a.ext_from[0], ex1 = a.ext_from[1];

    // ---- stage the input nodes (u block, then v block of every node): row by row of
    //      the tile, each thread keeping the same (node column, coefficient) slots in
    //      every row, so that the column's index and x ghost sign are computed once ----
    auto stage = [&](const GIn src, auto md_tag, int base) {
        constexpr int MD = decltype(md_tag)::value, NB = MD * MD;
        constexpr int PER_ROW = NXT * NB, SLOTS = (PER_ROW + DENSE_BLOCK - 1) / DENSE_BLOCK;
        int col[SLOTS], dst[SLOTS];
        bool negx[SLOTS], ylflip_even[SLOTS];
#pragma unroll
        for (int k = 0; k < SLOTS; ++k) {
            const int e = tid + k * DENSE_BLOCK;
            const int xx = e / NB, l = e - xx * NB;
            bool gxg;
            const int gx = wrap_node(x0 + xx + off, ex0, a.bc[0], gxg);
            col[k] = gx * NB + l;
            dst[k] = xx * NIP + base + l;
            negx[k] = gxg && flips(a.bc[0], l % MD);
            ylflip_even[k] = ((l / MD) & 1) == 0;
        }
        // Dirichlet (bc 1) mirrors flip the even l_y, Neumann (bc 2) the odd ones
        const bool yflip_even = a.bc[1] == 1;
        // groups of rows whose loads are all issued before the first is written to LDS
        // (at most 32 values in flight per thread)
        constexpr int RG = SLOTS >= 32 ? 1 : (32 / SLOTS < NYT ? 32 / SLOTS : NYT);
        for (int yg = 0; yg < NYT; yg += RG) {
            T v[RG][SLOTS];
            bool gyg[RG];
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                if (yg + r >= NYT) break;
                const int gy = wrap_node(y0 + yg + r + off, ex1, a.bc[1], gyg[r]);
                const GIn row = src + (int64_t)gy * ex0 * NB;
#pragma unroll
                for (int k = 0; k < SLOTS; ++k)
                    if (k * DENSE_BLOCK + tid < PER_ROW) v[r][k] = row[col[k]];
            }
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                if (yg + r >= NYT) break;
#pragma unroll
                for (int k = 0; k < SLOTS; ++k) {
                    if (k * DENSE_BLOCK + tid >= PER_ROW) break;
                    const bool neg = negx[k] != (gyg[r] && ylflip_even[k] == yflip_even);
                    sm[(yg + r) * NXT * NIP + dst[k]] = neg ? -v[r][k] : v[r][k];
                }
            }
        }
    };
    stage(reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.u_in)), std::integral_constant<int, MU>{}, 0);
    if constexpr (!CONS)
        stage(reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.v_in)), std::integral_constant<int, MV>{}, NU);
    __syncthreads();

    // ---- per lane: corners from LDS, sums S_p, products with G (scalar operands) ----
    const int tx = tid % TX, ty = tid / TX;
    const ConstPtr G = reinterpret_cast<ConstPtr>(reinterpret_cast<uintptr_t>(a.G));
    T acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = T(0);
    auto opar = [](int o, int i) {
        const int md = o < NU ? MU : MV, oo = o < NU ? o : o - NU;
        return (i == 0 ? oo % md : (oo / md) % md) & 1;
    };
    const T* __restrict__ n00 = sm + (ty * NXT + tx) * NIP;
    auto block = [&](auto md_tag, int in0) {
        constexpr int MD = decltype(md_tag)::value;
#pragma unroll 1
        for (int ly = 0; ly < MD; ++ly)
#pragma unroll
            for (int lx = 0; lx < MD; ++lx) {
                const int l = in0 + lx + MD * ly;
                const T x00 = n00[l], x10 = n00[NIP + l], x01 = n00[NXT * NIP + l], x11 = n00[(NXT + 1) * NIP + l];
                const T p = x00 + x10, q = x00 - x10, r = x01 + x11, t = x01 - x11;
                const bool ly_odd = (ly & 1) != 0;
                T Sv[4];
                Sv[0] = ly_odd ? p - r : p + r;
                Sv[1] = ly_odd ? q - t : q + t;
                Sv[2] = ly_odd ? p + r : p - r;
                Sv[3] = ly_odd ? q + t : q - t;
                const ConstPtr g = G + (int64_t)l * NO;
#pragma unroll
                for (int o = 0; o < NO; ++o) acc[o] += g[o] * Sv[((opar(o, 0) + lx) & 1) + 2 * opar(o, 1)];
            }
    };
    block(std::integral_constant<int, MU>{}, 0);
    if constexpr (!CONS) block(std::integral_constant<int, MV>{}, NU);
    __syncthreads(); // every lane is done with the nodes: the outputs reuse the LDS

#pragma unroll
    for (int o = 0; o < NO; ++o) sm[tid * NOP + o] = acc[o];
    __syncthreads();

    // ---- coalesced stores of the tile's rows (conservative: u_new = 2 S - u_old), row by
    //      row, each thread keeping the same (cell column, coefficient) slots ----
    auto put = [&](GOut dst, const GIn old, int nb_tag, auto nbc) {
        constexpr int NB = decltype(nbc)::value, PER_ROW = TX * NB;
        constexpr int SLOTS = (PER_ROW + DENSE_BLOCK - 1) / DENSE_BLOCK;
        const int base = nb_tag;
        int gofs[SLOTS], sofs[SLOTS];
        bool okx[SLOTS];
#pragma unroll
        for (int k = 0; k < SLOTS; ++k) {
            const int e = tid + k * DENSE_BLOCK;
            const int xx = e / NB, o = e - xx * NB;
            okx[k] = e < PER_ROW && x0 + xx < a.ext_to[0];
            gofs[k] = (x0 + xx) * NB + o;
            sofs[k] = xx * NOP + base + o;
        }
        // conservative: the old level of a group of rows is read before any of its stores
        constexpr int RG = !CONS ? 1 : (SLOTS >= 32 ? 1 : (32 / SLOTS < TY ? 32 / SLOTS : TY));
        for (int yg = 0; yg < TY; yg += RG) {
            T ov[RG][SLOTS];
            if constexpr (CONS) {
#pragma unroll
                for (int r = 0; r < RG; ++r) {
                    const int gy = y0 + yg + r;
                    if (yg + r >= TY || gy >= a.ext_to[1]) break;
                    const int64_t rb = (int64_t)gy * a.ext_to[0] * NB;
#pragma unroll
                    for (int k = 0; k < SLOTS; ++k)
                        if (okx[k]) ov[r][k] = old[rb + gofs[k]];
                }
            }
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                const int gy = y0 + yg + r;
                if (yg + r >= TY || gy >= a.ext_to[1]) break;
                const int64_t rb = (int64_t)gy * a.ext_to[0] * NB;
#pragma unroll
                for (int k = 0; k < SLOTS; ++k) {
                    if (!okx[k]) continue;
                    const T sv = sm[(yg + r) * TX * NOP + sofs[k]];
                    if constexpr (CONS) dst[rb + gofs[k]] = T(2) * sv - ov[r][k];
                    else dst[rb + gofs[k]] = sv;
                }
            }
        }
    };
    put(reinterpret_cast<GOut>(reinterpret_cast<uintptr_t>(a.u_out)),
        reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.u_old)), 0, std::integral_constant<int, NU>{});
    if constexpr (!CONS)
        put(reinterpret_cast<GOut>(reinterpret_cast<uintptr_t>(a.v_out)), nullptr, NU,
            std::integral_constant<int, NV>{});
}

// Row-chunked staged form (for large nodes, whose whole records would not fit in LDS): the
// tile's nodes are staged one coefficient row at a time (the MD values l_x = 0..MD-1 of
// one l_y of the u or v block: contiguous in the node record), double-buffered, each
// chunk's loads issued before the previous chunk is computed; the lanes accumulate every
// output over all chunks in registers and store their cell's outputs directly.
template <typename T, int MU, bool CONS>
struct ChunkShape {
    static constexpr int MV = CONS ? 0 : MU - 1;
    static constexpr int CW = MU | 1; // odd node stride of a chunk row in LDS
    static constexpr size_t lds_words(int tx) { return (size_t)2 * (tx + 1) * (DENSE_BLOCK / tx + 1) * CW; }
};

template <typename T, int MU, bool CONS, int TX>
__device__ void dense_tile_chunked(const DenseArgs& a, int x0, int y0, T* __restrict__ sm)
{
    using CS = ChunkShape<T, MU, CONS>;
    constexpr int TY = DENSE_BLOCK / TX, NXT = TX + 1, NYT = TY + 1, CW = CS::CW;
    constexpr int MV = CS::MV, NU = MU * MU, NV = MV * MV, NO = NU + NV, BUF = NYT * NXT * CW;
    constexpr int SU = (NXT * MU + DENSE_BLOCK - 1) / DENSE_BLOCK;         // slots per row, u chunks
    constexpr int SV = MV > 0 ? (NXT * MV + DENSE_BLOCK - 1) / DENSE_BLOCK : 1; // v chunks
    constexpr int SL = SU > SV ? SU : SV;
    typedef const __attribute__((address_space(1))) T* GIn;
    typedef __attribute__((address_space(1))) T* GOut;
    typedef const __attribute__((address_space(4))) T* ConstPtr;
    const int tid = threadIdx.x;
    const int off = a.to_grid == 1 ? 0 : -1;
    const int ex0 = a.ext_from[0], ex1 = a.ext_from[1];
    const GIn uin = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.u_in));
    const GIn vin = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.v_in));

    // node rows of the tile (shared by every chunk) and, per block, the thread's slots
    int rowbase[NYT];
    bool rowghost[NYT];
#pragma unroll
    for (int r = 0; r < NYT; ++r) {
        bool g;
        rowbase[r] = wrap_node(y0 + r + off, ex1, a.bc[1], g) * ex0;
        rowghost[r] = g;
    }
    struct Slots {
        int node[SL], dst[SL], lx[SL];
        bool on[SL], negx[SL];
    };
    auto slots_of = [&](auto md_tag) {
        constexpr int MD = decltype(md_tag)::value, PER_ROW = NXT * MD;
        Slots sl;
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            const int e = tid + k * DENSE_BLOCK;
            const int xx = e / MD, lx = e - xx * MD;
            bool gxg;
            sl.node[k] = wrap_node(x0 + xx + off, ex0, a.bc[0], gxg);
            sl.dst[k] = xx * CW + lx;
            sl.lx[k] = lx;
            sl.on[k] = e < PER_ROW;
            sl.negx[k] = gxg && flips(a.bc[0], lx);
        }
        return sl;
    };
    const Slots su = slots_of(std::integral_constant<int, MU>{});
    const Slots sv = slots_of(std::integral_constant<int, (MV > 0 ? MV : 1)>{});

    T v[NYT][SL];
    // chunk loads into registers (row ly of the u or v block)
    auto load = [&](bool ublk, int ly) {
        const GIn src = ublk ? uin : vin;
        const int md = ublk ? MU : MV, nb = ublk ? NU : NV;
        const Slots& sl = ublk ? su : sv;
#pragma unroll
        for (int r = 0; r < NYT; ++r)
#pragma unroll
            for (int k = 0; k < SL; ++k)
                if (sl.on[k]) v[r][k] = src[((int64_t)rowbase[r] + sl.node[k]) * nb + ly * md + sl.lx[k]];
    };
    auto put = [&](bool ublk, int ly, T* buf) {
        const Slots& sl = ublk ? su : sv;
        const bool yflip = flips(a.bc[1], ly);
#pragma unroll
        for (int r = 0; r < NYT; ++r)
#pragma unroll
            for (int k = 0; k < SL; ++k)
                if (sl.on[k]) {
                    const bool neg = sl.negx[k] != (rowghost[r] && yflip);
                    buf[r * NXT * CW + sl.dst[k]] = neg ? -v[r][k] : v[r][k];
                }
    };

    const int tx = tid % TX, ty = tid / TX;
    const ConstPtr G = reinterpret_cast<ConstPtr>(reinterpret_cast<uintptr_t>(a.G));
    T acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) acc[o] = T(0);
    auto opar = [](int o, int i) {
        const int md = o < NU ? MU : MV, oo = o < NU ? o : o - NU;
        return (i == 0 ? oo % md : (oo / md) % md) & 1;
    };
    // products of one chunk: inputs l = in0 + MD ly + l_x
    auto compute = [&](auto md_tag, int in0, int ly, const T* buf) {
        constexpr int MD = decltype(md_tag)::value;
        const T* __restrict__ n00 = buf + (ty * NXT + tx) * CW;
        const bool ly_odd = (ly & 1) != 0;
#pragma unroll
        for (int lx = 0; lx < MD; ++lx) {
            const T x00 = n00[lx], x10 = n00[CW + lx], x01 = n00[NXT * CW + lx], x11 = n00[(NXT + 1) * CW + lx];
            const T p = x00 + x10, q = x00 - x10, r = x01 + x11, t = x01 - x11;
            T Sv[4];
            Sv[0] = ly_odd ? p - r : p + r;
            Sv[1] = ly_odd ? q - t : q + t;
            Sv[2] = ly_odd ? p + r : p - r;
            Sv[3] = ly_odd ? q + t : q - t;
            const ConstPtr g = G + (int64_t)(in0 + MD * ly + lx) * NO;
#pragma unroll
            for (int o = 0; o < NO; ++o) acc[o] += g[o] * Sv[((opar(o, 0) + lx) & 1) + 2 * opar(o, 1)];
        }
    };

    // chunks 0 .. MU-1: u rows, MU .. MU+MV-1: v rows; buffer c & 1
    constexpr int NCH = MU + MV;
    load(true, 0);
#pragma unroll 1
    for (int c = 0; c < NCH; ++c) {
        T* buf = sm + (c & 1) * BUF;
        const bool ublk = c < MU;
        const int ly = ublk ? c : c - MU;
        put(ublk, ly, buf);
        if (c + 1 < NCH) load(c + 1 < MU, c + 1 < MU ? c + 1 : c + 1 - MU);
        __syncthreads();
        if (ublk) compute(std::integral_constant<int, MU>{}, 0, ly, buf);
        else if constexpr (MV > 0) compute(std::integral_constant<int, (MV > 0 ? MV : 1)>{}, NU, ly, buf);
    }

    // outputs: each lane stores its cell's (conservative: old level read in chunks of 16
    // before their stores)
    const int gx = x0 + tx, gy = y0 + ty;
    if (gx >= a.ext_to[0] || gy >= a.ext_to[1]) return;
    const int64_t cell = (int64_t)gy * a.ext_to[0] + gx;
    const GOut __restrict__ uo = reinterpret_cast<GOut>(reinterpret_cast<uintptr_t>(a.u_out)) + cell * NU;
    if constexpr (CONS) {
        const GIn __restrict__ old = reinterpret_cast<GIn>(reinterpret_cast<uintptr_t>(a.u_old)) + cell * NU;
        constexpr int CH = 16;
#pragma unroll
        for (int o0 = 0; o0 < NU; o0 += CH) {
            T ov[CH];
#pragma unroll
            for (int j = 0; j < CH; ++j)
                if (o0 + j < NU) ov[j] = old[o0 + j];
#pragma unroll
            for (int j = 0; j < CH; ++j)
                if (o0 + j < NU) uo[o0 + j] = T(2) * acc[o0 + j] - ov[j];
        }
    } else {
        const GOut __restrict__ vo = reinterpret_cast<GOut>(reinterpret_cast<uintptr_t>(a.v_out)) + cell * NV;
#pragma unroll
        for (int o = 0; o < NU; ++o) uo[o] = acc[o];
#pragma unroll
        for (int o = 0; o < NV; ++o) vo[o] = acc[NU + o];
    }
}

template <typename T, int MU, bool CONS, int TX, int FORM>
__global__ void __launch_bounds__(DENSE_BLOCK) k_dense_staged(DenseArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tiles_x = (a.ext_to[0] + TX - 1) / TX;
    const int x0 = (blockIdx.x % tiles_x) * TX, y0 = (blockIdx.x / tiles_x) * (DENSE_BLOCK / TX);
    if constexpr (FORM == 1) dense_tile_staged<T, MU, CONS, TX>(a, x0, y0, reinterpret_cast<T*>(smem_raw));
    else dense_tile_chunked<T, MU, CONS, TX>(a, x0, y0, reinterpret_cast<T*>(smem_raw));
}

// The batched launches run one workgroup per item of a work list (launched as 8 x
// ceil(n / 8) workgroups): workgroup b runs on XCD b mod 8, and the workgroups of one XCD
// take a contiguous part of the list (the items of a problem are contiguous), so items
// that share halo rows of input nodes share that XCD's L2.  (A persistent loop over items
// holds an item's loop-invariant values across items: up to a hundred more registers.)
__device__ inline int list_item(int n_items)
{
    const int b = blockIdx.x;
    return (b % 8) * ((n_items + 7) / 8) + b / 8;
}

template <typename T, int MU, bool CONS, int TX, int FORM>
__global__ void __launch_bounds__(DENSE_BLOCK) k_dense_staged_list(const DenseArgs* __restrict__ probs,
                                                                   const int4* __restrict__ tiles, int n_tiles)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int t = list_item(n_tiles);
    if (t >= n_tiles) return; // whole workgroup
    const int4 tl = tiles[t];
    const int pi = __builtin_amdgcn_readfirstlane(tl.x);
    const int x0 = __builtin_amdgcn_readfirstlane(tl.y), y0 = __builtin_amdgcn_readfirstlane(tl.z);
    const DenseArgs a = probs[pi];
    if constexpr (FORM == 1) dense_tile_staged<T, MU, CONS, TX>(a, x0, y0, reinterpret_cast<T*>(smem_raw));
    else dense_tile_chunked<T, MU, CONS, TX>(a, x0, y0, reinterpret_cast<T*>(smem_raw));
}

// many 2-D problems of one (m, method): one workgroup per item of a work list of tiles
// (problem, x0, y0) of TX x (256 / TX) cells (TX = that problem's tile_x).
template <typename T, int MU, bool CONS>
__global__ void __launch_bounds__(DENSE_BLOCK) k_dense_list(const DenseArgs* __restrict__ probs,
                                                            const int4* __restrict__ tiles, int n_tiles)
{
    const int t = list_item(n_tiles);
    if (t >= n_tiles) return; // whole workgroup
    // the tile and its problem are the same for the whole workgroup: read them as
    // wave-uniform values, so that the descriptor and the cell map G stay on the scalar
    // unit as in the single-problem kernel
    const int4 tl = tiles[t];
    const int pi = __builtin_amdgcn_readfirstlane(tl.x);
    const int x0 = __builtin_amdgcn_readfirstlane(tl.y), y0 = __builtin_amdgcn_readfirstlane(tl.z);
    const DenseArgs a = probs[pi];
    const int tx = a.tile_x;
    const int x = x0 + (int)threadIdx.x % tx;
    const int y = y0 + (int)threadIdx.x / tx;
    if (x < a.ext_to[0] && y < a.ext_to[1]) dense_cell<T, 2, MU, CONS>(a, x + (int64_t)a.ext_to[0] * y);
}

// the staged form's LDS: at most the 160 KB of a CU
constexpr size_t kMaxLds = 160 * 1024;

template <typename T, int MU, bool CONS, int FORM>
size_t staged_lds(int tx)
{
    return (FORM == 1 ? StagedShape<T, MU, CONS>::lds_words(tx) : ChunkShape<T, MU, CONS>::lds_words(tx)) * sizeof(T);
}

template <typename T, int MU, bool CONS, int TX, int FORM>
hipError_t launch_staged(const DenseArgs& a, hipStream_t st)
{
    const size_t lds = staged_lds<T, MU, CONS, FORM>(TX);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = k_dense_staged<T, MU, CONS, TX, FORM>;
    hipError_t e = hw_lds_limit<k_dense_staged<T, MU, CONS, TX, FORM>>(lds);
    if (e != hipSuccess) return e;
    const int blocks = ((a.ext_to[0] + TX - 1) / TX) * ((a.ext_to[1] + DENSE_BLOCK / TX - 1) / (DENSE_BLOCK / TX));
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(DENSE_BLOCK), lds, st, a);
    return hipGetLastError();
}

template <typename T, int D, int MU, bool CONS>
hipError_t launch(const DenseArgs& a, hipStream_t st)
{
    if constexpr (D == 2) {
        if (a.staged == 1) {
            if (a.tile_x == 32) return launch_staged<T, MU, CONS, 32, 1>(a, st);
            if (a.tile_x == 64) return launch_staged<T, MU, CONS, 64, 1>(a, st);
            return hipErrorInvalidValue;
        }
        if (a.staged == 2) {
            if (a.tile_x == 32) return launch_staged<T, MU, CONS, 32, 2>(a, st);
            if (a.tile_x == 64) return launch_staged<T, MU, CONS, 64, 2>(a, st);
            return hipErrorInvalidValue;
        }
    }
    const int tx = a.tile_x;
    const int64_t blocks = D == 1 ? (a.n_cells + DENSE_BLOCK - 1) / DENSE_BLOCK
                                  : (int64_t)((a.ext_to[0] + tx - 1) / tx) *
                                        ((a.ext_to[1] + DENSE_BLOCK / tx - 1) / (DENSE_BLOCK / tx));
    hipLaunchKernelGGL((k_dense<T, D, MU, CONS>), dim3((unsigned)blocks), dim3(DENSE_BLOCK), 0, st, a);
    return hipGetLastError();
}

template <typename T, int MU, bool CONS, int TX, int FORM>
hipError_t launch_staged_list(const DenseArgs* probs, const int4* tiles, int n_tiles, hipStream_t st)
{
    const size_t lds = staged_lds<T, MU, CONS, FORM>(TX);
    if (lds > kMaxLds) return hipErrorInvalidValue;
    auto kern = k_dense_staged_list<T, MU, CONS, TX, FORM>;
    hipError_t e = hw_lds_limit<k_dense_staged_list<T, MU, CONS, TX, FORM>>(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(8 * ((n_tiles + 7) / 8)), dim3(DENSE_BLOCK), lds, st, probs, tiles, n_tiles);
    return hipGetLastError();
}

template <typename T, int MU, bool CONS>
hipError_t launch_list(const DenseArgs* probs, const int4* tiles, int n_tiles, int staged_tx, hipStream_t st)
{
    switch (staged_tx) {
    case 0: break;
    case 32: return launch_staged_list<T, MU, CONS, 32, 1>(probs, tiles, n_tiles, st);
    case 64: return launch_staged_list<T, MU, CONS, 64, 1>(probs, tiles, n_tiles, st);
    case 1032: return launch_staged_list<T, MU, CONS, 32, 2>(probs, tiles, n_tiles, st);
    case 1064: return launch_staged_list<T, MU, CONS, 64, 2>(probs, tiles, n_tiles, st);
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_dense_list<T, MU, CONS>), dim3(8 * ((n_tiles + 7) / 8)), dim3(DENSE_BLOCK), 0, st, probs, tiles,
                       n_tiles);
    return hipGetLastError();
}

template <typename T>
hipError_t dispatch_list(const DenseArgs* probs, const int4* tiles, int n_tiles, int m, bool cons, int staged_tx,
                         hipStream_t st)
{
    if (cons) {
        switch (m) {
        case 0: return launch_list<T, 1, true>(probs, tiles, n_tiles, staged_tx, st);
        case 1: return launch_list<T, 2, true>(probs, tiles, n_tiles, staged_tx, st);
        case 2: return launch_list<T, 3, true>(probs, tiles, n_tiles, staged_tx, st);
        case 3: return launch_list<T, 4, true>(probs, tiles, n_tiles, staged_tx, st);
        case 4: return launch_list<T, 5, true>(probs, tiles, n_tiles, staged_tx, st);
        case 5: return launch_list<T, 6, true>(probs, tiles, n_tiles, staged_tx, st);
        case 6: return launch_list<T, 7, true>(probs, tiles, n_tiles, staged_tx, st);
        }
    } else {
        switch (m) {
        case 1: return launch_list<T, 2, false>(probs, tiles, n_tiles, staged_tx, st);
        case 2: return launch_list<T, 3, false>(probs, tiles, n_tiles, staged_tx, st);
        case 3: return launch_list<T, 4, false>(probs, tiles, n_tiles, staged_tx, st);
        case 4: return launch_list<T, 5, false>(probs, tiles, n_tiles, staged_tx, st);
        case 5: return launch_list<T, 6, false>(probs, tiles, n_tiles, staged_tx, st);
        case 6: return launch_list<T, 7, false>(probs, tiles, n_tiles, staged_tx, st);
        }
    }
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch(const DenseArgs& a, int d, int m, bool cons, hipStream_t st)
{
    if (d == 1) {
        if (cons) {
            switch (m) {
            case 0: return launch<T, 1, 1, true>(a, st);
            case 1: return launch<T, 1, 2, true>(a, st);
            case 2: return launch<T, 1, 3, true>(a, st);
            case 3: return launch<T, 1, 4, true>(a, st);
            case 4: return launch<T, 1, 5, true>(a, st);
            case 5: return launch<T, 1, 6, true>(a, st);
            case 6: return launch<T, 1, 7, true>(a, st);
            }
        } else {
            switch (m) {
            case 1: return launch<T, 1, 2, false>(a, st);
            case 2: return launch<T, 1, 3, false>(a, st);
            case 3: return launch<T, 1, 4, false>(a, st);
            case 4: return launch<T, 1, 5, false>(a, st);
            case 5: return launch<T, 1, 6, false>(a, st);
            case 6: return launch<T, 1, 7, false>(a, st);
            }
        }
    } else if (d == 2) {
        if (cons) {
            switch (m) {
            case 0: return launch<T, 2, 1, true>(a, st);
            case 1: return launch<T, 2, 2, true>(a, st);
            case 2: return launch<T, 2, 3, true>(a, st);
            case 3: return launch<T, 2, 4, true>(a, st);
            case 4: return launch<T, 2, 5, true>(a, st);
            case 5: return launch<T, 2, 6, true>(a, st);
            }
        } else {
            switch (m) {
            case 1: return launch<T, 2, 2, false>(a, st);
            case 2: return launch<T, 2, 3, false>(a, st);
            case 3: return launch<T, 2, 4, false>(a, st);
            case 4: return launch<T, 2, 5, false>(a, st);
            case 5: return launch<T, 2, 6, false>(a, st);
            case 6: return launch<T, 2, 7, false>(a, st);
            }
        }
    }
    return hipErrorInvalidValue;
}

} // namespace

bool hw_dense_staged_fits(int m, bool cons, bool fp64, int tx, int form)
{
    if (m < 0 || m > 6 || (!cons && m < 1) || (tx != 32 && tx != 64) || form < 1 || form > 2) return false;
    const int mu = m + 1, mv = cons ? 0 : m;
    const size_t nodes = (size_t)(tx + 1) * (DENSE_BLOCK / tx + 1);
    size_t words;
    if (form == 1) {
        const size_t nip = (size_t)(mu * mu + mv * mv) | 1;
        words = std::max(nodes * nip, (size_t)DENSE_BLOCK * nip);
    } else {
        words = 2 * nodes * (size_t)(mu | 1);
    }
    return words * (fp64 ? 8 : 4) <= kMaxLds;
}

hipError_t hw_launch_dense_list(const DenseArgs* probs, const int4* tiles, int n_tiles, int m, bool cons, bool fp64,
                                int staged_tx, hipStream_t st)
{
    if (n_tiles <= 0) return hipSuccess;
    if (n_tiles > INT32_MAX - 7) return hipErrorInvalidValue;
    return fp64 ? dispatch_list<double>(probs, tiles, n_tiles, m, cons, staged_tx, st)
                : dispatch_list<float>(probs, tiles, n_tiles, m, cons, staged_tx, st);
}

hipError_t hw_launch_dense1d_steps(const DenseArgs* args, int k0, int n_half, int m, bool cons, bool fp64,
                                   hipStream_t st)
{
    if (!args || k0 < 0 || k0 > 3 || n_half < 0 || n_half > INT32_MAX - 4) return hipErrorInvalidValue;
    if (n_half == 0) return hipSuccess;
    return fp64 ? dispatch_1d_steps<double>(args, k0, n_half, m, cons, st)
                : dispatch_1d_steps<float>(args, k0, n_half, m, cons, st);
}

hipError_t hw_launch_dense(const DenseArgs& a, int d, int m, bool cons, bool fp64, hipStream_t st)
{
    if (!a.G || a.n_cells < 0) return hipErrorInvalidValue;
    if (d == 2 && (a.tile_x < 1 || a.tile_x > DENSE_BLOCK || DENSE_BLOCK % a.tile_x)) return hipErrorInvalidValue;
    if (a.staged && (d != 2 || a.staged < 1 || a.staged > 2 || (a.tile_x != 32 && a.tile_x != 64)))
        return hipErrorInvalidValue;
    if (a.n_cells == 0) return hipSuccess;
    for (int i = 0; i < d; ++i)
        if (a.ext_to[i] < 1 || a.ext_from[i] < 1) return hipErrorInvalidValue;
    return fp64 ? dispatch<double>(a, d, m, cons, st) : dispatch<float>(a, d, m, cons, st);
}
