// Host-side declarations of the kernel launchers of libhermite_wave.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hw_device.h"
#include "../../include/hermite_wave.h"

#include <atomic>
#include <functional>
#include <string>
#include <vector>

size_t hw_generic_lds_bytes(int d, int m, int variant, int elem_size);
size_t hw_energy_lds_bytes(int d, int m);

hipError_t hw_launch_generic(int d, bool fp64, const ProblemDesc* descs, const int64_t* prefix,
                             int nprob, int64_t total, const void* ops, size_t lds, int grid,
                             hipStream_t st, const ForcingArgs* forcing = nullptr);
hipError_t hw_launch_energy(int d, bool fp64, const EnergyDesc& E, const double* dops,
                            double* partials, int grid, hipStream_t st);
hipError_t hw_launch_convert(const void* src, bool src64, void* dst, bool dst64, int64_t n,
                             hipStream_t st);
// Energy without allocation: both passes' partial sums go to a file-scope device array
// of 2 x HW_ENERGY_MAX_GROUPS doubles (one per GPU); a final one-workgroup kernel writes
// E = 2 (pass 0 - pass 1) to e_out (device).  Calls that overlap on one GPU race on the
// array.  hipErrorInvalidValue for a grid outside 1..HW_ENERGY_MAX_GROUPS.
constexpr int HW_ENERGY_MAX_GROUPS = 2048;
constexpr int HW_MAX_DEVICES = 64;

// Raises kernel K's dynamic LDS limit (hipFuncSetAttribute) only when a launch needs more than
// the limit already set for K on the current device, so that launches in a loop or while a
// graph is captured do not repeat the call.
template <auto K>
inline hipError_t hw_lds_limit(size_t bytes)
{
    static std::atomic<int> set_bytes[HW_MAX_DEVICES];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= HW_MAX_DEVICES)
        return hipFuncSetAttribute((const void*)K, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if ((int)bytes <= set_bytes[dev].load(std::memory_order_acquire)) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute((const void*)K, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) {
        int cur = set_bytes[dev].load(std::memory_order_relaxed);
        while ((int)bytes > cur && !set_bytes[dev].compare_exchange_weak(cur, (int)bytes)) {
        }
    }
    return e;
}
hipError_t hw_launch_energy_noalloc(int d, bool fp64, const EnergyDesc& E0, int grid0, const EnergyDesc& E1,
                                    int grid1, const double* dops, double* e_out, hipStream_t st);

// LDS-tiled MFMA kernel for the 3-D dissipative full method with m = 3 (periodic or
// not).  Returns hipErrorInvalidValue when the problem is outside its scope.
struct TiledArgs {
    int ext_from[3], ext_to[3], bc[3], to_grid;
    const void* u_in;
    const void* v_in;
    void* u_out;
    void* v_out;
    double tau, lam2[3];
    const void* tables;           // from hw_tiled_tables_create / hw_cmap3d_tables_create
    const void* u_old = nullptr;  // composed-map kernel, conservative: old level on the grid written
    int cons = 0;                 // composed-map kernel: 1 = conservative method
};
// Per-lane dense kernel for d <= 2 (kernel_dense.hip): each output node is the product
// of the problem's cell matrix G (hw_cell_map, FP64 on the host, uploaded in the state
// precision) with its 2^d corner nodes; ghost corners mirrored as in the other kernels.
struct DenseArgs {
    int ext_from[3], ext_to[3], bc[3], to_grid;
    const void* u_in;
    const void* v_in;  // dissipative
    const void* u_old; // conservative: old level on the grid written
    void* u_out;
    void* v_out;       // dissipative
    const void* G;     // rows of corner 0 of the cell matrix: [n_in / 2^d][n_out], input-major
    int64_t n_cells;
    int tile_x = 64;   // 2-D: cells along x of a workgroup's tile of 256 (a divisor of 256)
    int staged = 0;    // 2-D: 0 = per-lane gathers; LDS-staged forms (tile_x 32 or 64): 1 = whole
                       // node records, 2 = one coefficient row of every node at a time;
                       // 3 = the composed-map form on the matrix cores (kernel_cmap2d.hip)
    const void* cm2 = nullptr; // tables of the composed-map form (hw_cmap2d_tables_create)
};
bool hw_dense_supported(int d, int m, int method, int precision);


// The descriptor's time-sum weights (tau, lam2, F, cuQ, cuR, cvQ, cvR) for problem p with
// cell widths h (cellmap.cpp); the same tables serve every kernel.
void hw_fill_weights(const hw_problem& p, const double h[3], ProblemDesc& D);
void hw_cell_map(const ProblemDesc& D, std::vector<double>& G, int& n_in, int& n_out);
hipError_t hw_launch_dense(const DenseArgs& a, int d, int m, bool cons, bool fp64, hipStream_t st);
// n_half consecutive half steps of one 1-D problem in one launch of one workgroup, half step
// k0 + j (k0 = the first one's index mod 4) with the device arguments
// args[((k0 + j) & 1) * 2 + (((k0 + j) >> 1) & 1)]; for problems of a few hundred cells
hipError_t hw_launch_dense1d_steps(const DenseArgs* args, int k0, int n_half, int m, bool cons, bool fp64,
                                   hipStream_t st);
// One launch over the tiles of many 2-D problems of one (m, method), one workgroup per
// tile: probs[i] are their descriptors, tiles {problem i, x0, y0, 0} of tile_x x
// (256 / tile_x) cells;
// staged_tx = 32 or 64 selects the LDS-staged form (whole node records) with tiles of
// that width, 1032 or 1064 the row-chunked staged form with tiles 32 or 64 wide, 0 the
// per-lane gather form.
hipError_t hw_launch_dense_list(const DenseArgs* probs, const int4* tiles, int n_tiles, int m, bool cons, bool fp64,
                                int staged_tx, hipStream_t st);
// whether staged form `form` (1 or 2) with tiles tx cells wide fits a CU's LDS for
// (m, method, precision)
bool hw_dense_staged_fits(int m, bool cons, bool fp64, int tx, int form);

// Composed-map MFMA kernel for 2-D problems, m = 3..6, both methods (kernel_cmap2d.hip):
// tables from corner 0's rows of the cell matrix (G0: [NI][NI], input-major, FP64); single
// problems in strips of 16 cells walking chunks of ry cell rows, or one launch over a work
// list of strips {problem, x0, cy0, cy1} of many problems of one (m, method), one
// workgroup per strip (the descriptors' cm2 fields name each problem's tables).
bool hw_cmap2d_supported(int m);
// whether a row of ext nodes of either grid fits the kernel's 32-bit byte offsets
bool hw_cmap2d_rows_fit(int m, bool cons, bool fp64, int64_t ext);
hipError_t hw_cmap2d_tables_create(const std::vector<double>& G0, int m, bool cons, bool fp64, void** out);
hipError_t hw_launch_cmap2d(const DenseArgs& a, int m, bool cons, bool fp64, int ry, hipStream_t st);
hipError_t hw_launch_cmap2d_list(const DenseArgs* probs, const int4* items, int n_items, int m, bool cons, bool fp64,
                                 hipStream_t st);

// Composed-map MFMA kernel for the 3-D dissipative and conservative methods, m = 3 (kernel_cmap3d.hip):
// the tables come from the problem's descriptor (cell matrix, hw_cell_map) and are
// passed in TiledArgs::tables.
hipError_t hw_cmap3d_tables_create(const ProblemDesc& D, bool fp64, void** out);
hipError_t hw_launch_cmap3d(const TiledArgs& a, bool fp64, hipStream_t st);

bool hw_tiled_supported(int d, int m, int method, int precision);
// Device tables of the kernel for one (precision, lam2, tau): the time-sum weights carry
// the scalings in lam2 and tau.  Allocates and uploads synchronously (call outside
// capture); the caller frees them with hw_tiled_tables_destroy.
hipError_t hw_tiled_tables_create(int precision, const double lam2[3], double tau, void** out);
void hw_tiled_tables_destroy(void* tables);
hipError_t hw_launch_tiled(const TiledArgs& a, int precision, hipStream_t st);

// Autotuner (tune.cpp): the candidate with the smallest time_us(candidate) for a key,
// timed once per process (or read from the HW_TUNE_CACHE file) and cached.
bool hw_tune_enabled();
int hw_tune_size_class(int64_t cells);
// the choice HW_TUNE_FORCE imposes on `kernel`, if any (also used to select a code path in
// tests, e.g. "cmap3d_offsets=64")
bool hw_tune_forced(const char* kernel, int& choice);
int hw_tune_choose(const char* kernel, int d, int m, int method, bool fp64, int size_class,
                   const std::vector<int>& candidates, const std::function<double(int)>& time_us);
std::string hw_tune_report_text();

// Peak probes (probes.hip): STREAM triad over FP64 arrays of n elements; independent MFMA
// chains over `groups` workgroups of 256 threads, `iters` rounds of 8 products per wave.
hipError_t hw_probe_triad_launch(double* a, const double* b, const double* c, int64_t n, hipStream_t st);
hipError_t hw_probe_mfma_launch(bool fp64, void* sink, int groups, int iters, hipStream_t st);
// mode 0: matrix-core products only, 1: vector FMAs only, 2: both in every wave
hipError_t hw_probe_coexec_launch(int mode, float* sink, int groups, int iters, hipStream_t st);
