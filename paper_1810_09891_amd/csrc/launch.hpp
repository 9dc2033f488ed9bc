// Host-side launchers of the NFFT kernels (one definition per kernel file).  Every
// launcher enqueues on `stream` and returns hipGetLastError() of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nfft_device.hpp"

namespace nfft {

// ------------------------------------------------------------------ node precompute

// bin_count[0..nbins) = 0, counters[0..1] = 0.
hipError_t launch_node_reset(const Geom &g, const Nodes &nd, hipStream_t s);
// key, rank, bin_count, copy of x; non-finite flag in counters[1].
hipError_t launch_node_key(const Geom &g, const Nodes &nd, double *xcopy, hipStream_t s);
// bin_start, bin_chunk (exclusive scans), counters[0] = number of work items.
hipError_t launch_node_scan(const Geom &g, const Nodes &nd, hipStream_t s);
// sorted u, delta, perm; work-item lists.
hipError_t launch_node_scatter(const Geom &g, const Nodes &nd, bool dbl, hipStream_t s);

// ------------------------------------------------------------------ FFT passes

struct FftPass {
    void *grid;          // complex grid (in place)
    const void *fin;     // coefficients read by the first forward pass (mode 0)
    void *fout;          // coefficients written by the last adjoint pass (mode 2)
    const void *mul;     // optional factors (shape N, complex) applied in that write, or null
    const double *w[kMaxDim];  // deconvolution factors per dimension, centred index
    const void *tw;      // e^{-2 pi i k / L}, k < L, for the transformed dimension
    int d, t;            // dimension count, transformed dimension
    int L;               // n_t
    int N[kMaxDim], n[kMaxDim];
    int64_t stride[kMaxDim];  // grid strides (elements)
    int nl;              // lines per workgroup
    int pitch;           // LDS elements per line
    int in_mode;         // 0: coefficients with D, 1: grid, N_t nonzero entries, 2: grid, full line
    int out_mode;        // 0: full line to grid, 1: N_t entries to grid, 2: N_t entries to coefficients with D^H
    int sign;            // -1 forward, +1 adjoint
    int rows;            // 1 when t == d-1 (lines are contiguous rows)
    int64_t ngroups;     // line groups
    int nrows;           // rows (t == d-1): prod_{q<d-1} N_q
    int ncb;             // column blocks (t < d-1): n_{d-1} / nl
    int vpt;             // points per thread: max(1, nl*L/256)
    int pp;              // 1: radix stages alternate between two LDS line buffers (one barrier
                         // per stage), 0: in place (two barriers per stage)
};

// LDS bytes of one workgroup of an FFT pass: its line buffer(s), then the twiddles.
inline size_t fft_lds_bytes(const FftPass &p, size_t cs)
{
    return ((size_t)(p.pp ? 2 : 1) * p.nl * p.pitch + p.L) * cs;
}
// Two line buffers when they and the twiddles fit in 64 KB (two or more workgroups per CU).
inline void fft_choose_buffers(FftPass &p, size_t cs)
{
    p.pp = 1;
    if (fft_lds_bytes(p, cs) > 65536)
        p.pp = 0;
}
hipError_t launch_fft_pass(const FftPass &p, bool dbl, int grid_blocks, hipStream_t s);

// ------------------------------------------------------------------ window kernels

hipError_t launch_interp(const Geom &g, const Nodes &nd, bool dbl, const void *grid, void *f, int blocks,
                         size_t lds, hipStream_t s);
hipError_t launch_spread_tiles(const Geom &g, const Nodes &nd, bool dbl, const void *f, void *scratch,
                               int blocks, size_t lds, hipStream_t s);
hipError_t launch_fold(const Geom &g, const Nodes &nd, bool dbl, const void *scratch, void *grid,
                       hipStream_t s);
hipError_t launch_grad_x(const Geom &g, const Nodes &nd, bool dbl, const void *grid, const void *v,
                         void *grad, int blocks, size_t lds, hipStream_t s);

// Owner-computes spreading of 3-D plans (Geom::own): every tile's entries (the nodes whose
// stencils reach it), tile entry offsets and work items (counters[2] = number of items), run
// in the node precomputation.
hipError_t launch_own_items(const Geom &g, const Nodes &nd, hipStream_t s);
// Every output tile's cells summed over the nodes whose stencils reach it; tiles with one
// work item are written to `grid`, split tiles to per-item slots of `scratch` (tile cells
// each), which launch_own_fold then sums in item order into `grid`.  `fs` (M complex)
// receives the node values in sorted order.
hipError_t launch_spread_own(const Geom &g, const Nodes &nd, bool dbl, const void *f, void *fs, void *grid,
                             void *scratch, int max_items, hipStream_t s);
hipError_t launch_own_fold(const Geom &g, const Nodes &nd, bool dbl, const void *scratch, void *grid,
                           hipStream_t s);

// Tile edges of the owner-computes spreading: along dimension 0 (registers per lane) and
// along dimensions 1 and 2 (four 8 x 8 lane blocks).
constexpr int kOwnTile0 = 16;
constexpr int kOwnTile12 = 16;
constexpr int kOwnMaxRanges = 512;  // contiguous node ranges of one tile's list

// LDS bytes per workgroup of the interpolation / spreading / gradient kernels.
size_t interp_lds_bytes(const Geom &g, bool dbl);
// LDS of one spreading launch for a single plan (in-register 2-D kernel or tile kernel)
size_t spread_lds_bytes(const Geom &g, bool dbl);
// LDS of the tile kernel (the batched spreading launch always uses it)
size_t spread_batch_lds_bytes(const Geom &g, bool dbl);
// Whether single-plan spreading uses the in-register 2-D kernel: d = 2, 2m+2 equal to the
// compiled stencil width (even m), bins of 32 x 32 (complex64) or 16 x 32 (complex128)
// cells, padded tile width at most 64.
bool spread_in_registers(const Geom &g, bool dbl);
// Largest number of (bin, offset) pairs a grid index can have in one dimension; the
// fold kernel supports up to kFoldMaxPairs.
constexpr int kFoldMaxPairs = 24;
int fold_max_pairs(const Geom &g, int t);

// ------------------------------------------------------------------ batched launches
//
// One launch covers pass / step of every plan in `plans` (a device array of `count`
// PlanDev, count <= kMaxBatch, all with the same d, compiled width WMv and precision).
// The interpolation and spreading kernels take work items from the queue `queue`
// (two ints, zero between launches).

struct PlanDev;
struct BatchPtrs;
hipError_t launch_fft_batch(const PlanDev *plans, int count, int pass, bool forward, const BatchPtrs &ptrs,
                            bool dbl, bool mix, int vpt, int blocks, size_t lds, hipStream_t s);
hipError_t launch_interp_batch(const PlanDev *plans, int count, const BatchPtrs &ptrs, int *queue, int d,
                               bool dbl, int WMv, int blocks, size_t lds, hipStream_t s);
hipError_t launch_spread_batch(const PlanDev *plans, int count, const BatchPtrs &ptrs, int *queue, int d,
                               bool dbl, int WMv, int blocks, size_t lds, hipStream_t s);
// Batched 2-D spreading with tile columns in registers (every plan of the group must satisfy
// spread_in_registers; LDS as spread_lds_bytes).
hipError_t launch_spread_cols_batch(const PlanDev *plans, int count, const BatchPtrs &ptrs, int *queue, bool dbl,
                                    int WMv, int blocks, size_t lds, hipStream_t s);
hipError_t launch_fold_batch(const PlanDev *plans, int count, int d, bool dbl, int blocks, hipStream_t s);

// ------------------------------------------------------------------ direct sums

struct NdftArgs {
    int d;
    int N[kMaxDim];
    int64_t M;
    int64_t K;  // prod N
    const double *x;
    const void *in;
    void *out;
};
hipError_t launch_ndft(const NdftArgs &a, bool dbl, bool adjoint, hipStream_t s);

// ------------------------------------------------------------------ utilities

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_fill_lin(const Geom &g, int t, bool dbl, void *tab, void *dtab, hipStream_t s);

}  // namespace nfft
