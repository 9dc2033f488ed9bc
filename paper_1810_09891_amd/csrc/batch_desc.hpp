// Device-side description of a batch of plans: one PlanDev per plan (geometry, node data,
// workspace regions and FFT pass parameters), plus the per-call data pointers passed by
// value to the batched kernels.
#pragma once

#include "launch.hpp"

namespace nfft {

constexpr int kMaxBatch = 64;  // plans per batched launch (larger batches use several)

struct PlanDev {
    Geom g;
    Nodes nd;
    void *grid;      // forward grid
    void *grid_adj;  // adjoint grid
    void *scratch;   // spreading tiles
    int64_t ngrid;   // grid cells
    int nfft;        // FFT passes (= d)
    FftPass fwd[kMaxDim];  // forward passes with the batch's line packing
    FftPass adj[kMaxDim];  // adjoint passes
};

struct BatchPtrs {
    const void *in[kMaxBatch];
    void *out[kMaxBatch];
};

// Index of the plan owning flattened item `it`, given prefix[0..count] in LDS.
__device__ __forceinline__ int batch_find(const int *prefix, int count, int it)
{
    int lo = 0, hi = count;  // prefix[lo] <= it < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= it)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// prefix[0..count] of per-plan item counts, computed by the workgroup into LDS.
__device__ __forceinline__ void batch_prefix(int *prefix, int count, const int *counts_per_plan_lds)
{
    if (threadIdx.x == 0) {
        int acc = 0;
        prefix[0] = 0;
        for (int p = 0; p < count; ++p) {
            acc += counts_per_plan_lds[p];
            prefix[p + 1] = acc;
        }
    }
    __syncthreads();
}

// Dynamic work queue of a batched launch: queue[0] hands out item indices, queue[1]
// counts the workgroups that have finished; the last one resets both, so every launch
// starts from zero without a separate clearing step (a batch is used by one stream at a
// time, so launches on one queue never overlap).
__device__ __forceinline__ int queue_next(int *queue, int *s_item)
{
    __syncthreads();  // every thread has read the previous item
    if (threadIdx.x == 0)
        *s_item = atomicAdd(queue, 1);
    __syncthreads();
    return *s_item;
}

__device__ __forceinline__ void queue_done(int *queue)
{
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(queue + 1, 1) == (int)gridDim.x - 1) {
            atomicExch(queue, 0);
            atomicExch(queue + 1, 0);
        }
    }
}

}  // namespace nfft
