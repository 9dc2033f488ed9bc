// Node precomputation (the node setting step that Sec. 4.2 times as "precomputation"):
// per node and dimension, in FP64, y = n_t x_t, u = floor(y) mod n_t and delta = y - floor(y)
// (the stencil index set of Sec. 2 eq. (2.13) starts at u - m), then a counting sort of
// the nodes into bins of B_0 x ... x B_{d-1} grid cells and the list of work items
// (chunks of at most chunk_cap nodes of one bin) the window kernels iterate over.
#include <math.h>

#include "launch.hpp"

namespace nfft {

namespace {

__global__ void k_node_reset(int32_t *bin_count, int nbins, int32_t *counters)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nbins)
        bin_count[i] = 0;
    if (i < 2)
        counters[i] = 0;
}

// Grid index and offset of coordinate x in a dimension of length n.  Returns false for
// non-finite input (index 0, offset NaN).  n * x is exact for a power-of-two n, floor is
// exact, and y - floor(y) is exact, so u and delta are the exact values.  fmod is exact
// too, so the index is right for any finite x.
__device__ __forceinline__ bool node_index(double x, int n, int &u, double &delta)
{
    double y = (double)n * x;
    if (!isfinite(y)) {
        u = 0;
        delta = __builtin_nan("");
        return false;
    }
    double fl = floor(y);
    delta = y - fl;
    double r = fmod(fl, (double)n);
    if (r < 0.0)
        r += (double)n;
    u = (int)r;
    if (u >= n)  // r == n cannot occur for exact fmod, kept as a guard
        u -= n;
    return true;
}

template <int D> __global__ __launch_bounds__(kBlock) void k_node_key(Geom g, Nodes nd, double *xcopy)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nd.M)
        return;
    int bin = 0;
    bool finite = true;
#pragma unroll
    for (int t = 0; t < D; ++t) {
        double x = nd.x[j * D + t];
        xcopy[j * D + t] = x;
        int u;
        double delta;
        finite &= node_index(x, g.n[t], u, delta);
        bin = bin * g.nb[t] + (u >> g.lgB[t]);
    }
    if (!finite)
        atomicOr(&nd.counters[1], 1);
    nd.key[j] = bin;
    // A slot in the bin: one atomic per distinct bin of the wave (lanes of a wave often
    // share a bin), the lanes of a bin numbered by lane order.  The slots only place the
    // node inside its bin's range; the order inside the range is fixed afterwards by
    // sorting it by caller index, so the final order does not depend on the atomics.
    const uint64_t active = __ballot(1);
    const int lane = __lane_id();
    uint64_t todo = active;
    int slot = 0;
    while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int lbin = __shfl(bin, leader);
        const uint64_t same = __ballot(bin == lbin) & active;
        int base = 0;
        if (lane == leader)
            base = atomicAdd(&nd.bin_count[lbin], __popcll(same));
        base = __shfl(base, leader);
        if (bin == lbin)
            slot = base + __popcll(same & ((1ull << lane) - 1ull));
        todo &= ~same;
    }
    nd.rank[j] = slot;
}

// One workgroup of 1024 threads: exclusive scans of the bin counts (-> bin_start) and of
// the work items per bin, ceil(count / cap) (-> bin_chunk); counters[0] = total items.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void k_node_scan(Nodes nd, int nbins)
{
    __shared__ int64_t s_a[kScanThreads];
    __shared__ int64_t s_b[kScanThreads];
    const int tid = threadIdx.x;
    const int per = (nbins + kScanThreads - 1) / kScanThreads;
    const int lo = tid * per;
    const int hi = min(nbins, lo + per);
    int64_t sa = 0, sb = 0;
    for (int i = lo; i < hi; ++i) {
        int c = nd.bin_count[i];
        sa += c;
        sb += (c + nd.chunk_cap - 1) / nd.chunk_cap;
    }
    s_a[tid] = sa;
    s_b[tid] = sb;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 1024 partial sums
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int64_t va = tid >= off ? s_a[tid - off] : 0;
        int64_t vb = tid >= off ? s_b[tid - off] : 0;
        __syncthreads();
        s_a[tid] += va;
        s_b[tid] += vb;
        __syncthreads();
    }
    int64_t ra = s_a[tid] - sa;  // exclusive prefix of this segment
    int64_t rb = s_b[tid] - sb;
    for (int i = lo; i < hi; ++i) {
        int c = nd.bin_count[i];
        nd.bin_start[i] = (int32_t)ra;
        nd.bin_chunk[i] = (int32_t)rb;
        ra += c;
        rb += (c + nd.chunk_cap - 1) / nd.chunk_cap;
    }
    if (tid == kScanThreads - 1) {
        nd.bin_start[nbins] = (int32_t)s_a[tid];
        nd.bin_chunk[nbins] = (int32_t)s_b[tid];
        nd.counters[0] = (int32_t)s_b[tid];
    }
}

// Caller index of every node at a position of its bin's range (the order inside a bin is
// arbitrary here and fixed by the sort below).
__global__ __launch_bounds__(kBlock) void k_node_place(Nodes nd, int32_t *dst)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nd.M)
        return;
    dst[nd.bin_start[nd.key[j]] + nd.rank[j]] = (int32_t)j;
}

// Sorting every bin's range by caller index, so that the sorted order -- and with it the
// work items, the order of every floating-point sum over a work item's nodes and the
// fold -- is the same on every run.  Caller indices are unique, so the sorted order is
// unique.  First each tile of kSortTile positions is sorted by (bin, caller index) in LDS;
// positions are already grouped by bin, so every node stays inside its bin's range and
// the part of a bin inside a tile becomes sorted.  Then runs are merged pairwise: with
// runs [r L, (r+1) L) clipped to the bin's range, a node's position in the merged pair
// is its offset in its own run plus the number of smaller caller indices in the partner
// run (binary search), for L = kSortTile, 2 kSortTile, ... until L reaches M.
constexpr int kSortTile = 1024;
__device__ __forceinline__ void bitonic(unsigned long long *keys, int n);

__global__ __launch_bounds__(kBlock) void k_bin_tile_sort(Nodes nd, int32_t *buf)
{
    __shared__ unsigned long long keys[kSortTile];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int len = (int)min<int64_t>(kSortTile, nd.M - base);
    for (int i = threadIdx.x; i < kSortTile; i += kBlock) {
        unsigned long long k = ~0ull;
        if (i < len) {
            const int32_t v = buf[base + i];
            k = ((unsigned long long)(uint32_t)nd.key[v] << 32) | (uint32_t)v;
        }
        keys[i] = k;
    }
    __syncthreads();
    bitonic(keys, kSortTile);
    for (int i = threadIdx.x; i < len; i += kBlock)
        buf[base + i] = (int32_t)(keys[i] & 0xffffffffull);
}

__global__ __launch_bounds__(kBlock) void k_bin_merge(Nodes nd, const int32_t *__restrict__ src,
                                                       int32_t *__restrict__ dst, int64_t L)
{
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= nd.M)
        return;
    const int32_t v = src[pos];
    const int b = nd.key[v];
    const int64_t first = nd.bin_start[b], end = nd.bin_start[b + 1];
    const int64_t r = pos / L;
    const int64_t own_lo = max(first, r * L);
    const int64_t pr = r ^ 1;
    const int64_t p_lo = max(first, pr * L), p_hi = min(end, (pr + 1) * L);
    if (p_lo >= p_hi) {
        dst[pos] = v;
        return;
    }
    int64_t lo = p_lo, hi = p_hi;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (src[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    const int64_t merged_lo = max(first, (r & ~(int64_t)1) * L);
    dst[merged_lo + (pos - own_lo) + (lo - p_lo)] = v;
}

// Cell index and offset of every sorted node, from its caller index.
template <int D, typename T> __global__ __launch_bounds__(kBlock) void k_node_scatter(Geom g, Nodes nd)
{
    int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= nd.M)
        return;
    const int64_t j = nd.perm[pos];
#pragma unroll
    for (int t = 0; t < D; ++t) {
        int u;
        double delta;
        node_index(nd.x[j * D + t], g.n[t], u, delta);
        nd.u[t][pos] = u;
        static_cast<T *>(nd.delta[t])[pos] = (T)delta;
    }
}

// Window factors of every sorted node (the tensor-product precomputation of Table 3.2,
// PRE_PSI): psi[node][t][s] = normalised window phi_t(delta_t - (s - m)), s < 2m+2.  One
// thread per factor, so the writes are coalesced.
template <typename T, bool AllW> __global__ __launch_bounds__(kBlock) void k_node_psi(Geom g, Nodes nd)
{
    const int W = g.W;
    const int dW = g.d * W;
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nd.M * dW)
        return;
    int64_t node = q / dW;
    int r = (int)(q - node * dW);
    int t = r / W;
    int s = r - t * W;
    T delta = static_cast<const T *>(nd.delta[t])[node];
    // a non-finite node (offset NaN) gets NaN factors, so that its results are NaN too
    static_cast<T *>(nd.psi)[q] = isnan(delta) ? delta : win_value<T, AllW>(g, nd, t, delta, s);
}

// The lookup tables of dimension t (plans with NFFT_PRE_LIN_PSI): entry s (kLinK + 1) + i holds
// the factor and its derivative at stencil point s for delta = i / kLinK, evaluated in FP64
// and rounded once.
template <typename T> __global__ __launch_bounds__(kBlock) void k_fill_lin(Geom g, int t, T *tab, T *dtab)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)g.W * (kLinK + 1))
        return;
    const int s = (int)(e / (kLinK + 1));
    const int i = (int)(e - (int64_t)s * (kLinK + 1));
    const double delta = (double)i / kLinK;
    tab[e] = (T)win_point<double, true>(g, t, delta, s);
    dtab[e] = (T)win_point_d<double, true>(g, t, delta, s);
}

// One thread per bin writes the bin's work items.
__global__ __launch_bounds__(kBlock) void k_node_chunks(Nodes nd, int nbins)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins)
        return;
    int count = nd.bin_count[b];
    int first = nd.bin_start[b];
    int c0 = nd.bin_chunk[b];
    for (int i = 0; i * nd.chunk_cap < count; ++i) {
        nd.chunk_bin[c0 + i] = b;
        nd.chunk_first[c0 + i] = first + i * nd.chunk_cap;
        nd.chunk_len[c0 + i] = min(nd.chunk_cap, count - i * nd.chunk_cap);
    }
}

// Order the nodes of every work item for the window kernels.  With r the residue mod 32
// of a node's cell position in the padded tile (its LDS bank pair), the nodes are first
// sorted by (r, cell, caller index) -- unique, so the order is deterministic -- and then
// dealt round-robin over the residue classes: the first node of every class, then the
// second, and so on.  Consecutive nodes therefore have different residues, and the
// interpolation kernels, which give consecutive nodes to consecutive lanes, read 32
// different bank pairs per half-wave.
constexpr int kSortMax = 1024;  // chunk_cap is at most this
// Bitonic sort of n (a power of two, <= kSortMax) keys in LDS by the workgroup.
__device__ __forceinline__ void bitonic(unsigned long long *keys, int n)
{
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < n; i += kBlock) {
                const int ij = i ^ j;
                if (ij > i) {
                    const unsigned long long a = keys[i], b = keys[ij];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        keys[i] = b;
                        keys[ij] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

template <int D, typename T> __global__ __launch_bounds__(kBlock) void k_chunk_sort(Geom g, Nodes nd)
{
    __shared__ unsigned long long keys[kSortMax];
    __shared__ int cls_start[32];
    const int nchunks = nd.counters[0];
    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int first = nd.chunk_first[c];
        const int len = nd.chunk_len[c];
        int npow = 1;
        while (npow < len)
            npow <<= 1;
        for (int i = threadIdx.x; i < npow; i += kBlock) {
            unsigned long long key = ~0ull;
            if (i < len) {
                const int node = first + i;
                int pos = 0, cell = 0;
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    const int ul = nd.u[t][node] & ((1 << g.lgB[t]) - 1);
                    pos = pos * g.P[t] + ul;
                    cell = (cell << g.lgB[t]) | ul;
                }
                const unsigned long long r = (unsigned)pos & 31u;
                key = (r << 58) | ((unsigned long long)cell << 41) | ((unsigned long long)nd.perm[node] << 10) |
                      (unsigned long long)i;
            }
            keys[i] = key;
        }
        __syncthreads();
        // bitonic sort of npow keys by (bank residue, cell, caller index)
        bitonic(keys, npow);
        // Deal the nodes round-robin over the residue classes: key (rank in class,
        // residue), so that consecutive nodes -- taken by consecutive lanes of the
        // interpolation kernels -- start on different LDS banks.
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const int r = (int)(keys[i] >> 58);
            if (i == 0 || (int)(keys[i - 1] >> 58) != r)
                cls_start[r] = i;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const unsigned long long r = keys[i] >> 58;
            const unsigned long long rank = (unsigned long long)(i - cls_start[r]);
            keys[i] = (rank << 20) | (r << 15) | (keys[i] & 1023ull);
        }
        __syncthreads();
        bitonic(keys, npow);
        // gather the node data in the new order (read all, then write)
        int u_new[kSortMax / kBlock][D];
        T d_new[kSortMax / kBlock][D];
        int p_new[kSortMax / kBlock];
#pragma unroll
        for (int q = 0; q < kSortMax / kBlock; ++q) {
            const int i = threadIdx.x + q * kBlock;
            if (i < len) {
                const int src = first + (int)(keys[i] & 1023ull);
                p_new[q] = nd.perm[src];
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    u_new[q][t] = nd.u[t][src];
                    d_new[q][t] = static_cast<const T *>(nd.delta[t])[src];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kSortMax / kBlock; ++q) {
            const int i = threadIdx.x + q * kBlock;
            if (i < len) {
                nd.perm[first + i] = p_new[q];
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    nd.u[t][first + i] = u_new[q][t];
                    static_cast<T *>(nd.delta[t])[first + i] = d_new[q][t];
                }
            }
        }
        __syncthreads();
        if constexpr (D == 2) {
            if (nd.spos) {
                // order for the 2-D spreading kernel that keeps tile columns in registers:
                // by tile row, ties by position in the work item
                const int rmask = (1 << g.lgB[0]) - 1;
                for (int i = threadIdx.x; i < npow; i += kBlock)
                    keys[i] = i < len ? ((unsigned long long)(nd.u[0][first + i] & rmask) << 10) | (unsigned)i : ~0ull;
                __syncthreads();
                bitonic(keys, npow);
                for (int i = threadIdx.x; i < len; i += kBlock) {
                    const int k = (int)(keys[i] & 1023ull);
                    const int r0 = (int)(keys[i] >> 10);
                    const int c0 = nd.u[1][first + k] & 31;
                    nd.spos[2 * (first + i)] = (k << 10) | (r0 << 5) | c0;
                    nd.spos[2 * (first + i) + 1] = nd.perm[first + k];
                }
                __syncthreads();
            }
        }
    }
}

__global__ void k_fill_zero(uint32_t *p, int64_t words)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride)
        p[i] = 0u;
}

inline int blocks_for(int64_t n, int per = kBlock) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_node_reset(const Geom &g, const Nodes &nd, hipStream_t s)
{
    int n = g.nbins > 2 ? g.nbins : 2;
    hipLaunchKernelGGL(k_node_reset, dim3(blocks_for(n)), dim3(kBlock), 0, s, nd.bin_count, g.nbins,
                       nd.counters);
    return hipGetLastError();
}

hipError_t launch_node_key(const Geom &g, const Nodes &nd, double *xcopy, hipStream_t s)
{
    dim3 grid(blocks_for(nd.M)), block(kBlock);
    switch (g.d) {
    case 1: hipLaunchKernelGGL(k_node_key<1>, grid, block, 0, s, g, nd, xcopy); break;
    case 2: hipLaunchKernelGGL(k_node_key<2>, grid, block, 0, s, g, nd, xcopy); break;
    case 3: hipLaunchKernelGGL(k_node_key<3>, grid, block, 0, s, g, nd, xcopy); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_node_scan(const Geom &g, const Nodes &nd, hipStream_t s)
{
    hipLaunchKernelGGL(k_node_scan, dim3(1), dim3(kScanThreads), 0, s, nd, g.nbins);
    return hipGetLastError();
}

hipError_t launch_node_scatter(const Geom &g, const Nodes &nd, bool dbl, hipStream_t s)
{
    dim3 grid(blocks_for(nd.M)), block(kBlock);
    {
        // merge passes: L = kSortTile, 2 kSortTile, ... while L < M; the tile sort and the
        // passes ping-pong between perm and u[0] (free until the cell indices are written),
        // starting in the buffer that makes the last pass end in perm
        int passes = 0;
        for (int64_t L = kSortTile; L < nd.M; L *= 2)
            ++passes;
        int32_t *a = (passes & 1) ? nd.u[0] : nd.perm;
        int32_t *b = (passes & 1) ? nd.perm : nd.u[0];
        hipLaunchKernelGGL(k_node_place, grid, block, 0, s, nd, a);
        hipLaunchKernelGGL(k_bin_tile_sort, dim3(blocks_for(nd.M, kSortTile)), block, 0, s, nd, a);
        for (int64_t L = kSortTile; L < nd.M; L *= 2) {
            hipLaunchKernelGGL(k_bin_merge, grid, block, 0, s, nd, (const int32_t *)a, b, L);
            int32_t *t = a;
            a = b;
            b = t;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    switch (g.d * 2 + (dbl ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((k_node_scatter<1, float>), grid, block, 0, s, g, nd); break;
    case 3: hipLaunchKernelGGL((k_node_scatter<1, double>), grid, block, 0, s, g, nd); break;
    case 4: hipLaunchKernelGGL((k_node_scatter<2, float>), grid, block, 0, s, g, nd); break;
    case 5: hipLaunchKernelGGL((k_node_scatter<2, double>), grid, block, 0, s, g, nd); break;
    case 6: hipLaunchKernelGGL((k_node_scatter<3, float>), grid, block, 0, s, g, nd); break;
    case 7: hipLaunchKernelGGL((k_node_scatter<3, double>), grid, block, 0, s, g, nd); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_node_chunks, dim3(blocks_for(g.nbins)), block, 0, s, nd, g.nbins);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    {
        const int sort_blocks = nd.max_chunks < 4096 ? nd.max_chunks : 4096;
        switch (g.d * 2 + (dbl ? 1 : 0)) {
        case 2: hipLaunchKernelGGL((k_chunk_sort<1, float>), dim3(sort_blocks), block, 0, s, g, nd); break;
        case 3: hipLaunchKernelGGL((k_chunk_sort<1, double>), dim3(sort_blocks), block, 0, s, g, nd); break;
        case 4: hipLaunchKernelGGL((k_chunk_sort<2, float>), dim3(sort_blocks), block, 0, s, g, nd); break;
        case 5: hipLaunchKernelGGL((k_chunk_sort<2, double>), dim3(sort_blocks), block, 0, s, g, nd); break;
        case 6: hipLaunchKernelGGL((k_chunk_sort<3, float>), dim3(sort_blocks), block, 0, s, g, nd); break;
        case 7: hipLaunchKernelGGL((k_chunk_sort<3, double>), dim3(sort_blocks), block, 0, s, g, nd); break;
        default: return hipErrorInvalidValue;
        }
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    const int64_t nf = nd.M * g.d * g.W;
    if (dbl) {
        auto kf = window_needs_all(g) ? k_node_psi<double, true> : k_node_psi<double, false>;
        hipLaunchKernelGGL(kf, dim3(blocks_for(nf)), block, 0, s, g, nd);
    } else {
        auto kf = window_needs_all(g) ? k_node_psi<float, true> : k_node_psi<float, false>;
        hipLaunchKernelGGL(kf, dim3(blocks_for(nf)), block, 0, s, g, nd);
    }
    return hipGetLastError();
}

hipError_t launch_fill_lin(const Geom &g, int t, bool dbl, void *tab, void *dtab, hipStream_t s)
{
    const int64_t n = (int64_t)g.W * (kLinK + 1);
    if (dbl)
        hipLaunchKernelGGL(k_fill_lin<double>, dim3(blocks_for(n)), dim3(kBlock), 0, s, g, t,
                           static_cast<double *>(tab), static_cast<double *>(dtab));
    else
        hipLaunchKernelGGL(k_fill_lin<float>, dim3(blocks_for(n)), dim3(kBlock), 0, s, g, t,
                           static_cast<float *>(tab), static_cast<float *>(dtab));
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s)
{
    int64_t words = (int64_t)(bytes / 4);
    if (words == 0)
        return hipSuccess;
    int blocks = blocks_for(words);
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(kBlock), 0, s, static_cast<uint32_t *>(p), words);
    return hipGetLastError();
}

}  // namespace nfft
