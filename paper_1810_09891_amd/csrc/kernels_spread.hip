// Spreading (Algorithm 2.2 step 1): LDS tile accumulation per work item and the
// deterministic fold of the tiles into the grid.  Geometry as in window_common.hpp.
#include "window_common.hpp"

namespace nfft {

namespace {

using namespace window;

// ------------------------------------------------------------------ spreading
//
// A wave takes one node at a time and its lanes cover the node's stencil, so within a
// wave no two lanes touch the same cell and the accumulation is a plain read-add-write
// in LDS (no LDS atomics, which are slow for FP32 on this hardware, and a fixed order of
// additions).  The window factors come from the node precomputation (psi).
//  * 1-D / 2-D: lane (r, s1) with s1 = lane mod W, r = lane / W covers stencil row
//    s0 = r, r + R, r + 2R, ... (R = 64 / W rows per pass) and column s1.  Each of the
//    four waves of a workgroup accumulates its share of the work item's nodes into its
//    own padded tile; the four tiles are summed in wave order when the item is done.
//  * 3-D: the four waves share one padded tile and split each node's planes s0 (wave w
//    takes s0 = w, w+4, ...); lanes cover (s1, s2) like the rows and columns above; a
//    barrier separates consecutive nodes.

constexpr int kWaves = kBlock / 64;

template <typename T> __device__ __forceinline__ T lane_shfl(T v, int src) { return __shfl(v, src, 64); }

template <typename T, int D, int WM>
__global__ __launch_bounds__(kBlock) void k_spread_tiles(Geom g, Nodes nd, const Cplx<T> *__restrict__ f,
                                                         Cplx<T> *__restrict__ scratch)
{
    using C = Cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tiles = reinterpret_cast<C *>(smem_raw);
    const T *psi = static_cast<const T *>(nd.psi);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int W = g.W;
    const int dW = D * W;
    const int R = 64 / W;  // stencil rows per pass
    const int r = lane / W;
    const int sc = lane - r * W;  // stencil column of this lane
    const bool lane_ok = r < R;
    const int nchunks = nd.counters[0];
    for (int c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int first = nd.chunk_first[c];
        const int len = nd.chunk_len[c];
        if constexpr (D < 3) {
            C *sub = tiles + wave * g.Ptot;
            for (int i = lane; i < g.Ptot; i += 64)
                sub[i] = C{T(0), T(0)};
            for (int i = wave; i < len; i += kWaves) {
                const int node = first + i;
                const C fv = f[nd.perm[node]];
                const T wv = lane < dW ? psi[(int64_t)node * dW + lane] : T(0);
                if constexpr (D == 1) {
                    const int ul0 = nd.u[0][node] & ((1 << g.lgB[0]) - 1);
                    if (lane < W) {
                        C v = sub[ul0 + lane];
                        v.x += fv.x * wv;
                        v.y += fv.y * wv;
                        sub[ul0 + lane] = v;
                    }
                } else {
                    const int ul0 = nd.u[0][node] & ((1 << g.lgB[0]) - 1);
                    const int ul1 = nd.u[1][node] & ((1 << g.lgB[1]) - 1);
                    const T w1 = lane_shfl(wv, W + sc);
                    const T ax = fv.x * w1, ay = fv.y * w1;
                    const int base = ul0 * g.P[1] + ul1 + sc;
                    for (int s0b = 0; s0b < W; s0b += R) {
                        const int s0 = s0b + r;
                        const T w0 = lane_shfl(wv, s0 < W ? s0 : W - 1);
                        if (lane_ok && s0 < W) {
                            const int idx = base + s0 * g.P[1];
                            C v = sub[idx];
                            v.x += ax * w0;
                            v.y += ay * w0;
                            sub[idx] = v;
                        }
                    }
                }
            }
            __syncthreads();
            C *slot = scratch + (int64_t)c * g.Ptot;
            for (int i = threadIdx.x; i < g.Ptot; i += kBlock) {
                C a = tiles[i];
#pragma unroll
                for (int w = 1; w < kWaves; ++w) {
                    C b = tiles[w * g.Ptot + i];
                    a.x += b.x;
                    a.y += b.y;
                }
                slot[i] = a;
            }
            __syncthreads();
        } else {
            for (int i = threadIdx.x; i < g.Ptot; i += kBlock)
                tiles[i] = C{T(0), T(0)};
            __syncthreads();
            const int P1 = g.P[1], P2 = g.P[2];
            for (int i = 0; i < len; ++i) {
                const int node = first + i;
                const C fv = f[nd.perm[node]];
                const int64_t prow = (int64_t)node * dW;
                const T wv0 = lane < dW ? psi[prow + lane] : T(0);
                const T wv1 = lane + 64 < dW ? psi[prow + 64 + lane] : T(0);
                const int ul0 = nd.u[0][node] & ((1 << g.lgB[0]) - 1);
                const int ul1 = nd.u[1][node] & ((1 << g.lgB[1]) - 1);
                const int ul2 = nd.u[2][node] & ((1 << g.lgB[2]) - 1);
                const int slot2 = 2 * W + sc;  // factor of dimension 2 at this lane's column
                const T w2a = lane_shfl(wv0, slot2 < 64 ? slot2 : 0);
                const T w2b = lane_shfl(wv1, slot2 >= 64 ? slot2 - 64 : 0);
                const T w2 = slot2 < 64 ? w2a : w2b;
                const T ax = fv.x * w2, ay = fv.y * w2;
                for (int s0 = wave; s0 < W; s0 += kWaves) {
                    const T w0 = lane_shfl(wv0, s0);
                    const T bx = ax * w0, by = ay * w0;
                    const int pbase = (ul0 + s0) * P1 + ul1;
                    for (int s1b = 0; s1b < W; s1b += R) {
                        const int s1 = s1b + r;
                        const T w1 = lane_shfl(wv0, W + (s1 < W ? s1 : W - 1));
                        if (lane_ok && s1 < W) {
                            const int idx = (pbase + s1) * P2 + ul2 + sc;
                            C v = tiles[idx];
                            v.x += bx * w1;
                            v.y += by * w1;
                            tiles[idx] = v;
                        }
                    }
                }
                __syncthreads();
            }
            C *slot = scratch + (int64_t)c * g.Ptot;
            for (int i = threadIdx.x; i < g.Ptot; i += kBlock)
                slot[i] = tiles[i];
            __syncthreads();
        }
    }
}

// (bin, offset) pairs of one dimension covering grid index l: bin b covers the unwrapped
// indices b*B - m .. b*B - m + P - 1; l is covered through l + k*n for k = -1, 0, 1.
__device__ __forceinline__ int cover_pairs(int l, int n, int B, int lgB, int nb, int m, int P, int *bins,
                                           int *offs)
{
    int cnt = 0;
    for (int k = -1; k <= 1; ++k) {
        int lu = l + k * n + m;  // unwrapped index relative to origin shift
        // need 0 <= lu - b*B < P  ->  (lu - P + 1)/B <= b <= lu/B
        int hi = lu >= 0 ? (lu >> lgB) : -1;
        int lo_num = lu - P + 1;
        int lo = lo_num <= 0 ? 0 : ((lo_num + B - 1) >> lgB);
        if (hi > nb - 1)
            hi = nb - 1;
        for (int b = lo; b <= hi && cnt < kFoldMaxPairs; ++b) {
            bins[cnt] = b;
            offs[cnt] = lu - b * B;
            ++cnt;
        }
    }
    return cnt;
}

template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_fold(Geom g, Nodes nd, const Cplx<T> *__restrict__ scratch,
                                                 Cplx<T> *__restrict__ grid)
{
    using C = Cplx<T>;
    int64_t total = 1;
#pragma unroll
    for (int t = 0; t < D; ++t)
        total *= g.n[t];
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total)
        return;
    int l[kMaxDim];
    {
        int64_t r = q;
#pragma unroll
        for (int t = D - 1; t >= 0; --t) {
            l[t] = (int)(r & (g.n[t] - 1));
            r >>= (31 - __clz(g.n[t]));
        }
    }
    int bins[kMaxDim][kFoldMaxPairs], offs[kMaxDim][kFoldMaxPairs], cnt[kMaxDim];
#pragma unroll
    for (int t = 0; t < D; ++t)
        cnt[t] = cover_pairs(l[t], g.n[t], 1 << g.lgB[t], g.lgB[t], g.nb[t], g.m, g.P[t], bins[t], offs[t]);
    T ax = 0, ay = 0;
    if constexpr (D == 1) {
        for (int a = 0; a < cnt[0]; ++a) {
            int bin = bins[0][a];
            for (int c = nd.bin_chunk[bin]; c < nd.bin_chunk[bin + 1]; ++c) {
                C v = scratch[(int64_t)c * g.Ptot + offs[0][a]];
                ax += v.x;
                ay += v.y;
            }
        }
    } else if constexpr (D == 2) {
        for (int a = 0; a < cnt[0]; ++a)
            for (int e = 0; e < cnt[1]; ++e) {
                int bin = bins[0][a] * g.nb[1] + bins[1][e];
                int off = offs[0][a] * g.P[1] + offs[1][e];
                for (int c = nd.bin_chunk[bin]; c < nd.bin_chunk[bin + 1]; ++c) {
                    C v = scratch[(int64_t)c * g.Ptot + off];
                    ax += v.x;
                    ay += v.y;
                }
            }
    } else {
        for (int a = 0; a < cnt[0]; ++a)
            for (int e = 0; e < cnt[1]; ++e)
                for (int h = 0; h < cnt[2]; ++h) {
                    int bin = (bins[0][a] * g.nb[1] + bins[1][e]) * g.nb[2] + bins[2][h];
                    int off = (offs[0][a] * g.P[1] + offs[1][e]) * g.P[2] + offs[2][h];
                    for (int c = nd.bin_chunk[bin]; c < nd.bin_chunk[bin + 1]; ++c) {
                        C v = scratch[(int64_t)c * g.Ptot + off];
                        ax += v.x;
                        ay += v.y;
                    }
                }
    }
    grid[q] = C{ax, ay};
}

#define NFFT_WM_SWITCH(WMV, CALL)                                                                       \
    switch (WMV) {                                                                                     \
    case 6: CALL(6); break;                                                                            \
    case 10: CALL(10); break;                                                                          \
    case 14: CALL(14); break;                                                                          \
    case 18: CALL(18); break;                                                                          \
    case 22: CALL(22); break;                                                                          \
    case 26: CALL(26); break;                                                                          \
    default: return hipErrorInvalidValue;                                                              \
    }

#define NFFT_DT_SWITCH(FN, ...)                                                                        \
    switch (g.d * 2 + (dbl ? 1 : 0)) {                                                                 \
    case 2: return FN<float, 1>(__VA_ARGS__);                                                          \
    case 3: return FN<double, 1>(__VA_ARGS__);                                                         \
    case 4: return FN<float, 2>(__VA_ARGS__);                                                          \
    case 5: return FN<double, 2>(__VA_ARGS__);                                                         \
    case 6: return FN<float, 3>(__VA_ARGS__);                                                          \
    case 7: return FN<double, 3>(__VA_ARGS__);                                                         \
    default: return hipErrorInvalidValue;                                                              \
    }

template <typename T, int D>
hipError_t spread_typed(const Geom &g, const Nodes &nd, const void *f, void *scratch, int blocks, size_t lds,
                        hipStream_t s)
{
    using C = Cplx<T>;
#define CALL(W_)                                                                                       \
    {                                                                                                  \
        auto kf = k_spread_tiles<T, D, W_>;                                                            \
        (void)hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        hipLaunchKernelGGL(kf, dim3(blocks), dim3(kBlock), lds, s, g, nd, static_cast<const C *>(f),    \
                           static_cast<C *>(scratch));                                                 \
    }
    NFFT_WM_SWITCH(g.WM, CALL)
#undef CALL
    return hipGetLastError();
}
template <typename T, int D>
hipError_t fold_typed(const Geom &g, const Nodes &nd, const void *scratch, void *grid, hipStream_t s)
{
    using C = Cplx<T>;
    int64_t total = 1;
    for (int t = 0; t < D; ++t)
        total *= g.n[t];
    int blocks = (int)((total + kBlock - 1) / kBlock);
    hipLaunchKernelGGL((k_fold<T, D>), dim3(blocks), dim3(kBlock), 0, s, g, nd,
                       static_cast<const C *>(scratch), static_cast<C *>(grid));
    return hipGetLastError();
}
}  // namespace

hipError_t launch_spread_tiles(const Geom &g, const Nodes &nd, bool dbl, const void *f, void *scratch,
                               int blocks, size_t lds, hipStream_t s)
{
    NFFT_DT_SWITCH(spread_typed, g, nd, f, scratch, blocks, lds, s)
}
hipError_t launch_fold(const Geom &g, const Nodes &nd, bool dbl, const void *scratch, void *grid, hipStream_t s)
{
    NFFT_DT_SWITCH(fold_typed, g, nd, scratch, grid, s)
}

}  // namespace nfft
