// Interpolation (Algorithm 2.1 step 3) and the LDS sizes of the window kernels.
//
// Nodes are sorted into bins of B_0 x ... x B_{d-1} grid cells and cut into work items of
// at most chunk_cap nodes of one bin.  The stencil of a node with u = floor(n x) covers
// the 2m+2 grid indices u-m .. u+m+1 per dimension (eq. (2.13), read with 2m+2 points), so
// every stencil of a bin lies in its padded tile: origin b*B - m, edge P = B + WM - 1
// (WM >= 2m+2 is the compiled stencil width, extra points carry weight zero).
//
// A workgroup stages the padded tile of its bin from the grid into LDS with coalesced row
// reads (indices taken mod n, Sec. 2 eq. (2.5)), then each thread takes one node and sums
// its (2m+2)^d stencil from LDS as nested tensor-product sums of the precomputed window
// factors (the structure the PRE_PSI flag of Table 3.2 exploits).  Spreading, the other
// window kernel, is in kernels_spread.hip.
#include "batch_desc.hpp"
#include "window_common.hpp"

namespace nfft {

namespace {

using namespace window;

// ------------------------------------------------------------------ interpolation

// One work item c of a plan: stage the bin's padded tile, then interpolate its nodes.
template <typename T, int D, int WM>
__device__ __forceinline__ void interp_item(const Geom &g, const Nodes &nd, const Cplx<T> *__restrict__ grid,
                                            Cplx<T> *__restrict__ f, int c, Cplx<T> *tile)
{
    using C = Cplx<T>;
    const T *psi = static_cast<const T *>(nd.psi);
    const int W = g.W;
    const int dW = D * W;
    const int bin = nd.chunk_bin[c];
    const int first = nd.chunk_first[c];
    const int len = nd.chunk_len[c];
    int bc[kMaxDim];
    bin_coords<T, D>(g, bin, bc);
    // Factors of the dimensions whose factors are held in registers: all of them, except
    // dimension 0 of the 3-D complex128 kernels with more than 14 points, which read theirs
    // plane by plane.
    constexpr int T0 = (D == 3 && !(sizeof(T) == 4 || WM <= 14)) ? 1 : 0;
    // Cell indices and window factors (aligned pairs; W and WM are even and the factor
    // table is padded past its end) of the thread's next node.  The first node's are
    // loaded before the tile is staged, so that both loads are in flight together.
    int ul[kMaxDim];
    Pair<T> raw[D][WM / 2];
    auto load_node = [&](int node) {
#pragma unroll
        for (int t = 0; t < D; ++t)
            ul[t] = nd.u[t][node] & ((1 << g.lgB[t]) - 1);
        const Pair<T> *p2 = reinterpret_cast<const Pair<T> *>(psi + (int64_t)node * dW);
#pragma unroll
        for (int t = T0; t < D; ++t)
#pragma unroll
            for (int s = 0; s < WM / 2; ++s)
                raw[t][s] = p2[t * (W / 2) + s];
    };
    // window factors of dimension t at the WM compiled points (zero beyond W)
    auto factors = [&](int t, T *w) {
#pragma unroll
        for (int s = 0; s < WM / 2; ++s) {
            const Pair<T> v = raw[t][s];
            w[2 * s] = 2 * s < W ? v.x : T(0);
            w[2 * s + 1] = 2 * s + 1 < W ? v.y : T(0);
        }
    };
    if ((int)threadIdx.x < len)
        load_node(first + threadIdx.x);
    stage_tile<T, D>(g, bc, grid, tile);
    __syncthreads();
    // 2-D items with more nodes than threads: the first 256 nodes one per thread, the rest
    // (below) shared by all four waves, so the item does not take two rounds of whole nodes
    const int lmain = (D == 2 && len > kBlock) ? kBlock : len;
    // Thread t takes nodes t, t + 256, ...: the nodes are dealt round-robin over the bank
    // residues of their tile positions, so consecutive lanes start on different LDS banks.
    for (int i = threadIdx.x; i < lmain; i += kBlock) {
        const int node = first + i;
        const T *pw = psi + (int64_t)node * dW;  // window factors [d][W] of this node
        if (i != (int)threadIdx.x)
            load_node(node);
        T wl[WM];  // innermost dimension
        factors(D - 1, wl);
        T ax = 0, ay = 0;
        // Rows of the stencil (WM points along the innermost dimension) are read from LDS one
        // row ahead of their use, so a row's reads are in flight while the previous row is
        // summed.  Rows past 2m+1 lie inside the padded tile and carry weight zero.
        // (complex128 rows of 18 or more points keep one buffer: two would halve occupancy)
        constexpr bool kAhead = sizeof(T) == 4 ? WM <= 22 : WM <= 10;
        C buf[2][WM];
        auto load_row = [&](const C *row, C *dst) {
#pragma unroll
            for (int s = 0; s < WM; ++s)
                dst[s] = lds_entry<T>(row + s);
        };
        // without the look-ahead buffer a row is summed straight from LDS
        auto sum_lds = [&](const C *row, T &rx, T &ry) {
            rx = 0;
            ry = 0;
#pragma unroll
            for (int s = 0; s < WM; ++s) {
                const C v = lds_entry<T>(row + s);
                rx += wl[s] * v.x;
                ry += wl[s] * v.y;
            }
        };
        auto sum_row = [&](const C *v, T &rx, T &ry) {
            rx = 0;
            ry = 0;
#pragma unroll
            for (int s = 0; s < WM; ++s) {
                rx += wl[s] * v[s].x;
                ry += wl[s] * v[s].y;
            }
        };
        if constexpr (D == 1) {
            sum_lds(tile + ul[0], ax, ay);
        } else if constexpr (D == 2) {
            T w0r[WM];
            factors(0, w0r);
            const int P1 = g.P[1];
            const C *base = tile + ul[0] * P1 + ul[1];
            if (kAhead)
                load_row(base, buf[0]);
#pragma unroll
            for (int s0 = 0; s0 < WM; ++s0) {
                T rx, ry;
                if constexpr (kAhead) {
                    if (s0 + 1 < WM)
                        load_row(base + (s0 + 1) * P1, buf[(s0 + 1) & 1]);
                    sum_row(buf[s0 & 1], rx, ry);
                } else {
                    sum_lds(base + s0 * P1, rx, ry);
                }
                ax += w0r[s0] * rx;
                ay += w0r[s0] * ry;
            }
        } else {
            T wmid[WM];
            factors(1, wmid);
            const int P1 = g.P[1], P2 = g.P[2];
            if constexpr (sizeof(T) == 4 || WM <= 14) {
                // planes unrolled, their factors loaded once
                T w0r[WM];
                factors(0, w0r);
#pragma unroll
                for (int s0 = 0; s0 < WM; ++s0) {
                    if (s0 < W) {  // uniform
                        const T w0 = w0r[s0];
                        const C *plane = tile + ((ul[0] + s0) * P1 + ul[1]) * P2 + ul[2];
                        if (kAhead)
                            load_row(plane, buf[0]);
                        T px = 0, py = 0;
#pragma unroll
                        for (int s1 = 0; s1 < WM; ++s1) {
                            T rx, ry;
                            if constexpr (kAhead) {
                                if (s1 + 1 < WM)
                                    load_row(plane + (s1 + 1) * P2, buf[(s1 + 1) & 1]);
                                sum_row(buf[s1 & 1], rx, ry);
                            } else {
                                sum_lds(plane + s1 * P2, rx, ry);
                            }
                            px += wmid[s1] * rx;
                            py += wmid[s1] * ry;
                        }
                        ax += w0 * px;
                        ay += w0 * py;
                    }
                }
            } else {
                for (int s0 = 0; s0 < W; ++s0) {
                    const T w0 = pw[s0];
                    const C *plane = tile + ((ul[0] + s0) * P1 + ul[1]) * P2 + ul[2];
                    if (kAhead)
                        load_row(plane, buf[0]);
                    T px = 0, py = 0;
#pragma unroll
                    for (int s1 = 0; s1 < WM; ++s1) {
                        T rx, ry;
                        if constexpr (kAhead) {
                            if (s1 + 1 < WM)
                                load_row(plane + (s1 + 1) * P2, buf[(s1 + 1) & 1]);
                            sum_row(buf[s1 & 1], rx, ry);
                        } else {
                            sum_lds(plane + s1 * P2, rx, ry);
                        }
                        px += wmid[s1] * rx;
                        py += wmid[s1] * ry;
                    }
                    ax += w0 * px;
                    ay += w0 * py;
                }
            }
        }
        f[nd.perm[node]] = C{ax, ay};
    }
    if constexpr (D == 2) {
        // Nodes past the first 256, 64 at a time: lane l takes node e0 + l and wave w sums
        // stencil rows [w W / 4, (w + 1) W / 4) of it (a range uniform over the wave); the
        // four partial sums meet in LDS after the tile and are added in wave order.
        if (len > kBlock) {
            C *part = tile + g.Ptot;
            const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
            const int lane = threadIdx.x & 63;
            const int lo = (wv * W) >> 2, hi = ((wv + 1) * W) >> 2;
            const int P1 = g.P[1];
            for (int e0 = kBlock; e0 < len; e0 += 64) {
                const int i = e0 + lane;
                T ax = 0, ay = 0;
                if (i < len) {
                    load_node(first + i);
                    T wl[WM], w0r[WM];
                    factors(1, wl);
                    factors(0, w0r);
                    const C *base = tile + ul[0] * P1 + ul[1];
#pragma unroll
                    for (int s0 = 0; s0 < WM; ++s0) {
                        if (s0 >= lo && s0 < hi) {
                            T rx = 0, ry = 0;
#pragma unroll
                            for (int s1 = 0; s1 < WM; ++s1) {
                                const C v = lds_entry<T>(base + s0 * P1 + s1);
                                rx += wl[s1] * v.x;
                                ry += wl[s1] * v.y;
                            }
                            ax += w0r[s0] * rx;
                            ay += w0r[s0] * ry;
                        }
                    }
                }
                part[wv * 64 + lane] = C{ax, ay};
                __syncthreads();
                if (wv == 0 && i < len) {
                    const C a = part[lane], b = part[64 + lane], c2 = part[128 + lane], d2 = part[192 + lane];
                    f[nd.perm[first + i]] = C{((a.x + b.x) + c2.x) + d2.x, ((a.y + b.y) + c2.y) + d2.y};
                }
                __syncthreads();
            }
        }
    }
    __syncthreads();
}

template <typename T, int D, int WM>
__global__ __launch_bounds__(kBlock) void k_interp_nodes(Geom g, Nodes nd, const Cplx<T> *__restrict__ grid,
                                                         Cplx<T> *__restrict__ f)
{
    using C = Cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tile = reinterpret_cast<C *>(smem_raw);
    const int nchunks = nd.counters[0];
    // work items are mapped over the first min(grid, items) workgroups, XCD by XCD
    const int nwg = min((int)gridDim.x, nchunks);
    if ((int)blockIdx.x >= nwg)
        return;
    for (int c = xcd_local_id(blockIdx.x, nwg); c < nchunks; c += nwg)
        interp_item<T, D, WM>(g, nd, grid, f, c, tile);
}

// All plans of a batch in one launch: the work items of every plan, flattened in plan
// order and handed out by the dynamic queue (plans come largest first).
template <typename T, int D, int WM>
__global__ __launch_bounds__(kBlock) void k_interp_batch(const PlanDev *__restrict__ plans, int count, BatchPtrs ptrs,
                                                         int *queue)
{
    using C = Cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tile = reinterpret_cast<C *>(smem_raw);
    __shared__ int s_cnt[kMaxBatch];
    __shared__ int s_prefix[kMaxBatch + 1];
    __shared__ int s_item;
    if ((int)threadIdx.x < count)
        s_cnt[threadIdx.x] = plans[threadIdx.x].nd.counters[0];
    __syncthreads();
    batch_prefix(s_prefix, count, s_cnt);
    const int total = s_prefix[count];
    for (int it = queue_next(queue, &s_item); it < total; it = queue_next(queue, &s_item)) {
        const int p = batch_find(s_prefix, count, it);
        const PlanDev &pd = plans[p];
        interp_item<T, D, WM>(pd.g, pd.nd, static_cast<const C *>(pd.grid), static_cast<C *>(ptrs.out[p]),
                              it - s_prefix[p], tile);
    }
    queue_done(queue);
}

template <typename T, int D, int WM> constexpr auto pick_interp() { return k_interp_nodes<T, D, WM>; }

template <typename T, int D>
hipError_t interp_typed(const Geom &g, const Nodes &nd, const void *grid, void *f, int blocks, size_t lds,
                        hipStream_t s)
{
    using C = Cplx<T>;
#define CALL(W_)                                                                                       \
    {                                                                                                  \
        auto kf = pick_interp<T, D, W_>();                                                                  \
        (void)hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        hipLaunchKernelGGL(kf, dim3(blocks), dim3(kBlock), lds, s, g, nd, static_cast<const C *>(grid), \
                           static_cast<C *>(f));                                                       \
    }
    NFFT_WM_SWITCH(g.WM, CALL)
#undef CALL
    return hipGetLastError();
}
}  // namespace

// the padded tile, and for d = 2 the 4 x 64 partial sums of the nodes past the first 256
size_t interp_lds_bytes(const Geom &g, bool dbl)
{
    return ((size_t)g.Ptot + (g.d == 2 ? 256 : 0)) * (dbl ? 16 : 8);
}
// spreading tiles per workgroup: four (1-D); two (2-D) or one (3-D) followed by one dummy
// slot per thread
bool spread_in_registers(const Geom &g, bool dbl)
{
    return g.d == 2 && g.W == g.WM && g.lgB[0] == (dbl ? 4 : 5) && g.lgB[1] == 5 && g.P[1] <= 64;
}

size_t spread_lds_bytes(const Geom &g, bool dbl)
{
    const size_t cs = dbl ? 16 : 8;
    if (spread_in_registers(g, dbl)) {
        // two batch buffers per wave (factor records of 16 or 8 list entries, rounded up
        // to whole 1 KB copies, and their values), and the two tiles the waves' columns are
        // summed in, which reuse that memory
        const int kb = dbl ? 8 : 16;
        const int rec = 2 * g.WM * (int)(cs / 2) / 16;
        const size_t buf = (size_t)((kb * rec + 63) / 64) * 1024 + (dbl ? 1024 : 512);
        return std::max(4 * 2 * buf, 2 * (size_t)g.Ptot * cs);
    }
    return spread_batch_lds_bytes(g, dbl);
}

size_t spread_batch_lds_bytes(const Geom &g, bool dbl)
{
    const size_t cs = dbl ? 16 : 8;
    if (g.d == 1)
        return (size_t)g.Ptot * cs * 4;
    return ((size_t)g.Ptot * (g.d == 2 ? 2 : 1) + kBlock) * cs;
}

int fold_max_pairs(const Geom &g, int t)
{
    // brute force over the grid indices of dimension t (host copy of cover_pairs)
    int B = 1 << g.lgB[t], n = g.n[t], worst = 0;
    for (int l = 0; l < n; ++l) {
        int cnt = 0;
        for (int k = -1; k <= 1; ++k) {
            int lu = l + k * n + g.m;
            for (int b = 0; b < g.nb[t]; ++b) {
                int o = lu - b * B;
                if (o >= 0 && o < g.P[t])
                    ++cnt;
            }
        }
        if (cnt > worst)
            worst = cnt;
    }
    return worst;
}

namespace {
template <typename T, int D>
hipError_t interp_batch_typed(const PlanDev *plans, int count, const BatchPtrs &ptrs, int *queue, int WMv,
                              int blocks, size_t lds, hipStream_t s)
{
#define CALL(W_)                                                                                       \
    {                                                                                                  \
        auto kf = k_interp_batch<T, D, W_>;                                                            \
        (void)hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL(kf, dim3(blocks), dim3(kBlock), lds, s, plans, count, ptrs, queue);         \
    }
    NFFT_WM_SWITCH(WMv, CALL)
#undef CALL
    return hipGetLastError();
}
}  // namespace

hipError_t launch_interp_batch(const PlanDev *plans, int count, const BatchPtrs &ptrs, int *queue, int d,
                               bool dbl, int WMv, int blocks, size_t lds, hipStream_t s)
{
    switch (d * 2 + (dbl ? 1 : 0)) {
    case 2: return interp_batch_typed<float, 1>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    case 3: return interp_batch_typed<double, 1>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    case 4: return interp_batch_typed<float, 2>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    case 5: return interp_batch_typed<double, 2>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    case 6: return interp_batch_typed<float, 3>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    case 7: return interp_batch_typed<double, 3>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_interp(const Geom &g, const Nodes &nd, bool dbl, const void *grid, void *f, int blocks,
                         size_t lds, hipStream_t s)
{
    NFFT_DT_SWITCH(interp_typed, g, nd, grid, f, blocks, lds, s)
}

}  // namespace nfft
