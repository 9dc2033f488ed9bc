// Gradient of the interpolation (Algorithm 2.1 step 3) with respect to the nodes.
// Geometry as in window_common.hpp.
#include "window_common.hpp"

namespace nfft {

namespace {

using namespace window;

// ------------------------------------------------------------------ gradient

// The sums of one 3-D node's stencil plane s0 (tile plane `plane`): acc[0] gets the
// derivative in dimension 0, acc[1] and acc[2] those in dimensions 1 and 2.
template <typename T, int WM, bool AllW>
__device__ __forceinline__ void grad_plane(const Geom &g, const Nodes &nd, T d0, int s0, const Cplx<T> *plane,
                                           const T *wl, const T *dwl, const T *wmid, const T *dwmid, Cplx<T> *acc)
{
    using C = Cplx<T>;
    const T w0 = win_value<T, AllW>(g, nd, 0, d0, s0);
    const T dw0 = win_value_d<T, AllW>(g, nd, 0, d0, s0);
    const int P2 = g.P[2];
    T px = 0, py = 0, qx = 0, qy = 0, hx = 0, hy = 0;
#pragma unroll
    for (int s1 = 0; s1 < WM; ++s1) {
        const C *row = plane + s1 * P2;
        T rx = 0, ry = 0, dx = 0, dy = 0;
#pragma unroll
        for (int s2 = 0; s2 < WM; ++s2) {
            const C gv = lds_entry<T>(row + s2);
            rx += wl[s2] * gv.x;
            ry += wl[s2] * gv.y;
            dx += dwl[s2] * gv.x;
            dy += dwl[s2] * gv.y;
        }
        px += wmid[s1] * rx;  // plain in dims 1, 2
        py += wmid[s1] * ry;
        qx += dwmid[s1] * rx;  // derivative in dim 1
        qy += dwmid[s1] * ry;
        hx += wmid[s1] * dx;  // derivative in dim 2
        hy += wmid[s1] * dy;
    }
    acc[0].x += dw0 * px;
    acc[0].y += dw0 * py;
    acc[1].x += w0 * qx;
    acc[1].y += w0 * qy;
    acc[2].x += w0 * hx;
    acc[2].y += w0 * hy;
}

// grad[j][t] of node j from its three derivative sums (NaN for a non-finite node).
template <typename T, int D>
__device__ __forceinline__ void grad_store(const Geom &g, const Cplx<T> vj, const T *dl, const Cplx<T> *acc,
                                           T *__restrict__ grad, int j)
{
    bool finite = true;  // a non-finite node (offset NaN) gets a NaN gradient
#pragma unroll
    for (int t = 0; t < D; ++t)
        finite = finite && !isnan(dl[t]);
#pragma unroll
    for (int t = 0; t < D; ++t)
        grad[(int64_t)j * D + t] = finite ? (T)g.n[t] * (vj.x * acc[t].x + vj.y * acc[t].y) : __builtin_nan("");
}

// One work item of a 3-D plan whose padded tile is staged in slabs (g.islab > 0, at most
// kBlock nodes): each thread keeps its node's sums across the slabs, adding the stencil
// planes each slab holds in plane order, as the whole-tile gather does.
template <typename T, int WM, bool AllW>
__device__ __forceinline__ void grad_item_slab(const Geom &g, const Nodes &nd, const Cplx<T> *__restrict__ grid,
                                               const Cplx<T> *__restrict__ v, T *__restrict__ grad, int c,
                                               Cplx<T> *tile)
{
    using C = Cplx<T>;
    const int first = nd.chunk_first[c];
    const int len = nd.chunk_len[c];
    int bc[kMaxDim];
    bin_coords<T, 3>(g, nd.chunk_bin[c], bc);
    const bool has = (int)threadIdx.x < len;
    const int node = first + (has ? (int)threadIdx.x : 0);
    int ul[3];
    T dl[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        ul[t] = nd.u[t][node] & ((1 << g.lgB[t]) - 1);
        dl[t] = static_cast<const T *>(nd.delta[t])[node];
    }
    T wl[WM], dwl[WM], wmid[WM], dwmid[WM];
    window_row_d<T, WM, AllW>(dl[2], g, nd, 2, wl, dwl);
    window_row_d<T, WM, AllW>(dl[1], g, nd, 1, wmid, dwmid);
    C acc[3] = {C{T(0), T(0)}, C{T(0), T(0)}, C{T(0), T(0)}};
    const int P0 = g.P[0], P1 = g.P[1], P2 = g.P[2];
    for (int z0 = 0; z0 < P0; z0 += g.islab) {
        const int S = min(g.islab, P0 - z0);
        __syncthreads();  // the previous slab is consumed
        stage_slab<T>(g, bc, z0, S, grid, tile);
        __syncthreads();
        if (has) {
            const int lo = max(0, z0 - ul[0]), hi = min(g.W, z0 + S - ul[0]);
            for (int s0 = lo; s0 < hi; ++s0)
                grad_plane<T, WM, AllW>(g, nd, dl[0], s0, tile + ((ul[0] + s0 - z0) * P1 + ul[1]) * P2 + ul[2], wl,
                                        dwl, wmid, dwmid, acc);
        }
    }
    if (has) {
        const int j = nd.perm[node];
        grad_store<T, 3>(g, v[j], dl, acc, grad, j);
    }
    __syncthreads();
}

// grad[j][t] = Re(conj(v_j) * n_t * sum_s g[u+s] phi_t'(.) prod_{t' != t} phi_t'(.)).
template <typename T, int D, int WM, bool AllW>
__global__ __launch_bounds__(kBlock) void k_grad_x(Geom g, Nodes nd, const Cplx<T> *__restrict__ grid,
                                                   const Cplx<T> *__restrict__ v, T *__restrict__ grad)
{
    using C = Cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tile = reinterpret_cast<C *>(smem_raw);
    const int nchunks = nd.counters[0];
    // work items are mapped over the first min(grid, items) workgroups, XCD by XCD
    const int nwg = min((int)gridDim.x, nchunks);
    if ((int)blockIdx.x >= nwg)
        return;
    for (int c = xcd_local_id(blockIdx.x, nwg); c < nchunks; c += nwg) {
        if constexpr (D == 3) {
            if (g.islab > 0) {
                grad_item_slab<T, WM, AllW>(g, nd, grid, v, grad, c, tile);
                continue;
            }
        }
        const int bin = nd.chunk_bin[c];
        const int first = nd.chunk_first[c];
        const int len = nd.chunk_len[c];
        int bc[kMaxDim];
        bin_coords<T, D>(g, bin, bc);
        stage_tile<T, D>(g, bc, grid, tile);
        __syncthreads();
        for (int i = threadIdx.x; i < len; i += kBlock) {
            const int node = first + i;
            int ul[kMaxDim];
            T dl[kMaxDim];
#pragma unroll
            for (int t = 0; t < D; ++t) {
                ul[t] = nd.u[t][node] & ((1 << g.lgB[t]) - 1);
                dl[t] = static_cast<const T *>(nd.delta[t])[node];
            }
            T wl[WM], dwl[WM];
            window_row_d<T, WM, AllW>(dl[D - 1], g, nd, D - 1, wl, dwl);
            C acc[kMaxDim];
#pragma unroll
            for (int t = 0; t < D; ++t)
                acc[t] = C{T(0), T(0)};
            if constexpr (D == 1) {
                const C *row = tile + ul[0];
#pragma unroll
                for (int s = 0; s < WM; ++s) {
                    const C gv = lds_entry<T>(row + s);
                    acc[0].x += dwl[s] * gv.x;
                    acc[0].y += dwl[s] * gv.y;
                }
            } else if constexpr (D == 2) {
                for (int s0 = 0; s0 < g.W; ++s0) {
                    const T w0 = win_value<T, AllW>(g, nd, 0, dl[0], s0);
                    const T dw0 = win_value_d<T, AllW>(g, nd, 0, dl[0], s0);
                    const C *row = tile + (ul[0] + s0) * g.P[1] + ul[1];
                    T rx = 0, ry = 0, dx = 0, dy = 0;
#pragma unroll
                    for (int s1 = 0; s1 < WM; ++s1) {
                        const C gv = lds_entry<T>(row + s1);
                        rx += wl[s1] * gv.x;
                        ry += wl[s1] * gv.y;
                        dx += dwl[s1] * gv.x;
                        dy += dwl[s1] * gv.y;
                    }
                    acc[0].x += dw0 * rx;
                    acc[0].y += dw0 * ry;
                    acc[1].x += w0 * dx;
                    acc[1].y += w0 * dy;
                }
            } else {
                T wmid[WM], dwmid[WM];
                window_row_d<T, WM, AllW>(dl[1], g, nd, 1, wmid, dwmid);
                const int P1 = g.P[1], P2 = g.P[2];
                for (int s0 = 0; s0 < g.W; ++s0)
                    grad_plane<T, WM, AllW>(g, nd, dl[0], s0, tile + ((ul[0] + s0) * P1 + ul[1]) * P2 + ul[2], wl,
                                            dwl, wmid, dwmid, acc);
            }
            const int j = nd.perm[node];
            grad_store<T, D>(g, v[j], dl, acc, grad, j);
        }
        __syncthreads();
    }
}



template <typename T, int D>
hipError_t grad_typed(const Geom &g, const Nodes &nd, const void *grid, const void *v, void *grad, int blocks,
                      size_t lds, hipStream_t s)
{
    using C = Cplx<T>;
#define CALL(W_)                                                                                       \
    {                                                                                                  \
        auto kf = window_needs_all(g) ? k_grad_x<T, D, W_, true> : k_grad_x<T, D, W_, false>;         \
        (void)hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        hipLaunchKernelGGL(kf, dim3(blocks), dim3(kBlock), lds, s, g, nd, static_cast<const C *>(grid), \
                           static_cast<const C *>(v), static_cast<T *>(grad));                         \
    }
    NFFT_WM_SWITCH(g.WM, CALL)
#undef CALL
    return hipGetLastError();
}
}  // namespace

hipError_t launch_grad_x(const Geom &g, const Nodes &nd, bool dbl, const void *grid, const void *v, void *grad,
                         int blocks, size_t lds, hipStream_t s)
{
    NFFT_DT_SWITCH(grad_typed, g, nd, grid, v, grad, blocks, lds, s)
}

}  // namespace nfft
