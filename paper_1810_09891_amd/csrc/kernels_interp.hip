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
#include <algorithm>

#include "batch_desc.hpp"
#include "window_common.hpp"

namespace nfft {

namespace {

using namespace window;

// ------------------------------------------------------------------ interpolation

// One work item c of a 3-D plan whose padded tile exceeds the LDS (g.islab > 0, at most
// kBlock nodes per item): the tile is staged g.islab planes at a time, and each thread keeps
// its node's sum across the slabs, adding the planes of its stencil that each slab holds in
// plane order -- the same sums in the same order as with the whole tile.
template <typename T, int WM>
__device__ __forceinline__ void interp_item_slab(const Geom &g, const Nodes &nd, const Cplx<T> *__restrict__ grid,
                                                 Cplx<T> *__restrict__ f, int c, Cplx<T> *tile)
{
    using C = Cplx<T>;
    const T *psi = static_cast<const T *>(nd.psi);
    const int W = g.W;
    const int first = nd.chunk_first[c];
    const int len = nd.chunk_len[c];
    int bc[kMaxDim];
    bin_coords<T, 3>(g, nd.chunk_bin[c], bc);
    const bool has = (int)threadIdx.x < len;
    const int node = first + (has ? (int)threadIdx.x : 0);
    int ul[3];
#pragma unroll
    for (int t = 0; t < 3; ++t)
        ul[t] = nd.u[t][node] & ((1 << g.lgB[t]) - 1);
    const T *pw = psi + (int64_t)node * 3 * W;  // window factors [3][W] of this node
    T w1[WM], w2[WM];
#pragma unroll
    for (int s = 0; s < WM; ++s) {
        w1[s] = s < W ? pw[W + s] : T(0);
        w2[s] = s < W ? pw[2 * W + s] : T(0);
    }
    const int P0 = g.P[0], P1 = g.P[1], P2 = g.P[2];
    T ax = 0, ay = 0;
    for (int z0 = 0; z0 < P0; z0 += g.islab) {
        const int S = min(g.islab, P0 - z0);
        __syncthreads();  // the previous slab is consumed
        stage_slab<T>(g, bc, z0, S, grid, tile);
        __syncthreads();
        if (has) {
            const int lo = max(0, z0 - ul[0]), hi = min(W, z0 + S - ul[0]);
            for (int s0 = lo; s0 < hi; ++s0) {
                const T w0 = pw[s0];
                const C *plane = tile + ((ul[0] + s0 - z0) * P1 + ul[1]) * P2 + ul[2];
                T px = 0, py = 0;
#pragma unroll
                for (int s1 = 0; s1 < WM; ++s1) {
                    T rx = 0, ry = 0;
#pragma unroll
                    for (int s2 = 0; s2 < WM; ++s2) {
                        const C v = lds_entry<T>(plane + s1 * P2 + s2);
                        rx += w2[s2] * v.x;
                        ry += w2[s2] * v.y;
                    }
                    px += w1[s1] * rx;
                    py += w1[s1] * ry;
                }
                ax += w0 * px;
                ay += w0 * py;
            }
        }
    }
    if (has)
        f[nd.perm[node]] = C{ax, ay};
    __syncthreads();
}

// One work item c of a plan: stage the bin's padded tile, then interpolate its nodes.
template <typename T, int D, int WM>
__device__ __forceinline__ void interp_item(const Geom &g, const Nodes &nd, const Cplx<T> *__restrict__ grid,
                                            Cplx<T> *__restrict__ f, int c, Cplx<T> *tile)
{
    using C = Cplx<T>;
    if constexpr (D == 3) {
        if (g.islab > 0) {
            interp_item_slab<T, WM>(g, nd, grid, f, c, tile);
            return;
        }
    }
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

// ------------------------------------------------------------------ 3-D interpolation by lane groups
//
// In 3-D a node's stencil has (2m+2)^3 points, and one thread per node reads its stencil
// rows at scattered tile offsets: the LDS reads of a wave conflict on banks (three conflict
// cycles per LDS cycle measured in complex128).  Here G lanes share a node (G = 16 for
// stencils of at most 16 points per dimension, else 32): lane s takes column s of the
// innermost dimension and sums psi_0[s0] sum_{s1} psi_1[s1] g[u0+s0][u1+s1][u2+s] over the
// two outer dimensions, one tile entry per (s0, s1), so the lanes of a group read one
// contiguous row; the column sums are multiplied by psi_2[s] and added over the group by a
// butterfly (a fixed order).  The next round's node data is loaded while the current round
// is summed.
//
// A workgroup has eight waves.  Waves 0-3 interpolate the nodes of the current work item;
// waves 4-7 meanwhile load the padded tile of their next work item into registers (up to
// i3_keep entries per thread) and, after a barrier, write it to LDS, so that the tile loads
// of one item overlap the sums of the previous one.  Workgroups are persistent.
constexpr int kI3Threads = 512;
constexpr int kI3Half = 256;
// tile entries a loading thread keeps in registers: a whole tile of 21^3 entries (m = 6 and
// 8^3 bins) and, in complex128, any tile that fits the LDS; complex64 stays within 128
// registers, so that two workgroups of eight waves share a compute unit
template <typename T> constexpr int i3_keep() { return sizeof(T) == 8 ? 40 : 37; }

// Data-parallel-primitive lane moves within rows of 16 lanes (no LDS): quad permutations,
// the half-row mirror (lane i <-> 7 - i within each 8) and the row mirror (i <-> 15 - i).
template <int CTRL> __device__ __forceinline__ float dpp_move(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// Sum over each row of 16 lanes, every lane receiving its row's sum: pairs, quads, eights,
// then the two halves of the row (a fixed order).
template <typename T> __device__ __forceinline__ T row16_sum(T v)
{
    v += dpp_move<0xB1>(v);   // quad_perm [1, 0, 3, 2]
    v += dpp_move<0x4E>(v);   // quad_perm [2, 3, 0, 1]
    v += dpp_move<0x141>(v);  // row_half_mirror
    v += dpp_move<0x140>(v);  // row_mirror
    return v;
}

template <typename T, int WM>
__device__ __forceinline__ void interp3_item(const Geom &g, const Nodes &nd, Cplx<T> *__restrict__ f, int c,
                                             const Cplx<T> *tile)
{
    using C = Cplx<T>;
    constexpr int G = WM <= 16 ? 16 : 32;
    constexpr int NG = kI3Half / G;  // nodes per round
    const T *psi = static_cast<const T *>(nd.psi);
    const int tid = threadIdx.x;  // < kI3Half
    const int grp = tid / G;
    const int s2 = tid & (G - 1);
    const int W = g.W;
    const int dW = 3 * W;
    const int first = nd.chunk_first[c];
    const int len = nd.chunk_len[c];
    const int P1 = g.P[1], P2 = g.P[2];
    const int s2c = s2 < WM ? s2 : WM - 1;  // lanes past the stencil read a valid entry, weight 0
    const int s2w = s2 < W ? s2 : W - 1;
    // Node data as loaded (cell indices, factor pairs), consumed only in the round that
    // uses it, so that the loads of the next round stay in flight during this one.
    struct NodeData {
        int u0, u1, u2;
        Pair<T> w0[WM / 2], w1[WM / 2];
        T w2;
    };
    auto load = [&](int i, NodeData &q) {
        const int node = first + (i < len ? i : len - 1);
        q.u0 = nd.u[0][node];
        q.u1 = nd.u[1][node];
        q.u2 = nd.u[2][node];
        // aligned pairs (W and the record length 3W are even; reads stay inside the record)
        const Pair<T> *p2 = reinterpret_cast<const Pair<T> *>(psi + (int64_t)node * dW);
#pragma unroll
        for (int s = 0; s < WM / 2; ++s) {
            q.w0[s] = p2[s];
            q.w1[s] = p2[W / 2 + s];
        }
        q.w2 = psi[(int64_t)node * dW + 2 * W + s2w];
    };
    NodeData cur, nxt;
    if (len > 0)
        load(grp, cur);
    for (int base = 0; base < len; base += NG) {
        const int i = base + grp;
        if (base + NG < len)
            load(i + NG, nxt);
        T w0[WM], w1[WM];  // factors of dimensions 0 and 1, zero past W
#pragma unroll
        for (int s = 0; s < WM / 2; ++s) {
            w0[2 * s] = 2 * s < W ? cur.w0[s].x : T(0);
            w0[2 * s + 1] = 2 * s + 1 < W ? cur.w0[s].y : T(0);
            w1[2 * s] = 2 * s < W ? cur.w1[s].x : T(0);
            w1[2 * s + 1] = 2 * s + 1 < W ? cur.w1[s].y : T(0);
        }
        const T w2 = s2 < W ? cur.w2 : T(0);
        const int off = ((cur.u0 & ((1 << g.lgB[0]) - 1)) * P1 + (cur.u1 & ((1 << g.lgB[1]) - 1))) * P2 +
                        (cur.u2 & ((1 << g.lgB[2]) - 1)) + s2c;
        // Planes are read one ahead of their sums where the registers allow: the WM reads of
        // plane s0 + 1 are issued before plane s0 is summed.  Planes past W carry weight zero
        // and stay inside the tile.
        constexpr bool kAhead = sizeof(T) == 8 ? WM <= 14 : WM <= 10;
        const C *p = tile + off;
        const int PP = P1 * P2;
        C row[WM];
        if constexpr (kAhead) {
#pragma unroll
            for (int s1 = 0; s1 < WM; ++s1)
                row[s1] = p[s1 * P2];
        }
        T ax = 0, ay = 0;
#pragma unroll
        for (int s0 = 0; s0 < WM; ++s0) {
            C ahead[WM];
            if (kAhead && s0 + 1 < WM) {
#pragma unroll
                for (int s1 = 0; s1 < WM; ++s1)
                    ahead[s1] = p[(s0 + 1) * PP + s1 * P2];
            }
            if constexpr (!kAhead) {
#pragma unroll
                for (int s1 = 0; s1 < WM; ++s1)
                    row[s1] = p[s0 * PP + s1 * P2];
            }
            T rx = 0, ry = 0;
#pragma unroll
            for (int s1 = 0; s1 < WM; ++s1) {
                rx = fma(w1[s1], row[s1].x, rx);
                ry = fma(w1[s1], row[s1].y, ry);
            }
            ax = fma(w0[s0], rx, ax);
            ay = fma(w0[s0], ry, ay);
            if (kAhead && s0 + 1 < WM) {
#pragma unroll
                for (int s1 = 0; s1 < WM; ++s1)
                    row[s1] = ahead[s1];
            }
        }
        ax *= w2;
        ay *= w2;
        ax = row16_sum(ax);
        ay = row16_sum(ay);
        if constexpr (G == 32) {  // the two rows of a 32-lane group
            ax += __shfl_xor(ax, 16, 32);
            ay += __shfl_xor(ay, 16, 32);
        }
        if (i < len && s2 == 0)
            f[nd.perm[first + i]] = C{ax, ay};
        cur = nxt;
    }
}

// Tile entries from `from` on, staged by all threads of the workgroup (eight loads in
// flight per thread).  Stores past the tile go to the dummy entry after it, so that every
// store is unconditional and the loads are not sunk into per-entry branches (which would
// serialise them).
template <typename T, bool P2>
__device__ __forceinline__ void stage_rest3(const Geom &g, const int *bc, const Cplx<T> *grid, Cplx<T> *tile, int from)
{
    using C = Cplx<T>;
    constexpr int K = 8;
    const TileMap<3, P2> map(g, bc);
    const int Ptot = g.Ptot;
    for (int base = from; base < Ptot; base += K * kI3Threads) {
        T vx[K], vy[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = base + threadIdx.x + k * kI3Threads;
            const C a = grid[map.src(g, idx < Ptot ? idx : 0)];
            vx[k] = a.x;
            vy[k] = a.y;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = base + threadIdx.x + k * kI3Threads;
            tile[idx < Ptot ? idx : Ptot] = C{vx[k], vy[k]};
        }
    }
}

// One step of the loading waves: the padded tile of work item cn is loaded into registers
// (entries ptid + k kI3Half, k < count), the workgroup meets at a barrier (the current item's
// sums are done with the tile), and the entries are written to LDS, the rest of the tile
// staged by all threads, and the workgroup meets again.  Grids of fewer than 2^28 cells
// index the grid with 32-bit offsets; larger ones keep half as many entries.
template <typename T, bool P2, bool O32>
__device__ __forceinline__ void loader_step(const Geom &g, const Nodes &nd, const Cplx<T> *__restrict__ grid,
                                            Cplx<T> *tile, int cn, int nchunks, int ptid)
{
    using C = Cplx<T>;
    constexpr int K = O32 ? i3_keep<T>() : i3_keep<T>() / 2;
    T vx[K], vy[K];  // real arrays, so that they are kept in registers
    int bc[3] = {0, 0, 0};
    const bool more = cn < nchunks;
    if (more) {
        bin_coords<T, 3>(g, nd.chunk_bin[cn], bc);
        const TileMap<3, P2> map(g, bc);
        const int Ptot = g.Ptot;
        // The tile coordinates of a thread's entries are the same for every item; an empty
        // asm statement hides that, so that they are recomputed here rather than kept in K
        // times three registers across the loop (it emits no instruction).
        int pt = ptid;
        asm volatile("" : "+v"(pt));
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = pt + k * kI3Half;
            const int e = idx < Ptot ? idx : 0;
            // 32-bit byte offsets from the uniform grid base (one address register per load)
            const C a = O32 ? *reinterpret_cast<const C *>(reinterpret_cast<const char *>(grid) +
                                                            map.src32(g, e) * (uint32_t)sizeof(C))
                            : grid[map.src(g, e)];
            vx[k] = a.x;
            vy[k] = a.y;
        }
    }
    __syncthreads();  // the item's sums are done with the tile
    if (more) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int idx = ptid + k * kI3Half;
            tile[idx < g.Ptot ? idx : g.Ptot] = C{vx[k], vy[k]};  // past the tile: the dummy entry
        }
        if (g.Ptot > K * kI3Half)
            stage_rest3<T, P2>(g, bc, grid, tile, K * kI3Half);
    }
    __syncthreads();
}

template <typename T, int WM>
__global__ __launch_bounds__(kI3Threads) void k_interp3(Geom g, Nodes nd, const Cplx<T> *__restrict__ grid,
                                                         Cplx<T> *__restrict__ f)
{
    using C = Cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tile = reinterpret_cast<C *>(smem_raw);
    const int nchunks = nd.counters[0];
    const int nwg = min((int)gridDim.x, nchunks);
    if ((int)blockIdx.x >= nwg)
        return;
    const bool loader = threadIdx.x >= kI3Half;  // waves 4-7
    const int ptid = (int)threadIdx.x - kI3Half;
    // entries kept per loading thread: i3_keep with 32-bit offsets, half otherwise
    const bool o32 = (int64_t)g.n[0] * g.n[1] * g.n[2] < ((int64_t)1 << 28);
    const int keep = (o32 ? i3_keep<T>() : i3_keep<T>() / 2) * kI3Half;
    int c = xcd_local_id(blockIdx.x, nwg);
    {
        int bc[3];
        bin_coords<T, 3>(g, nd.chunk_bin[c], bc);
        if (g.p2)
            stage_rest3<T, true>(g, bc, grid, tile, 0);
        else
            stage_rest3<T, false>(g, bc, grid, tile, 0);
    }
    __syncthreads();
    // The two kinds of waves run separate loops with the same barriers, so that the kept
    // tile and the interpolation registers are never live together.
    if (loader) {
        for (; c < nchunks; c += nwg) {
            if (o32) {
                if (g.p2)
                    loader_step<T, true, true>(g, nd, grid, tile, c + nwg, nchunks, ptid);
                else
                    loader_step<T, false, true>(g, nd, grid, tile, c + nwg, nchunks, ptid);
            } else {
                if (g.p2)
                    loader_step<T, true, false>(g, nd, grid, tile, c + nwg, nchunks, ptid);
                else
                    loader_step<T, false, false>(g, nd, grid, tile, c + nwg, nchunks, ptid);
            }
        }
    } else {
        for (; c < nchunks; c += nwg) {
            const int cn = c + nwg;
            interp3_item<T, WM>(g, nd, f, c, tile);
            __syncthreads();
            if (cn < nchunks && g.Ptot > keep) {
                int bcn[3];
                bin_coords<T, 3>(g, nd.chunk_bin[cn], bcn);
                if (g.p2)
                    stage_rest3<T, true>(g, bcn, grid, tile, keep);
                else
                    stage_rest3<T, false>(g, bcn, grid, tile, keep);
            }
            __syncthreads();
        }
    }
}

template <typename T, int D, int WM> constexpr auto pick_interp() { return k_interp_nodes<T, D, WM>; }

template <typename T, int D>
hipError_t interp_typed(const Geom &g, const Nodes &nd, const void *grid, void *f, int blocks, size_t lds,
                        hipStream_t s)
{
    using C = Cplx<T>;
    // 3-D by lane groups, except complex128 stencils of 22 or more points, whose registers
    // do not fit eight waves, and plans staged in slabs (those take the kernel with one node
    // per thread)
    if (D == 3 && g.islab == 0 && !(sizeof(T) == 8 && g.WM >= 22)) {
        // persistent workgroups of eight waves: as many as are resident at once (registers
        // and LDS), never more than the work items
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
#define CALL3(W_)                                                                                      \
        {                                                                                              \
            auto kf = k_interp3<T, W_>;                                                                \
            (void)hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
            int per_cu = 0;                                                                            \
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)kf, kI3Threads, lds) != \
                    hipSuccess || per_cu < 1)                                                          \
                per_cu = 1;                                                                            \
            const int wgs = std::max(1, std::min(blocks, cus * per_cu));                               \
            hipLaunchKernelGGL(kf, dim3(wgs), dim3(kI3Threads), lds, s, g, nd, static_cast<const C *>(grid), \
                               static_cast<C *>(f));                                                   \
        }
        NFFT_WM_SWITCH(g.WM, CALL3)
#undef CALL3
        return hipGetLastError();
    }
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

// the padded tile, for d = 2 the 4 x 64 partial sums of the nodes past the first 256, for
// d = 3 one dummy entry after the tile (the target of stores past it)
size_t interp_lds_bytes(const Geom &g, bool dbl)
{
    if (g.islab > 0)
        return (size_t)g.islab * g.P[1] * g.P[2] * (dbl ? 16 : 8);
    return ((size_t)g.Ptot + (g.d == 2 ? 256 : 0) + (g.d == 3 ? 1 : 0)) * (dbl ? 16 : 8);
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
