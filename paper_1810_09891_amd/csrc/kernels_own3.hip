// Spreading (Algorithm 2.2 step 1) of 3-D plans by output tiles: every grid cell is written
// once, by the workgroup that owns it, as the sum over all nodes whose stencils reach it (the
// blockwise adjoint of Table 3.2, turned around so that no two workgroups write one cell and
// no floating-point atomics are needed).
//
// The grid is cut into tiles of 16 x 16 x 16 cells.  A workgroup of four waves holds one
// tile in registers: wave w owns the 16 rows (dimension 0) of the 8 x 8 block of
// (dimension 1, dimension 2) columns at (8 (w >> 1), 8 (w & 1)).  A node whose stencil starts
// at tile-relative cell (o0, o1, o2) adds the outer product of its row factors
// psi_0[r - o0] and its column values f_j psi_1[c1 - o1] psi_2[c2 - o2] to the block, so the
// block is a real (16 x K) by (K x 64 complex) matrix product over the K nodes that reach it,
// which the matrix cores take four nodes at a time.
//
// The node precomputation lists, for every tile, the nodes whose stencils reach it, each
// entry with its tile offsets and the mask of the waves' blocks it reaches (the bins around
// the tile in bin order, nodes that reach it only).  A work item is a slice of at most `cap`
// entries of one tile; items are ordered along a Morton curve of their tiles, so that the
// items that read one node's window factors run close together.  An item stages its entries
// in batches (window factors into LDS); each wave compacts the batch's entries that reach
// its block and multiplies them in.  A tile with one item writes the grid directly; the
// items of a split tile (a dense region) write partial tiles to their own slots and a second
// kernel adds the slots in item order.  In complex64 a cell's contributions are summed in two
// levels -- one batch, then the running total -- so that the FP32 rounding error of a cell
// that many nodes reach grows with the number of batches rather than of nodes.  Every sum
// has a fixed order.

#include "window_common.hpp"

namespace nfft {

namespace {

constexpr int kOwnNB = 64;  // entries staged per batch
constexpr int kOwnWaves = kBlock / 64;

__device__ __forceinline__ void own_tile_coords(const Geom &g, int tile, int *ti)
{
    int r = tile;
#pragma unroll
    for (int t = 2; t >= 0; --t) {
        ti[t] = r % g.ont[t];
        r /= g.ont[t];
    }
}

// First neighbour bin of tile index i along dimension t, wrapped into [0, nb).
__device__ __forceinline__ int own_first_bin(const Geom &g, int t, int i)
{
    if (g.oall[t])
        return 0;
    const int b = i * (g.oT[t] >> g.lgB[t]) + g.okb[t];
    return b < 0 ? b + g.nb[t] : b;
}

// Range r of the bins around the tile at coordinates ti: bin row (a0, a1) of the
// neighbourhood, part 0 or 1 of its dimension-2 bins (two parts when they wrap around).
// Returns the first sorted node and the count (possibly 0).
__device__ __forceinline__ void own_range(const Geom &g, const int32_t *__restrict__ bin_start, const int *ti, int r,
                                          int &start, int &len)
{
    const int part = r & 1;
    const int a = r >> 1;
    const int a1 = a % g.okn[1];
    const int a0 = a / g.okn[1];
    int b0 = own_first_bin(g, 0, ti[0]) + a0;
    if (b0 >= g.nb[0])
        b0 -= g.nb[0];
    int b1 = own_first_bin(g, 1, ti[1]) + a1;
    if (b1 >= g.nb[1])
        b1 -= g.nb[1];
    const int f2 = own_first_bin(g, 2, ti[2]);
    const int lo = part == 0 ? f2 : 0;
    const int hi = part == 0 ? min(f2 + g.okn[2], g.nb[2]) : max(0, f2 + g.okn[2] - g.nb[2]);
    start = 0;
    len = 0;
    if (hi > lo) {
        const int row = (b0 * g.nb[1] + b1) * g.nb[2];
        start = bin_start[row + lo];
        len = bin_start[row + hi] - start;
    }
}

// Packed entry of sorted node p for the tile with origin org: offsets o_t + 64 in bits
// 0-7, 8-15, 16-23 and the mask of the blocks the stencil reaches in bits 24-27; 0 when it
// reaches none.  Of the periodic images of the stencil only one can reach the tile
// (n_t >= tile edge + W - 1 is required).
__device__ __forceinline__ int own_meta(const Geom &g, const Nodes &nd, int p, const int *org)
{
    const int TT[3] = {kOwnTile0, kOwnTile12, kOwnTile12};
    int o[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        // u - m - org lies in (-3n/2, n) since 2m + 2 <= n: two conditional adds reduce it mod n
        int v = nd.u[t][p] - g.m - org[t];
        v += v < 0 ? g.n[t] : 0;
        v += v < 0 ? g.n[t] : 0;
        if (v >= TT[t])
            v -= g.n[t];
        o[t] = v;
    }
    int mask = 0;
    if (o[0] < kOwnTile0 && o[0] + g.W > 0) {
#pragma unroll
        for (int w = 0; w < kOwnWaves; ++w) {
            const int b1 = (w >> 1) * 8, b2 = (w & 1) * 8;
            if (o[1] < b1 + 8 && o[1] + g.W > b1 && o[2] < b2 + 8 && o[2] + g.W > b2)
                mask |= 1 << w;
        }
    }
    // a node that reaches a block has -W < o[t] < 16, so o + 64 fits in 8 bits
    return mask ? (o[0] + 64) | ((o[1] + 64) << 8) | ((o[2] + 64) << 16) | (mask << 24) : 0;
}

// ------------------------------------------------------------------ node precomputation

// One workgroup per tile: walk the bins around it (in range order) and keep the nodes that
// reach it.  FILL = false counts them (tile_count); FILL = true writes the entries (sorted
// position, packed offsets) from tile_entry[tile] on, in walk order.
template <bool FILL> __global__ __launch_bounds__(kBlock) void k_own_entries(Geom g, Nodes nd)
{
    __shared__ int s_rstart[kOwnMaxRanges];
    __shared__ int s_rcum[kOwnMaxRanges + 1];
    __shared__ int s_wcnt[kOwnWaves];
    const int tile = blockIdx.x;
    int ti[3];
    own_tile_coords(g, tile, ti);
    const int org[3] = {ti[0] * kOwnTile0, ti[1] * kOwnTile12, ti[2] * kOwnTile12};
    const int nR = g.okn[0] * g.okn[1] * 2;
    for (int r = threadIdx.x; r < nR; r += kBlock) {
        int st, ln;
        own_range(g, nd.bin_start, ti, r, st, ln);
        s_rstart[r] = st;
        s_rcum[r + 1] = ln;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s_rcum[0] = 0;
        for (int r = 0; r < nR; ++r)
            s_rcum[r + 1] += s_rcum[r];
    }
    __syncthreads();
    const int total = s_rcum[nR];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int out = FILL ? nd.tile_entry[tile] : 0;
    int kept = 0;
    for (int base = 0; base < total; base += kBlock) {
        const int e = base + threadIdx.x;
        int p = 0, meta = 0;
        if (e < total) {
            int a = 0, b = nR - 1;  // the last range r with s_rcum[r] <= e
            while (a < b) {
                const int mid = (a + b + 1) >> 1;
                if (s_rcum[mid] <= e)
                    a = mid;
                else
                    b = mid - 1;
            }
            p = s_rstart[a] + (e - s_rcum[a]);
            meta = own_meta(g, nd, p, org);
        }
        const uint64_t keep = __ballot(meta != 0);
        if (lane == 0)
            s_wcnt[wave] = __popcll(keep);
        __syncthreads();
        int before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < kOwnWaves; ++w) {
            before += w < wave ? s_wcnt[w] : 0;
            all += s_wcnt[w];
        }
        if (FILL && meta != 0) {
            const int rank = before + __popcll(keep & ((1ull << lane) - 1ull));
            reinterpret_cast<int2 *>(nd.entries)[out + rank] = int2{p, meta};
        }
        out += all;
        kept += all;
        __syncthreads();
    }
    if (!FILL && threadIdx.x == 0)
        nd.tile_count[tile] = kept;
}

// Work items of a tile with `count` entries (at least one, so that every cell is written).
__device__ __forceinline__ int own_items_of(const Geom &g, int count) { return max(1, (count + g.ocap - 1) / g.ocap); }

// One workgroup of 1024 threads: exclusive scans, over the tiles in Morton order (tile_order),
// of the entries per tile (tile_entry) and of the items per tile (tile_item), so that the
// items of tiles that share nodes -- and read the same window factors -- are consecutive and
// run at about the same time on one XCD; counters[2] = number of items.
constexpr int kOwnScan = 1024;
__global__ __launch_bounds__(kOwnScan) void k_own_scan(Geom g, Nodes nd)
{
    __shared__ int s_a[kOwnScan];
    __shared__ int s_b[kOwnScan];
    const int tid = threadIdx.x;
    const int n = g.ontiles;
    const int per = (n + kOwnScan - 1) / kOwnScan;
    const int lo = tid * per;
    const int hi = min(n, lo + per);
    auto items = [&](int i) { return own_items_of(g, nd.tile_count[nd.tile_order[i]]); };
    int sa = 0, sb = 0;
    for (int i = lo; i < hi; ++i) {
        sa += items(i);
        sb += nd.tile_count[nd.tile_order[i]];
    }
    s_a[tid] = sa;
    s_b[tid] = sb;
    __syncthreads();
    for (int off = 1; off < kOwnScan; off <<= 1) {
        const int va = tid >= off ? s_a[tid - off] : 0;
        const int vb = tid >= off ? s_b[tid - off] : 0;
        __syncthreads();
        s_a[tid] += va;
        s_b[tid] += vb;
        __syncthreads();
    }
    int ra = s_a[tid] - sa, rb = s_b[tid] - sb;
    for (int i = lo; i < hi; ++i) {
        const int t = nd.tile_order[i];
        nd.tile_item[t] = ra;
        nd.tile_entry[t] = rb;
        ra += items(i);
        rb += nd.tile_count[t];
    }
    if (tid == kOwnScan - 1) {
        nd.tile_item[n] = s_a[tid];
        nd.tile_entry[n] = s_b[tid];
        nd.counters[2] = s_a[tid];
    }
}

// The items of every tile: equal slices of its entry list.
__global__ __launch_bounds__(kBlock) void k_own_items(Geom g, Nodes nd)
{
    const int tile = blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= g.ontiles)
        return;
    const int first = nd.tile_item[tile];
    const int64_t count = nd.tile_count[tile];
    const int k = own_items_of(g, (int)count);
    for (int i = 0; i < k; ++i) {
        nd.item_tile[first + i] = tile;
        nd.item_lo[first + i] = (int)(count * i / k);
        nd.item_hi[first + i] = (int)(count * (i + 1) / k);
    }
}

// ------------------------------------------------------------------ staging and walk

// LDS record of one staged entry's factors: dimension 0 at the start (16-byte aligned),
// dimensions 1 and 2 each with 8 zeros on both sides, so that a lane whose column lies up to
// 8 cells outside the stencil reads a zero instead of branching.
template <typename T, int W> struct OwnRec {
    static constexpr int V = 16 / (int)sizeof(T);
    static constexpr int W0 = (W + V - 1) / V * V;
    static constexpr int L = W + 16;
    static constexpr int D1 = W0;
    static constexpr int D2 = W0 + L;
    static constexpr int REC = (D2 + L + V - 1) / V * V;
    static constexpr int NL = (kOwnNB * 3 * W + kBlock - 1) / kBlock;  // factor loads per thread
};

template <typename T, int W> struct OwnLds {
    T psi[kOwnNB * OwnRec<T, W>::REC];
    Cplx<T> val[kOwnNB];  // node values
    int meta[kOwnNB];
    int pos[kOwnNB];
};

// Stage entries q, q + stride, ..., q + (nb - 1) stride of the tile's list (ent): packed
// offsets, sorted positions, window factors, and with `fs` (node values in sorted order) the
// values.  Every load is issued before the first LDS store; ends with a barrier.
// The factor table holds WR <= W factors per dimension (the plan's stencil, W the compiled
// width; WR = 0: the runtime width wr, for odd m); the record entries past it stay zero.
template <typename T, int W, int WR>
__device__ __forceinline__ void own_stage(const Nodes &nd, OwnLds<T, W> &L, const int2 *__restrict__ ent, int q,
                                          int nb, const Cplx<T> *__restrict__ fs, int stride, int wr_rt)
{
    const int wr = WR > 0 ? WR : wr_rt;
    using R = OwnRec<T, W>;
    const T *__restrict__ psi = static_cast<const T *>(nd.psi);
    int2 e{0, 0};
    Cplx<T> fv{T(0), T(0)};
    if ((int)threadIdx.x < nb) {
        e = ent[q + (int)threadIdx.x * stride];
        if (fs)
            fv = fs[e.x];
    }
    T v[R::NL];
    int dst[R::NL];
#pragma unroll
    for (int j = 0; j < R::NL; ++j) {
        const int idx = threadIdx.x + j * kBlock;
        const int k = idx / (3 * wr);
        const int rr = idx - k * (3 * wr);
        const bool ok = k < nb;
        const int p = ent[q + (ok ? k : 0) * stride].x;
        v[j] = psi[(int64_t)p * (3 * wr) + (ok ? rr : 0)];
        const int t = rr / wr;
        const int s = rr - t * wr;
        dst[j] = ok ? k * R::REC + (t == 0 ? s : (t == 1 ? R::D1 + 8 + s : R::D2 + 8 + s)) : -1;
    }
    if ((int)threadIdx.x < nb) {
        L.meta[threadIdx.x] = e.y;
        L.pos[threadIdx.x] = e.x;
        if (fs)
            L.val[threadIdx.x] = fv;
    }
#pragma unroll
    for (int j = 0; j < R::NL; ++j)
        if (dst[j] >= 0)
            L.psi[dst[j]] = v[j];
    __syncthreads();
}

// ------------------------------------------------------------------ spreading on matrix cores

// A wave's 16 x 64 block of a tile (16 rows along dimension 0 by its 8 x 8 columns) is the
// sum over the nodes k that reach it of the outer product of the node's row factors
// a_k[i] = psi_0[i - o0_k] and its column values b_k[c] = f_k psi_1[c1 - o1_k] psi_2[c2 - o2_k]:
// a real 16 x K by K x 64 complex product, K the number of such nodes.  The 16 x 16 x 4 MFMA
// takes four nodes per step: operand A (16 x 4) holds the row factors times the real or the
// imaginary part of the node values (lane l: row l % 16 of node l / 16), operand B (4 x 16)
// the column factors of sixteen of the columns (lane l: column l % 16 of node l / 16), and
// eight products (four column groups, real and imaginary parts) cover the block.  Lane l
// holds output column l % 16 in four elements r: rows l / 16 + 4 r of the FP64 product and
// rows 4 (l / 16) + r of the FP32 one (measured on gfx950).
template <typename T> struct MxVec;
template <> struct MxVec<double> {
    typedef double type __attribute__((ext_vector_type(4)));
    // output row of element r in lane l
    static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct MxVec<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

__device__ __forceinline__ MxVec<double>::type mx_step(double a, double b, MxVec<double>::type c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ MxVec<float>::type mx_step(float a, float b, MxVec<float>::type c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// The MFMA form of the entry walk: the entries of the batch that reach the wave's block,
// compacted into `list` (in batch order), four per step.  Column group s of the block holds
// columns c1 = 8 (wave >> 1) + 2 s + (j >> 3), c2 = 8 (wave & 1) + (j & 7), j = 0 .. 15.
template <typename T, int W>
__device__ __forceinline__ void own_mx_batch(const T *__restrict__ psi, const Cplx<T> *__restrict__ val,
                                             const int *__restrict__ meta, const int *__restrict__ list, int cnt,
                                             int lane, int wave, typename MxVec<T>::type (&acc)[8])
{
    using R = OwnRec<T, W>;
    const int k = lane >> 4, j = lane & 15;
    const int c1b = (wave >> 1) * 8 + (j >> 3);
    const int c2 = (wave & 1) * 8 + (j & 7);
    for (int q = 0; q < cnt; q += 4) {
        const bool ok = q + k < cnt;
        const int e = list[ok ? q + k : q];
        const int em = meta[e];
        const int o0 = (em & 255) - 64, o1 = ((em >> 8) & 255) - 64, o2 = ((em >> 16) & 255) - 64;
        const T *rec = psi + e * R::REC;
        const int s0 = j - o0;  // row j of operand A
        const T a0 = rec[min(max(s0, 0), W - 1)];
        const T a = ok && s0 >= 0 && s0 < W ? a0 : T(0);
        const Cplx<T> fv = val[e];
        // the node value enters operand A (real and imaginary parts in turn), so operand B is
        // the real column factor psi_1 psi_2
        const T ax = a * fv.x, ay = a * fv.y;
        const T w2 = rec[R::D2 + 8 + c2 - o2];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const T w = rec[R::D1 + 8 + c1b + 2 * g - o1] * w2;
            acc[2 * g] = mx_step(ax, w, acc[2 * g]);
            acc[2 * g + 1] = mx_step(ay, w, acc[2 * g + 1]);
        }
    }
}

template <typename T, int W> constexpr int own_mx_waves() { return 3; }

// NARROW: the plan's stencil is narrower than the compiled width W (odd m), its factor table
// holds g.W < W factors per dimension (a separate instantiation, so that the staging of the
// common case keeps its compile-time divisions and register budget)
template <typename T, int W, bool NARROW>
__global__ __launch_bounds__(kBlock, (own_mx_waves<T, W>())) void k_spread_own_mx(Geom g, Nodes nd,
                                                                              const Cplx<T> *__restrict__ fs,
                                                                              Cplx<T> *__restrict__ grid,
                                                                              Cplx<T> *__restrict__ scratch)
{
    using C = Cplx<T>;
    using V = typename MxVec<T>::type;
    constexpr int T0 = kOwnTile0, T1 = kOwnTile12, T2 = kOwnTile12;
    constexpr int TC = T0 * T1 * T2;
    static_assert(T0 == 16 && T1 == 16 && T2 == 16, "a wave's block is 16 rows by 8 x 8 columns");
    __shared__ __align__(16) OwnLds<T, W> L;
    __shared__ int s_list[kOwnWaves][kOwnNB];

    const int nitems = nd.counters[2];
    const int nwg = min((int)gridDim.x, nitems);
    if ((int)blockIdx.x >= nwg)
        return;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int2 *__restrict__ entries = reinterpret_cast<const int2 *>(nd.entries);

    for (int i = threadIdx.x; i < kOwnNB * OwnRec<T, W>::REC; i += kBlock)
        L.psi[i] = T(0);

    for (int it = xcd_local_id(blockIdx.x, nwg); it < nitems; it += nwg) {
        const int tile = nd.item_tile[it];
        const int lo = nd.item_lo[it], hi = nd.item_hi[it];
        const int2 *ent = entries + nd.tile_entry[tile];
        int ti[3];
        own_tile_coords(g, tile, ti);
        // complex64 sums a batch's contributions first and adds them to the running total,
        // so that the rounding error of a cell grows with the number of batches, not nodes
        constexpr bool kTwoLevel = sizeof(T) == 4;
        V acc[8], tot[kTwoLevel ? 8 : 1];
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            acc[b] = V{T(0), T(0), T(0), T(0)};
            if constexpr (kTwoLevel)
                tot[b] = V{T(0), T(0), T(0), T(0)};
        }
        // batch b takes entries lo + b, lo + b + nbat, ...: entries in list order are nodes of
        // neighbouring bins, which reach the same blocks, so that consecutive entries would
        // give one wave the whole batch while the others wait at the next barrier
        const int cnt = hi - lo;
        const int nbat = (cnt + kOwnNB - 1) / kOwnNB;
        for (int b = 0; b < nbat; ++b) {
            const int nb = (cnt - b + nbat - 1) / nbat;
            __syncthreads();  // the previous batch is consumed
            own_stage<T, W, NARROW ? 0 : W>(nd, L, ent, lo + b, nb, fs, nbat, g.W);
            const int emeta = lane < nb ? L.meta[lane] : 0;
            const bool mine = emeta != 0 && ((emeta >> (24 + wave)) & 1);
            const uint64_t bits = __ballot(mine);
            if (mine)
                s_list[wave][__popcll(bits & ((1ull << lane) - 1ull))] = lane;
            // each wave reads only its own list: the LDS operations of one wave complete in
            // order, so a wave-level fence suffices
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            own_mx_batch<T, W>(L.psi, L.val, L.meta, s_list[wave], __popcll(bits), lane, wave, acc);
            if constexpr (kTwoLevel) {
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    tot[b] += acc[b];
                    acc[b] = V{T(0), T(0), T(0), T(0)};
                }
            }
        }
        if constexpr (kTwoLevel) {
#pragma unroll
            for (int b = 0; b < 8; ++b)
                acc[b] = tot[b];
        }
        // lane l holds column j = l % 16 of every column group, rows MxVec<T>::row(l, r)
        const int j = lane & 15;
        const int c1b = (wave >> 1) * 8 + (j >> 3);
        const int c2 = (wave & 1) * 8 + (j & 7);
        const int org0 = ti[0] * T0, org1 = ti[1] * T1, org2 = ti[2] * T2;
        const int nsplit = own_items_of(g, nd.tile_count[tile]);
        if (nsplit == 1) {
            const int64_t row = (int64_t)g.n[1] * g.n[2];
            const int64_t base = ((int64_t)org0 * g.n[1] + org1 + c1b) * g.n[2] + org2 + c2;
#pragma unroll
            for (int gr = 0; gr < 4; ++gr)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    grid[base + MxVec<T>::row(lane, r) * row + 2 * gr * g.n[2]] = C{acc[2 * gr][r], acc[2 * gr + 1][r]};
        } else {
            C *slot = scratch + (int64_t)it * TC;
#pragma unroll
            for (int gr = 0; gr < 4; ++gr)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    slot[(MxVec<T>::row(lane, r) * T1 + c1b + 2 * gr) * T2 + c2] = C{acc[2 * gr][r], acc[2 * gr + 1][r]};
        }
    }
}

// Node values in sorted order (read once per entry by the spreading kernel).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_own_gather(Nodes nd, const Cplx<T> *__restrict__ f, Cplx<T> *__restrict__ fs)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nd.M)
        fs[p] = f[nd.perm[p]];
}

// Split tiles: the sum of their items' partial tiles, in item order, accumulated in FP64 (a
// dense complex64 tile has tens of partial tiles, and this level of the sum then adds no
// FP32 rounding).  Workgroup (tile, y) takes kBlock cells of the tile; the partial tiles'
// loads are issued four at a time.
template <typename T, int T0>
__global__ __launch_bounds__(kBlock) void k_own_fold(Geom g, Nodes nd, const Cplx<T> *__restrict__ scratch,
                                                      Cplx<T> *__restrict__ grid)
{
    using C = Cplx<T>;
    constexpr int T1 = kOwnTile12, T2 = kOwnTile12;
    constexpr int TC = T0 * T1 * T2;
    const int tile = blockIdx.x;
    const int k = own_items_of(g, nd.tile_count[tile]);
    if (k <= 1)
        return;
    const int first = nd.tile_item[tile];
    int ti[3];
    own_tile_coords(g, tile, ti);
    const int c = blockIdx.y * kBlock + threadIdx.x;
    const int r = c / (T1 * T2);
    const int cc1 = (c / T2) % T1;
    const int cc2 = c % T2;
    const C *src = scratch + (int64_t)first * TC + c;
    double ax = src[0].x, ay = src[0].y;
    int i = 1;
    for (; i + 4 <= k; i += 4) {
        C v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            v[q] = src[(int64_t)(i + q) * TC];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ax += (double)v[q].x;
            ay += (double)v[q].y;
        }
    }
    for (; i < k; ++i) {
        const C v = src[(int64_t)i * TC];
        ax += (double)v.x;
        ay += (double)v.y;
    }
    grid[((int64_t)(ti[0] * T0 + r) * g.n[1] + ti[1] * T1 + cc1) * g.n[2] + ti[2] * T2 + cc2] = C{(T)ax, (T)ay};
}

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_own_items(const Geom &g, const Nodes &nd, hipStream_t s)
{
    hipLaunchKernelGGL(k_own_entries<false>, dim3(g.ontiles), dim3(kBlock), 0, s, g, nd);
    hipLaunchKernelGGL(k_own_scan, dim3(1), dim3(kOwnScan), 0, s, g, nd);
    hipLaunchKernelGGL(k_own_entries<true>, dim3(g.ontiles), dim3(kBlock), 0, s, g, nd);
    hipLaunchKernelGGL(k_own_items, dim3(blocks_for(g.ontiles)), dim3(kBlock), 0, s, g, nd);
    return hipGetLastError();
}

hipError_t launch_spread_own(const Geom &g, const Nodes &nd, bool dbl, const void *f, void *fs, void *grid,
                             void *scratch, int max_items, hipStream_t s)
{
    if (g.d != 3 || !g.own || g.W > g.WM || g.oT[0] != kOwnTile0)
        return hipErrorInvalidValue;
    const int blocks = max_items > 0 ? max_items : 1;
    if (dbl) {
        using C = Cplx<double>;
        hipLaunchKernelGGL(k_own_gather<double>, dim3(blocks_for(nd.M)), dim3(kBlock), 0, s, nd,
                           static_cast<const C *>(f), static_cast<C *>(fs));
#define OWN_CASE(WMV)                                                                                       \
    hipLaunchKernelGGL((g.W == g.WM ? k_spread_own_mx<double, WMV, false> : k_spread_own_mx<double, WMV, true>), \
                       dim3(blocks), dim3(kBlock), 0, s, g, nd, static_cast<const C *>(fs), static_cast<C *>(grid), \
                       static_cast<C *>(scratch))
        NFFT_WM_SWITCH(g.WM, OWN_CASE)
#undef OWN_CASE
    } else {
        using C = Cplx<float>;
        hipLaunchKernelGGL(k_own_gather<float>, dim3(blocks_for(nd.M)), dim3(kBlock), 0, s, nd,
                           static_cast<const C *>(f), static_cast<C *>(fs));
#define OWN_CASE(WMV)                                                                                       \
    hipLaunchKernelGGL((g.W == g.WM ? k_spread_own_mx<float, WMV, false> : k_spread_own_mx<float, WMV, true>), \
                       dim3(blocks), dim3(kBlock), 0, s, g, nd, static_cast<const C *>(fs), static_cast<C *>(grid), \
                       static_cast<C *>(scratch))
        NFFT_WM_SWITCH(g.WM, OWN_CASE)
#undef OWN_CASE
    }
    return hipGetLastError();
}

hipError_t launch_own_fold(const Geom &g, const Nodes &nd, bool dbl, const void *scratch, void *grid, hipStream_t s)
{
    const dim3 grid_dim(g.ontiles, kOwnTile0 * kOwnTile12 * kOwnTile12 / kBlock);
    if (dbl)
        hipLaunchKernelGGL((k_own_fold<double, kOwnTile0>), grid_dim, dim3(kBlock), 0, s, g, nd,
                           static_cast<const Cplx<double> *>(scratch), static_cast<Cplx<double> *>(grid));
    else
        hipLaunchKernelGGL((k_own_fold<float, kOwnTile0>), grid_dim, dim3(kBlock), 0, s, g, nd,
                           static_cast<const Cplx<float> *>(scratch), static_cast<Cplx<float> *>(grid));
    return hipGetLastError();
}

}  // namespace nfft
