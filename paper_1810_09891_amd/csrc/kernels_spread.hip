// Spreading (Algorithm 2.2 step 1): LDS tile accumulation per work item and the
// deterministic fold of the tiles into the grid.  Geometry as in window_common.hpp.
#include <type_traits>
#include <utility>

#include "batch_desc.hpp"
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
//  * 1-D: each of the four waves of a workgroup accumulates a quarter of the work item's
//    nodes into its own padded tile (lanes over the stencil points); the four tiles are
//    summed in wave order when the item is done.
//  * 2-D: lane (r, s1) with s1 = lane mod WM, r = lane / WM covers stencil column s1 and
//    R = 64 / WM rows per pass.  The waves form two pairs, each pair with its own tile and
//    half of the work item's nodes; the two waves of a pair own the tile rows of even and
//    odd index and update those rows of every node's stencil.  The two tiles are summed
//    when the item is done.
//  * 3-D: the four waves share one padded tile; wave w owns the tile planes with index
//    w mod 4 and updates those planes of every node's stencil, lanes covering (s1, s2)
//    like the rows and columns above (no barrier between nodes).

constexpr int kWaves = kBlock / 64;
constexpr int kBatch = 16;  // nodes whose data a wave loads at once


// Value of v in the lane whose index times 4 is `byte_idx` (precomputed shuffle address).
__device__ __forceinline__ float bperm(int byte_idx, float v)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_idx, __float_as_int(v)));
}
__device__ __forceinline__ double bperm(int byte_idx, double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(byte_idx, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(byte_idx, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Value of lane k (k wave-uniform) in every lane.
__device__ __forceinline__ int bcast(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ float bcast(float v, int k)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double bcast(double v, int k)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One work item c: accumulate its nodes into LDS tiles, write the summed tile to its slot.
template <typename T, int D, int WM>
__device__ __forceinline__ void spread_item(const Geom &g, const Nodes &nd, const Cplx<T> *__restrict__ f,
                                            Cplx<T> *__restrict__ scratch, int c, Cplx<T> *tiles)
{
    using C = Cplx<T>;
    const T *psi = static_cast<const T *>(nd.psi);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int W = g.W;
    const int dW = D * W;
    // lane layout over the stencil, fixed by the compiled width WM: R rows of WM columns
    constexpr int R = 64 / WM;
    constexpr int NPASS = (WM + R - 1) / R;
    const int r = lane / WM;
    const int sc = lane - r * WM;  // stencil column of this lane
    const bool lane_ok = r < R && sc < W;
    const int first = nd.chunk_first[c];
    const int len = nd.chunk_len[c];
    if constexpr (D == 1) {
        C *sub = tiles + wave * g.Ptot;
        for (int i = lane; i < g.Ptot; i += 64)
            sub[i] = C{T(0), T(0)};
        // this wave's contiguous share of the work item, in batches of kBatch nodes whose
        // data is loaded one batch ahead (one node per lane; window factor l in lane l)
        const int lo = first + (len * wave) / kWaves;
        const int hi = first + (len * (wave + 1)) / kWaves;
        T fx = 0, fy = 0, wv[kBatch];
        int u0 = 0;
        auto load_batch = [&](int b0, T &lfx, T &lfy, int &lu0, T *lwv) {
            const int nb = min(kBatch, hi - b0);
            lfx = lfy = T(0);
            lu0 = 0;
            if (lane < nb) {
                const C fv = f[nd.perm[b0 + lane]];
                lfx = fv.x;
                lfy = fv.y;
                lu0 = nd.u[0][b0 + lane] & ((1 << g.lgB[0]) - 1);
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k)
                lwv[k] = (k < nb && lane < dW) ? psi[(int64_t)(b0 + k) * dW + lane] : T(0);
        };
        if (lo < hi)
            load_batch(lo, fx, fy, u0, wv);
        for (int b0 = lo; b0 < hi; b0 += kBatch) {
            const int nb = min(kBatch, hi - b0);
            T nfx = 0, nfy = 0, nwv[kBatch];
            int nu0 = 0;
            if (b0 + kBatch < hi)
                load_batch(b0 + kBatch, nfx, nfy, nu0, nwv);
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                if (k >= nb)
                    break;
                const T fxk = bcast(fx, k), fyk = bcast(fy, k);
                const int ul0 = bcast(u0, k);
                if (lane < W) {
                    C v = sub[ul0 + lane];
                    v.x += fxk * wv[k];
                    v.y += fyk * wv[k];
                    sub[ul0 + lane] = v;
                }
            }
            fx = nfx;
            fy = nfy;
            u0 = nu0;
#pragma unroll
            for (int k = 0; k < kBatch; ++k)
                wv[k] = nwv[k];
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
    } else if constexpr (D == 2) {
        // Two pairs of waves, each pair with its own padded tile and half of the work
        // item's nodes; in a pair, wave `par` owns the tile rows with index parity par and
        // updates those rows of every node's stencil (no two waves touch the same cell).
        constexpr int NR = WM / 2;                // stencil rows of one parity (WM is even)
        constexpr int NP2 = (NR + R - 1) / R;     // passes over them
        const int grp = wave >> 1, par = wave & 1;
        for (int i = threadIdx.x; i < 2 * g.Ptot; i += kBlock)
            tiles[i] = C{T(0), T(0)};
        __syncthreads();
        const int lo = first + (len * grp) / 2;
        const int hi = first + (len * (grp + 1)) / 2;
        const int P1 = g.P[1];
        // Per-lane constants of the item, for stencil row parity p = 0, 1 and pass q: the
        // lane's tile index relative to the node's base cell (plus the pair's tile offset),
        // and the shuffle address of its row factor.  Lanes with nothing to update in a pass
        // (outside the stencil) get a private dummy slot after the two tiles instead, so the
        // per-node code runs without predication: index = ok * base + A.
        int A[2][NP2], okv[2][NP2], widx[2][NP2];
        const int dummy = 2 * g.Ptot + wave * 64 + lane;
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < NP2; ++q) {
                const int s0 = p + 2 * (q * R + r);
                const bool ok = lane_ok && s0 < W;
                A[p][q] = ok ? grp * g.Ptot + s0 * P1 + sc : dummy;
                okv[p][q] = ok ? 1 : 0;
                widx[p][q] = (ok ? s0 : 0) * 4;
            }
        const int w1idx = (W + (sc < W ? sc : 0)) * 4;
        T fx = 0, fy = 0, wv[kBatch];
        int u0 = 0, u1 = 0;
        auto load_batch = [&](int b0, T &lfx, T &lfy, int &lu0, int &lu1, T *lwv) {
            const int nb = min(kBatch, hi - b0);
            lfx = lfy = T(0);
            lu0 = lu1 = 0;
            if (lane < nb) {
                const C fv = f[nd.perm[b0 + lane]];
                lfx = fv.x;
                lfy = fv.y;
                lu0 = nd.u[0][b0 + lane] & ((1 << g.lgB[0]) - 1);
                lu1 = nd.u[1][b0 + lane] & ((1 << g.lgB[1]) - 1);
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k)
                lwv[k] = (k < nb && lane < dW) ? psi[(int64_t)(b0 + k) * dW + lane] : T(0);
        };
        if (lo < hi)
            load_batch(lo, fx, fy, u0, u1, wv);
        for (int b0 = lo; b0 < hi; b0 += kBatch) {
            const int nb = min(kBatch, hi - b0);
            T nfx = 0, nfy = 0, nwv[kBatch];
            int nu0 = 0, nu1 = 0;
            if (b0 + kBatch < hi)
                load_batch(b0 + kBatch, nfx, nfy, nu0, nu1, nwv);
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                if (k >= nb)
                    break;
                const T fxk = bcast(fx, k), fyk = bcast(fy, k);
                const int ul0 = bcast(u0, k), ul1 = bcast(u1, k);
                const T w1 = bperm(w1idx, wv[k]);
                const T ax = fxk * w1, ay = fyk * w1;
                const int base = ul0 * P1 + ul1;  // the node's first stencil cell in the tile
                auto update = [&](const int(&Aq)[NP2], const int(&okq)[NP2], const int(&wq)[NP2]) {
                    T w0[NP2];
                    C v[NP2];
                    int idx[NP2];
#pragma unroll
                    for (int q = 0; q < NP2; ++q) {
                        idx[q] = __mul24(okq[q], base) + Aq[q];
                        w0[q] = bperm(wq[q], wv[k]);
                        v[q] = tiles[idx[q]];
                    }
#pragma unroll
                    for (int q = 0; q < NP2; ++q) {
                        v[q].x += ax * w0[q];
                        v[q].y += ay * w0[q];
                        tiles[idx[q]] = v[q];
                    }
                };
                // this wave's rows of the stencil start at parity (par - ul0) mod 2
                if (((par - ul0) & 1) == 0)
                    update(A[0], okv[0], widx[0]);
                else
                    update(A[1], okv[1], widx[1]);
            }
            fx = nfx;
            fy = nfy;
            u0 = nu0;
            u1 = nu1;
#pragma unroll
            for (int k = 0; k < kBatch; ++k)
                wv[k] = nwv[k];
        }
        __syncthreads();
        C *slot = scratch + (int64_t)c * g.Ptot;
        for (int i = threadIdx.x; i < g.Ptot; i += kBlock) {
            const C a0 = tiles[i], a1 = tiles[g.Ptot + i];
            slot[i] = C{a0.x + a1.x, a0.y + a1.y};
        }
        __syncthreads();
    } else {
        // 3-D: one tile shared by the workgroup; wave w owns the tile planes whose index is
        // w mod 4, so every wave goes through all nodes of the item and updates only its own
        // planes of each stencil -- no two waves touch the same cell and no barrier is needed
        // between nodes.  Node data is loaded in batches of kBatch, one batch ahead.
        for (int i = threadIdx.x; i < g.Ptot; i += kBlock)
            tiles[i] = C{T(0), T(0)};
        __syncthreads();
        constexpr int NW = (3 * WM + 63) / 64;  // registers of window factors per node and lane
        constexpr int KB = (NW > 1 || sizeof(T) == 8) ? kBatch / 2 : kBatch;  // nodes per batch (registers)
        constexpr int NPL = (WM + kWaves - 1) / kWaves;                         // planes per wave and node
        constexpr int G = NPL < 16 / NPASS ? NPL : (16 / NPASS > 0 ? 16 / NPASS : 1);  // planes per group
        const int P1 = g.P[1], P2 = g.P[2];
        const int hi = first + len;
        T fx = 0, fy = 0, wv[NW][KB];
        int u0 = 0, u1 = 0, u2 = 0;
        auto load_batch = [&](int b0, T &lfx, T &lfy, int &lu0, int &lu1, int &lu2, T (*lwv)[KB]) {
            const int nb = min(KB, hi - b0);
            lfx = lfy = T(0);
            lu0 = lu1 = lu2 = 0;
            if (lane < nb) {
                const C fv = f[nd.perm[b0 + lane]];
                lfx = fv.x;
                lfy = fv.y;
                lu0 = nd.u[0][b0 + lane] & ((1 << g.lgB[0]) - 1);
                lu1 = nd.u[1][b0 + lane] & ((1 << g.lgB[1]) - 1);
                lu2 = nd.u[2][b0 + lane] & ((1 << g.lgB[2]) - 1);
            }
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int k = 0; k < KB; ++k)
                    lwv[q][k] = (k < nb && lane + 64 * q < dW) ? psi[(int64_t)(b0 + k) * dW + lane + 64 * q] : T(0);
        };
        // the same slot for every lane (uniform j)
        auto factor_u = [&](int k, int j) -> T { return bcast(wv[0][k], j); };  // j < W <= 26
        // Per-lane constants of the item (lanes over (s1, s2) = (q R + r, sc)): the tile
        // index relative to a plane's first stencil cell and the shuffle addresses of the
        // lane's factors.  Lanes outside the stencil get a private dummy slot after the
        // tile, so the per-node code runs without predication: index = ok * base + A.
        int A3[NPASS], ok3[NPASS], w1idx[NPASS];
        const int dummy = g.Ptot + wave * 64 + lane;
#pragma unroll
        for (int q = 0; q < NPASS; ++q) {
            const int s1 = q * R + r;
            const bool ok = lane_ok && s1 < W;
            A3[q] = ok ? s1 * P2 + sc : dummy;
            ok3[q] = ok ? 1 : 0;
            w1idx[q] = (W + (ok ? s1 : 0)) * 4;  // < 2W <= 52: always in the first register
        }
        const int j2 = 2 * W + (sc < W ? sc : 0);
        const int w2idx = (j2 & 63) * 4;
        const bool w2hi = j2 >= 64;
        if (first < hi)
            load_batch(first, fx, fy, u0, u1, u2, wv);
        for (int b0 = first; b0 < hi; b0 += KB) {
            const int nb = min(KB, hi - b0);
            T nfx = 0, nfy = 0, nwv[NW][KB];
            int nu0 = 0, nu1 = 0, nu2 = 0;
            if (b0 + KB < hi)
                load_batch(b0 + KB, nfx, nfy, nu0, nu1, nu2, nwv);
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                if (k >= nb)
                    break;
                const T fxk = bcast(fx, k), fyk = bcast(fy, k);
                const int ul0 = bcast(u0, k), ul1 = bcast(u1, k), ul2 = bcast(u2, k);
                T w2 = bperm(w2idx, wv[0][k]);
                if constexpr (NW > 1) {
                    const T w2b = bperm(w2idx, wv[NW - 1][k]);
                    w2 = w2hi ? w2b : w2;
                }
                const T ax = fxk * w2, ay = fyk * w2;
                T w1[NPASS];
#pragma unroll
                for (int q = 0; q < NPASS; ++q)
                    w1[q] = bperm(w1idx[q], wv[0][k]);
                const int rbase = ul1 * P2 + ul2;
                // this wave's planes of the stencil: s0 = s0a, s0a + 4, ... (at most NPL), in
                // groups of G planes whose reads are all issued before their updates
                const int s0a = (wave - ul0) & (kWaves - 1);
#pragma unroll
                for (int t0 = 0; t0 < NPL; t0 += G) {
                    T w0[G];
                    C v[G][NPASS];
                    int idx[G][NPASS];
#pragma unroll
                    for (int t = 0; t < G; ++t) {
                        const int s0 = s0a + kWaves * (t0 + t);
                        w0[t] = factor_u(k, s0 < W ? s0 : 0);
                        if (t0 + t < NPL && s0 < W) {  // uniform
                            const int pbase = (ul0 + s0) * P1 * P2 + rbase;
#pragma unroll
                            for (int q = 0; q < NPASS; ++q) {
                                idx[t][q] = __mul24(ok3[q], pbase) + A3[q];
                                v[t][q] = tiles[idx[t][q]];
                            }
                        }
                    }
#pragma unroll
                    for (int t = 0; t < G; ++t) {
                        const int s0 = s0a + kWaves * (t0 + t);
                        if (t0 + t < NPL && s0 < W) {  // uniform
                            const T bx = ax * w0[t], by = ay * w0[t];
#pragma unroll
                            for (int q = 0; q < NPASS; ++q) {
                                v[t][q].x += bx * w1[q];
                                v[t][q].y += by * w1[q];
                                tiles[idx[t][q]] = v[t][q];
                            }
                        }
                    }
                }
            }
            fx = nfx;
            fy = nfy;
            u0 = nu0;
            u1 = nu1;
            u2 = nu2;
#pragma unroll
            for (int q = 0; q < NW; ++q)
#pragma unroll
                for (int k = 0; k < KB; ++k)
                    wv[q][k] = nwv[q][k];
        }
        __syncthreads();
        C *slot = scratch + (int64_t)c * g.Ptot;
        for (int i = threadIdx.x; i < g.Ptot; i += kBlock)
            slot[i] = tiles[i];
        __syncthreads();
    }
}

template <typename T, int D, int WM>
__global__ __launch_bounds__(kBlock) void k_spread_tiles(Geom g, Nodes nd, const Cplx<T> *__restrict__ f,
                                                         Cplx<T> *__restrict__ scratch)
{
    using C = Cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tiles = reinterpret_cast<C *>(smem_raw);
    const int nchunks = nd.counters[0];
    // work items are mapped over the first min(grid, items) workgroups, XCD by XCD
    const int nwg = min((int)gridDim.x, nchunks);
    if ((int)blockIdx.x >= nwg)
        return;
    for (int c = xcd_local_id(blockIdx.x, nwg); c < nchunks; c += nwg)
        spread_item<T, D, WM>(g, nd, f, scratch, c, tiles);
}

// ------------------------------------------------------------------ 2-D spreading in registers
//
// d = 2 with bins of B0 x 32 cells (B0 = 32 for complex64, 16 for complex128) and 2m+2 = WM,
// so that the padded tile is P0 = B0 + WM - 1 rows by P1 = 32 + WM - 1 <= 64 columns.  Lane
// c of a wave owns tile column c and keeps all P0 cells of that column in registers.  A
// node at tile-local cell (r0, c0) adds psi_0[s0] * (psi_1[c - c0] f_j) to rows r0 + s0 of
// column c.  The node precomputation lists every work item's nodes by tile row (spos).  A
// wave walks its part of the list in small batches with one unrolled update sequence per
// tile row, so every register index is a constant: per node it reads the row factors (the
// same address in every lane), its column factor and f_j from LDS and does 2 WM
// multiply-adds per lane.  The factor records and values of the next batch are copied
// from global memory straight into LDS (global_load_lds: no registers, asynchronous) while
// the current batch is walked.  The four waves of a workgroup take a quarter of the list
// each; their columns are summed in a fixed order through two LDS tiles when the item is
// done, so the result is deterministic.

// Inputs of the in-register spreading of one plan.
template <typename T> struct ColsIn {
    const int32_t *spos;  // pairs (packed entry, caller index) in tile-row order
    const T *psi;
    const Cplx<T> *f;
};

// Geometry of the staged batches of one wave.
template <typename T, int WM> struct ColsStage {
    static constexpr int KB = sizeof(T) == 4 ? 16 : 8;          // list entries per batch
    static constexpr int REC = 2 * WM * (int)sizeof(T) / 16;    // 16-byte pieces of a record
    static constexpr int NI = (KB * REC + 63) / 64;             // record copies per batch
    static constexpr int VAL = sizeof(T) == 4 ? 512 : 1024;     // bytes of the staged values
    static constexpr int NV = sizeof(T) == 4 ? 2 : 1;           // value copies per batch
    static constexpr int BUF = NI * 1024 + VAL;                 // bytes of one batch buffer
    static constexpr int COPIES = NI + NV;                      // memory instructions per batch
};

using lds_void = __attribute__((address_space(3))) void;

// Copy 4 or 16 bytes per lane from src into LDS at dst + 4 lane or dst + 16 lane.
__device__ __forceinline__ void to_lds4(const void *src, unsigned char *dst)
{
    __builtin_amdgcn_global_load_lds(src, (lds_void *)dst, 4, 0, 0);
}
__device__ __forceinline__ void to_lds16(const void *src, unsigned char *dst)
{
    __builtin_amdgcn_global_load_lds(src, (lds_void *)dst, 16, 0, 0);
}

// Wait until at most N memory instructions of this wave are outstanding (s_waitcnt vmcnt(N),
// the other counters at their maximum).  Also keeps the compiler from moving LDS reads
// above it, since it does not see the LDS writes of global_load_lds.
template <int N> __device__ __forceinline__ void wait_vm()
{
    static_assert(N < 16, "vmcnt field");
    __builtin_amdgcn_s_waitcnt(N | (0x7 << 4) | (0xf << 8));
}

// Start copying batch entries bb .. bb + nbb - 1 (lanes of ex / ey hold the list entries of
// the wave's current 64) into buf: records of 2 WM factors at buf + k * REC * 16, values
// f_j after the records.  Every lane takes part in every copy (indices past the batch are
// clamped to its last entry), so a batch is always exactly COPIES memory instructions.
template <typename T, int WM>
__device__ __forceinline__ void cols_issue(int bb, int nbb, int ex, int ey, int first, int lane, const ColsIn<T> &in,
                                           unsigned char *buf)
{
    using S = ColsStage<T, WM>;
    // records of the item start at a wave-uniform base; a lane adds a 32-bit offset
    const unsigned char *ibase = reinterpret_cast<const unsigned char *>(in.psi + (int64_t)first * (2 * WM));
#pragma unroll
    for (int j = 0; j < S::NI; ++j) {
        const int p = j * 64 + lane;
        const int e = min(p / S::REC, nbb - 1);
        const int q = p - (p / S::REC) * S::REC;
        const int off = __builtin_amdgcn_ds_bpermute((bb + e) * 4, ex) >> 10;
        to_lds16(ibase + (unsigned)(off * (S::REC * 16) + q * 16), buf + j * 1024);
    }
    const int e = min(lane, nbb - 1);
    const int cidx = __builtin_amdgcn_ds_bpermute((bb + e) * 4, ey);
    const T *fv = reinterpret_cast<const T *>(in.f + cidx);
    if constexpr (sizeof(T) == 4) {
        to_lds4(fv, buf + S::NI * 1024);
        to_lds4(fv + 1, buf + S::NI * 1024 + 256);
    } else {
        to_lds16(fv, buf + S::NI * 1024);
    }
}

// Add the staged batch entries i, i + 1, ... whose tile row is R (they follow each other):
// acc[R + s] += psi_0[s] * g for the WM rows of each.
template <int R, typename T, int P0, int WM>
__device__ __forceinline__ void cols_row(int &i, int nb, int bb, int ex, const unsigned char *buf, int lane,
                                         T (&ax)[P0], T (&ay)[P0])
{
    using S = ColsStage<T, WM>;
    for (; i < nb; ++i) {
        const int e = __builtin_amdgcn_readlane(ex, bb + i);
        if (((e >> 5) & 31) != R)
            break;
        const T *rec = reinterpret_cast<const T *>(buf + i * S::REC * 16);
        T w[WM];
#pragma unroll
        for (int s = 0; s < WM; ++s)
            w[s] = rec[s];
        const int s1 = lane - (e & 31);
        const int sc = min(max(s1, 0), WM - 1);
        const T v = rec[WM + sc];
        const T w1 = s1 == sc ? v : T(0);
        T fx, fy;
        if constexpr (sizeof(T) == 4) {
            fx = reinterpret_cast<const T *>(buf + S::NI * 1024)[i];
            fy = reinterpret_cast<const T *>(buf + S::NI * 1024 + 256)[i];
        } else {
            const Cplx<T> fv = reinterpret_cast<const Cplx<T> *>(buf + S::NI * 1024)[i];
            fx = fv.x;
            fy = fv.y;
        }
        const T gx = w1 * fx;
        const T gy = w1 * fy;
#pragma unroll
        for (int s = 0; s < WM; ++s) {
            ax[R + s] += w[s] * gx;
            ay[R + s] += w[s] * gy;
        }
    }
}

template <typename T, int P0, int WM, int... Rs>
__device__ __forceinline__ void cols_walk(std::integer_sequence<int, Rs...>, int nb, int bb, int ex,
                                          const unsigned char *buf, int lane, T (&ax)[P0], T (&ay)[P0])
{
    int i = 0;
    (cols_row<Rs, T, P0, WM>(i, nb, bb, ex, buf, lane, ax, ay), ...);
}

// Waves per SIMD the register allocation aims at: 4 for complex64 up to m = 8 (at most 128
// registers; the few values that no longer fit are kept outside the walk), else whatever
// the accumulators leave.
template <typename T, int WM> constexpr int cols_waves() { return sizeof(T) == 4 && WM <= 18 ? 4 : 1; }

// One work item (nodes first .. first + len - 1 of one bin) of a plan: accumulate in
// registers, then write the summed tile to the item's slot.  Called by all threads of the
// workgroup (it has barriers).
template <typename T, int B0, int WM>
__device__ __forceinline__ void cols_item(int first, int len, const ColsIn<T> &in, Cplx<T> *__restrict__ slot,
                                          unsigned char *smem)
{
    using C = Cplx<T>;
    using S = ColsStage<T, WM>;
    constexpr int P0 = B0 + WM - 1;
    constexpr int P1 = 32 + WM - 1;
    constexpr int Ptot = P0 * P1;
    C *lds = reinterpret_cast<C *>(smem);
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned char *bufs = smem + wave * 2 * S::BUF;
    const int lo = (len * wave) >> 2;
    const int hi = (len * (wave + 1)) >> 2;
    T ax[P0], ay[P0];
#pragma unroll
    for (int r = 0; r < P0; ++r) {
        ax[r] = 0;
        ay[r] = 0;
    }
    for (int sb = lo; sb < hi; sb += 64) {
        // lane k holds list entry sb + k (entries past the wave's part: offset 0, caller 0)
        const int nsb = min(64, hi - sb);
        int ex = 0, ey = 0;
        if (lane < nsb) {
            const int2 ent = reinterpret_cast<const int2 *>(in.spos)[first + sb + lane];
            ex = ent.x;
            ey = ent.y;
        }
        const int nbat = (nsb + S::KB - 1) / S::KB;
        cols_issue<T, WM>(0, min(S::KB, nsb), ex, ey, first, lane, in, bufs);
        for (int j = 0; j < nbat; ++j) {
            const int bb = j * S::KB;
            if (j + 1 < nbat) {
                cols_issue<T, WM>(bb + S::KB, min(S::KB, nsb - bb - S::KB), ex, ey, first, lane, in,
                                  bufs + ((j + 1) & 1) * S::BUF);
                wait_vm<S::COPIES>();
            } else {
                wait_vm<0>();
            }
            // the entries of a batch are sorted by row
            cols_walk<T, P0, WM>(std::make_integer_sequence<int, B0>{}, min(S::KB, nsb - bb), bb, ex,
                                 bufs + (j & 1) * S::BUF, lane, ax, ay);
        }
    }
    // Sum the four waves' columns: waves 0 and 1 store theirs in tiles A and B, waves 2
    // and 3 add theirs to A and B, and the workgroup writes A + B to the item's slot:
    // (w0 + w2) + (w1 + w3), a fixed order.  The tiles reuse the staging memory.
    __syncthreads();
    C *half = lds + (wave & 1) * Ptot;
    if (wave < 2 && lane < P1) {
#pragma unroll
        for (int r = 0; r < P0; ++r)
            half[r * P1 + lane] = C{ax[r], ay[r]};
    }
    __syncthreads();
    if (wave >= 2 && lane < P1) {
#pragma unroll
        for (int r = 0; r < P0; ++r) {
            const C o = half[r * P1 + lane];
            half[r * P1 + lane] = C{o.x + ax[r], o.y + ay[r]};
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < Ptot; i += kBlock) {
        const C a = lds[i];
        const C bv = lds[Ptot + i];
        slot[i] = C{a.x + bv.x, a.y + bv.y};
    }
    __syncthreads();
}

template <typename T, int B0, int WM>
__global__ __launch_bounds__(kBlock, (cols_waves<T, WM>())) void k_spread_cols(
    const int32_t *__restrict__ counters, const int32_t *__restrict__ chunk_first,
    const int32_t *__restrict__ chunk_len, ColsIn<T> in, Cplx<T> *__restrict__ scratch)
{
    constexpr int Ptot = (B0 + WM - 1) * (32 + WM - 1);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nchunks = counters[0];
    const int nwg = min((int)gridDim.x, nchunks);
    if ((int)blockIdx.x >= nwg)
        return;
    for (int c = xcd_local_id(blockIdx.x, nwg); c < nchunks; c += nwg)
        cols_item<T, B0, WM>(chunk_first[c], chunk_len[c], in, scratch + (int64_t)c * Ptot, smem_raw);
}

// All plans of a batch whose 2-D spreading runs in registers, items handed out by the
// dynamic queue.
template <typename T, int B0, int WM>
__global__ __launch_bounds__(kBlock, (cols_waves<T, WM>())) void k_spread_cols_batch(
    const PlanDev *__restrict__ plans, int count, BatchPtrs ptrs, int *queue)
{
    using C = Cplx<T>;
    constexpr int Ptot = (B0 + WM - 1) * (32 + WM - 1);
    extern __shared__ __align__(16) unsigned char smem_raw[];
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
        const int c = it - s_prefix[p];
        const ColsIn<T> in{pd.nd.spos, static_cast<const T *>(pd.nd.psi), static_cast<const C *>(ptrs.in[p])};
        cols_item<T, B0, WM>(pd.nd.chunk_first[c], pd.nd.chunk_len[c], in,
                             static_cast<C *>(pd.scratch) + (int64_t)c * Ptot, smem_raw);
    }
    queue_done(queue);
}

// All plans of a batch in one launch, items handed out by the dynamic queue.
template <typename T, int D, int WM>
__global__ __launch_bounds__(kBlock) void k_spread_batch(const PlanDev *__restrict__ plans, int count, BatchPtrs ptrs,
                                                         int *queue)
{
    using C = Cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C *tiles = reinterpret_cast<C *>(smem_raw);
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
        spread_item<T, D, WM>(pd.g, pd.nd, static_cast<const C *>(ptrs.in[p]), static_cast<C *>(pd.scratch),
                              it - s_prefix[p], tiles);
    }
    queue_done(queue);
}

// Fold: grid cell l receives, from every work item of every bin b whose padded tile covers
// it, the tile entry at offset o = l + k n + m - b B (k = -1, 0, 1 accounts for the
// periodic wrap; 0 <= o < P).  Bins are visited in increasing order per dimension and
// work items in order, so every cell is a sum in a fixed order.
struct Cover {
    int lo, hi;  // bins lo..hi (inclusive) cover unwrapped index lu
    int lu;
};

__device__ __forceinline__ Cover cover_range(int l, int k, int n, int lgB, int nb, int m, int P)
{
    Cover cv;
    cv.lu = l + k * n + m;
    cv.hi = cv.lu >= 0 ? (cv.lu >> lgB) : -1;
    const int lo_num = cv.lu - P + 1;
    cv.lo = lo_num <= 0 ? 0 : ((lo_num + (1 << lgB) - 1) >> lgB);
    if (cv.hi > nb - 1)
        cv.hi = nb - 1;
    return cv;
}

// The (at most two) covering (bin, tile offset) pairs of index l in one dimension, in the
// order of cover_range over k = -1, 0, 1.
struct Pairs2 {
    int b0, o0, b1, o1, n;
};
__device__ __forceinline__ Pairs2 cover_pairs2(int l, int n, int lgB, int nb, int m, int P)
{
    Pairs2 r{0, 0, 0, 0, 0};
#pragma unroll
    for (int k = -1; k <= 1; ++k) {
        const Cover cv = cover_range(l, k, n, lgB, nb, m, P);
        for (int b = cv.lo; b <= cv.hi; ++b) {
            const int o = cv.lu - (b << lgB);
            if (r.n == 0) {
                r.b0 = b;
                r.o0 = o;
            } else {
                r.b1 = b;
                r.o1 = o;
            }
            ++r.n;
        }
    }
    return r;
}

// fold_cell for plans whose tiles cover every grid index at most twice per dimension: the
// 2^D covering bins are found first, then their work-item ranges and the first work item's
// entries are loaded together (every load issued before the first use), and the sum is
// taken in the same order as in fold_cell, so the result is the same.
template <typename T, int D>
__device__ __forceinline__ void fold_cell2(const Geom &g, const Nodes &nd, const Cplx<T> *__restrict__ scratch,
                                           Cplx<T> *__restrict__ grid, int64_t q, const int (&l)[kMaxDim])
{
    using C = Cplx<T>;
    constexpr int NC = 1 << D;
    Pairs2 pr[D];
#pragma unroll
    for (int t = 0; t < D; ++t)
        pr[t] = cover_pairs2(l[t], g.n[t], g.lgB[t], g.nb[t], g.m, g.P[t]);
    int bin[NC], off[NC];
    bool ok[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        int b = 0, o = 0;
        bool v = true;
#pragma unroll
        for (int t = 0; t < D; ++t) {
            const int sel = (k >> (D - 1 - t)) & 1;  // dimension 0 outermost
            v = v && sel < pr[t].n;
            b = b * g.nb[t] + (sel ? pr[t].b1 : pr[t].b0);
            o = o * g.P[t] + (sel ? pr[t].o1 : pr[t].o0);
        }
        ok[k] = v;
        bin[k] = v ? b : 0;
        off[k] = v ? o : 0;
    }
    int c0[NC], c1[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        c0[k] = nd.bin_chunk[bin[k]];
        c1[k] = nd.bin_chunk[bin[k] + 1];
    }
    C first[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        ok[k] = ok[k] && c0[k] < c1[k];
        first[k] = scratch[(int64_t)(ok[k] ? c0[k] : 0) * g.Ptot + off[k]];
    }
    T ax = 0, ay = 0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
        if (!ok[k])
            continue;
        ax += first[k].x;
        ay += first[k].y;
        for (int c = c0[k] + 1; c < c1[k]; ++c) {
            const C v = scratch[(int64_t)c * g.Ptot + off[k]];
            ax += v.x;
            ay += v.y;
        }
    }
    grid[q] = C{ax, ay};
}

// Grid cell q of a plan: sum of the tile entries covering it, in a fixed order.
template <typename T, int D>
__device__ __forceinline__ void fold_cell(const Geom &g, const Nodes &nd, const Cplx<T> *__restrict__ scratch,
                                          Cplx<T> *__restrict__ grid, int64_t q)
{
    using C = Cplx<T>;

    int l[kMaxDim] = {0, 0, 0};
    {
        int64_t rq = q;
        if (g.p2) {
#pragma unroll
            for (int t = D - 1; t >= 0; --t) {
                l[t] = (int)(rq & (g.n[t] - 1));
                rq >>= (31 - __clz(g.n[t]));
            }
        } else {
#pragma unroll
            for (int t = D - 1; t >= 0; --t) {
                const int64_t qt = rq / g.n[t];
                l[t] = (int)(rq - qt * g.n[t]);
                rq = qt;
            }
        }
    }
    if (g.fold2) {
        fold_cell2<T, D>(g, nd, scratch, grid, q, l);
        return;
    }
    T ax = 0, ay = 0;
    auto add_bin = [&](int bin, int off) {
        const int c1 = nd.bin_chunk[bin + 1];
        for (int c = nd.bin_chunk[bin]; c < c1; ++c) {
            const C v = scratch[(int64_t)c * g.Ptot + off];
            ax += v.x;
            ay += v.y;
        }
    };
    for (int k0 = -1; k0 <= 1; ++k0) {
        const Cover c0 = cover_range(l[0], k0, g.n[0], g.lgB[0], g.nb[0], g.m, g.P[0]);
        for (int b0 = c0.lo; b0 <= c0.hi; ++b0) {
            const int o0 = c0.lu - (b0 << g.lgB[0]);
            if constexpr (D == 1) {
                add_bin(b0, o0);
            } else {
                for (int k1 = -1; k1 <= 1; ++k1) {
                    const Cover c1 = cover_range(l[1], k1, g.n[1], g.lgB[1], g.nb[1], g.m, g.P[1]);
                    for (int b1 = c1.lo; b1 <= c1.hi; ++b1) {
                        const int o1 = c1.lu - (b1 << g.lgB[1]);
                        if constexpr (D == 2) {
                            add_bin(b0 * g.nb[1] + b1, o0 * g.P[1] + o1);
                        } else {
                            for (int k2 = -1; k2 <= 1; ++k2) {
                                const Cover c2 = cover_range(l[2], k2, g.n[2], g.lgB[2], g.nb[2], g.m, g.P[2]);
                                for (int b2 = c2.lo; b2 <= c2.hi; ++b2) {
                                    const int o2 = c2.lu - (b2 << g.lgB[2]);
                                    add_bin((b0 * g.nb[1] + b1) * g.nb[2] + b2, (o0 * g.P[1] + o1) * g.P[2] + o2);
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    grid[q] = C{ax, ay};
}

template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_fold(Geom g, Nodes nd, const Cplx<T> *__restrict__ scratch,
                                                 Cplx<T> *__restrict__ grid)
{
    int64_t total = 1;
#pragma unroll
    for (int t = 0; t < D; ++t)
        total *= g.n[t];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < total)
        fold_cell<T, D>(g, nd, scratch, grid, q);
}

// Batched fold: items are blocks of kBlock cells of every plan's adjoint grid.
template <typename T, int D>
__global__ __launch_bounds__(kBlock) void k_fold_batch(const PlanDev *__restrict__ plans, int count)
{
    using C = Cplx<T>;
    __shared__ int s_cnt[kMaxBatch];
    __shared__ int s_prefix[kMaxBatch + 1];
    if ((int)threadIdx.x < count)
        s_cnt[threadIdx.x] = (int)((plans[threadIdx.x].ngrid + kBlock - 1) / kBlock);
    __syncthreads();
    batch_prefix(s_prefix, count, s_cnt);
    const int total = s_prefix[count];
    for (int it = xcd_local_id(blockIdx.x, gridDim.x); it < total; it += gridDim.x) {
        const int p = batch_find(s_prefix, count, it);
        const PlanDev &pd = plans[p];
        const int64_t q = (int64_t)(it - s_prefix[p]) * kBlock + threadIdx.x;
        if (q < pd.ngrid)
            fold_cell<T, D>(pd.g, pd.nd, static_cast<const C *>(pd.scratch), static_cast<C *>(pd.grid_adj), q);
    }
}

template <typename T, int B0>
hipError_t spread_cols_typed(const Geom &g, const Nodes &nd, const void *f, void *scratch, int blocks, size_t lds,
                             hipStream_t s)
{
    using C = Cplx<T>;
    ColsIn<T> in{nd.spos, static_cast<const T *>(nd.psi), static_cast<const C *>(f)};
#define CALL(W_)                                                                                       \
    {                                                                                                  \
        auto kf = k_spread_cols<T, B0, W_>;                                                            \
        (void)hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
        hipLaunchKernelGGL(kf, dim3(blocks), dim3(kBlock), lds, s, nd.counters, nd.chunk_first,           \
                           nd.chunk_len, in, static_cast<C *>(scratch));                               \
    }
    NFFT_WM_SWITCH(g.WM, CALL)
#undef CALL
    return hipGetLastError();
}

template <typename T, int D>
hipError_t spread_typed(const Geom &g, const Nodes &nd, const void *f, void *scratch, int blocks, size_t lds,
                        hipStream_t s)
{
    using C = Cplx<T>;
    if constexpr (D == 2) {
        if (spread_in_registers(g, sizeof(T) == 8))
            return spread_cols_typed<T, sizeof(T) == 8 ? 16 : 32>(g, nd, f, scratch, blocks, lds, s);
    }
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

namespace {
template <typename T, int D>
hipError_t spread_batch_typed(const PlanDev *plans, int count, const BatchPtrs &ptrs, int *queue, int WMv,
                              int blocks, size_t lds, hipStream_t s)
{
#define CALL(W_)                                                                                       \
    {                                                                                                  \
        auto kf = k_spread_batch<T, D, W_>;                                                            \
        (void)hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL(kf, dim3(blocks), dim3(kBlock), lds, s, plans, count, ptrs, queue);         \
    }
    NFFT_WM_SWITCH(WMv, CALL)
#undef CALL
    return hipGetLastError();
}
template <typename T, int B0>
hipError_t spread_cols_batch_typed(const PlanDev *plans, int count, const BatchPtrs &ptrs, int *queue, int WMv,
                                   int blocks, size_t lds, hipStream_t s)
{
#define CALL(W_)                                                                                       \
    {                                                                                                  \
        auto kf = k_spread_cols_batch<T, B0, W_>;                                                      \
        (void)hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL(kf, dim3(blocks), dim3(kBlock), lds, s, plans, count, ptrs, queue);         \
    }
    NFFT_WM_SWITCH(WMv, CALL)
#undef CALL
    return hipGetLastError();
}
template <typename T, int D> hipError_t fold_batch_typed(const PlanDev *plans, int count, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_fold_batch<T, D>), dim3(blocks), dim3(kBlock), 0, s, plans, count);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_spread_batch(const PlanDev *plans, int count, const BatchPtrs &ptrs, int *queue, int d,
                               bool dbl, int WMv, int blocks, size_t lds, hipStream_t s)
{
    switch (d * 2 + (dbl ? 1 : 0)) {
    case 2: return spread_batch_typed<float, 1>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    case 3: return spread_batch_typed<double, 1>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    case 4: return spread_batch_typed<float, 2>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    case 5: return spread_batch_typed<double, 2>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    case 6: return spread_batch_typed<float, 3>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    case 7: return spread_batch_typed<double, 3>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spread_cols_batch(const PlanDev *plans, int count, const BatchPtrs &ptrs, int *queue, bool dbl,
                                    int WMv, int blocks, size_t lds, hipStream_t s)
{
    if (dbl)
        return spread_cols_batch_typed<double, 16>(plans, count, ptrs, queue, WMv, blocks, lds, s);
    return spread_cols_batch_typed<float, 32>(plans, count, ptrs, queue, WMv, blocks, lds, s);
}

hipError_t launch_fold_batch(const PlanDev *plans, int count, int d, bool dbl, int blocks, hipStream_t s)
{
    switch (d * 2 + (dbl ? 1 : 0)) {
    case 2: return fold_batch_typed<float, 1>(plans, count, blocks, s);
    case 3: return fold_batch_typed<double, 1>(plans, count, blocks, s);
    case 4: return fold_batch_typed<float, 2>(plans, count, blocks, s);
    case 5: return fold_batch_typed<double, 2>(plans, count, blocks, s);
    case 6: return fold_batch_typed<float, 3>(plans, count, blocks, s);
    case 7: return fold_batch_typed<double, 3>(plans, count, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nfft
