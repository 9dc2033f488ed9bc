// Device-side building blocks of the NFFT library for gfx950: complex helpers, the
// Kaiser-Bessel window in its normalised form, and the parameter blocks the host
// passes to the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nfft {

constexpr int kMaxDim = 3;
constexpr int kBlock = 256;  // threads per workgroup of the window and node kernels

// ------------------------------------------------------------------ complex helpers

template <typename T> struct CplxOf;
template <> struct CplxOf<float> { using type = float2; };
template <> struct CplxOf<double> { using type = double2; };
template <typename T> using Cplx = typename CplxOf<T>::type;
template <typename T> using Pair = Cplx<T>;  // two reals loaded together

template <typename C> __host__ __device__ __forceinline__ C cmul(C a, C b)
{
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename C> __host__ __device__ __forceinline__ C cmulc(C a, C b)
{
    return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename C> __host__ __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __host__ __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C, typename T> __host__ __device__ __forceinline__ C cscale(C a, T s)
{
    return C{a.x * s, a.y * s};
}

// ------------------------------------------------------------------ launch mapping

// The dispatcher hands consecutive workgroups to the 8 XCDs in turn, and each XCD has
// its own L2.  This bijection of [0, G) gives XCD x (blocks b with b mod 8 = x) one
// contiguous range of logical work items, so neighbouring items -- which share cache
// lines of the grid -- run behind the same L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_local_id(int b, int G)
{
    const int x = b % kXcds;
    const int q = G / kXcds, r = G % kXcds;
    const int start = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return start + b / kXcds;
}

// ------------------------------------------------------------------ window

// Stencil width bucket: kernels are compiled for WM = 6, 10, ..., 26 points per
// dimension; a plan with 2m+2 < WM pads its window with zeros up to WM.
__host__ __device__ constexpr int wm_bucket(int m)
{
    return m <= 2 ? 6 : m <= 4 ? 10 : m <= 6 ? 14 : m <= 8 ? 18 : m <= 10 ? 22 : 26;
}

// Normalised Kaiser-Bessel window, interior branch (|z| <= m):
//     e^{-bm} * sinh(b s) / (pi s),   s = sqrt(m^2 - z^2),
// evaluated as (e^{b(s-m)} - e^{-b(s+m)}) / (2 pi s) with s - m = -z^2/(s+m), so the
// exponent stays near zero where the window is large and FP32 does not amplify the
// rounding of z.  Near s = 0 the series e^{-bm} (b/pi)(1 + (bs)^2/6 + (bs)^4/120 + ...).
template <typename T> __device__ __forceinline__ T kb_interior(T z, T m, T b, T emb)
{
    const T inv_pi = T(0.318309886183790671537767526745028724);
    T z2 = z * z;
    T a = m * m - z2;
    a = a > T(0) ? a : T(0);
    T s = sqrt(a);
    T bs = b * s;
    if (bs < T(1e-2)) {
        T q = bs * bs;
        return emb * b * inv_pi * (T(1) + q * (T(1) / T(6) + q * (T(1) / T(120) + q * (T(1) / T(5040)))));
    }
    T e1 = exp(-b * z2 / (s + m));
    T e2 = exp(-b * (s + m));
    return (e1 - e2) * (T(0.5) * inv_pi) / s;
}

// Normalised window at the two end points of the stencil (|z| >= m), the analytic
// continuation e^{-bm} sin(b t)/(pi t), t = sqrt(z^2 - m^2).
template <typename T> __device__ __forceinline__ T kb_edge(T z, T m, T b, T emb)
{
    const T inv_pi = T(0.318309886183790671537767526745028724);
    T a = z * z - m * m;
    a = a > T(0) ? a : T(0);
    T t = sqrt(a);
    T bt = b * t;
    if (bt < T(1e-2)) {
        T q = bt * bt;
        return emb * b * inv_pi * (T(1) - q * (T(1) / T(6) - q * (T(1) / T(120))));
    }
    return emb * sin(bt) * inv_pi / t;
}

// Window value at stencil point s (0..W-1) of a node with offset delta in [0,1):
// z = delta - (s - m).  Points s = 0 and s = W-1 are the end points, the 2m points
// between them lie strictly inside |z| < m (or on |z| = m for delta = 0).
template <typename T> __device__ __forceinline__ T kb_point(T delta, int s, int W, T m, T b, T emb)
{
    T z = delta - T(s - (int)m);
    if (s == 0 || s == W - 1)
        return kb_edge(z, m, b, emb);
    return kb_interior(z, m, b, emb);
}

// d/dz of the normalised window, interior branch:
//     phi'(z) = -(z/pi) e^{-bm} (b s cosh(bs) - sinh(bs)) / s^3,
// with e^{-bm} cosh(bs) = (e1 + e2)/2 and e^{-bm} sinh(bs) = (e1 - e2)/2; for small bs the
// series b^3 sum_k 2k/(2k+1)! (bs)^{2k-2}.
template <typename T> __device__ __forceinline__ T kb_interior_d(T z, T m, T b, T emb)
{
    const T inv_pi = T(0.318309886183790671537767526745028724);
    T z2 = z * z;
    T a = m * m - z2;
    a = a > T(0) ? a : T(0);
    T s = sqrt(a);
    T bs = b * s;
    if (bs < T(0.1)) {
        T q = bs * bs;
        T ser = T(1) / T(3) +
                q * (T(1) / T(30) + q * (T(1) / T(840) + q * (T(1) / T(45360) + q * (T(1) / T(3991680)))));
        return -z * inv_pi * emb * b * b * b * ser;
    }
    T e1 = exp(-b * z2 / (s + m));
    T e2 = exp(-b * (s + m));
    T num = T(0.5) * (bs * (e1 + e2) - (e1 - e2));
    return -z * inv_pi * num / (s * s * s);
}

// d/dz at the end points: phi'(z) = (z/pi) e^{-bm} (b t cos(bt) - sin(bt)) / t^3.
template <typename T> __device__ __forceinline__ T kb_edge_d(T z, T m, T b, T emb)
{
    const T inv_pi = T(0.318309886183790671537767526745028724);
    T a = z * z - m * m;
    a = a > T(0) ? a : T(0);
    T t = sqrt(a);
    T bt = b * t;
    if (bt < T(0.1)) {
        T q = bt * bt;
        T ser = -T(1) / T(3) +
                q * (T(1) / T(30) - q * (T(1) / T(840) - q * (T(1) / T(45360) - q * (T(1) / T(3991680)))));
        return z * inv_pi * emb * b * b * b * ser;
    }
    const T sn = sin(bt), cs = cos(bt);
    return z * inv_pi * emb * (bt * cs - sn) / (t * t * t);
}

template <typename T> __device__ __forceinline__ T kb_point_d(T delta, int s, int W, T m, T b, T emb)
{
    T z = delta - T(s - (int)m);
    if (s == 0 || s == W - 1)
        return kb_edge_d(z, m, b, emb);
    return kb_interior_d(z, m, b, emb);
}

// Gaussian window (the other window with a closed-form Fourier pair that the NFFT library
// offers; standard pair of the NFFT literature), divided by its peak (pi b)^{-1/2}:
// exp(-z^2 / b) in the grid variable z; the peak is carried by the deconvolution table.
template <typename T> __device__ __forceinline__ T gauss_point(T delta, int s, T m, T b)
{
    const T z = delta - T(s - (int)m);
    return exp(-z * z / b);
}
template <typename T> __device__ __forceinline__ T gauss_point_d(T delta, int s, T m, T b)
{
    const T z = delta - T(s - (int)m);
    return T(-2) * z / b * exp(-z * z / b);
}

// B-spline window (the library's third window; standard pair): phi(z) = M_2m(z), the centred
// cardinal B-spline of order 2m.  Stencil point s of a node with offset delta lies at
// z = delta + m - s, so phi(z) = N_2m(delta + 2m - s): entry j = 2m - s of de Boor's
// triangle at t = delta, which holds N_k(t + j), j = 0..k-1, and is built from N_1 = 1 on
// [0, 1) by N_q(x) = (x N_{q-1}(x) + (q - x) N_{q-1}(x - 1)) / (q - 1) with nonnegative
// terms only.  The loops are unrolled to the largest order (2m <= 24) so that every array
// index is a constant; orders past k are skipped (k is the same in every lane).
template <typename T> __device__ __forceinline__ T bspline_tri(T t, int k, int j)
{
    constexpr int KMAX = 24;
    T b[KMAX];
    b[0] = T(1);
#pragma unroll
    for (int i = 1; i < KMAX; ++i)
        b[i] = T(0);
#pragma unroll
    for (int q = 2; q <= KMAX; ++q) {
        if (q <= k) {
            const T inv = T(1) / T(q - 1);
#pragma unroll
            for (int i = q - 1; i >= 0; --i) {
                const T left = i > 0 ? b[i - 1] : T(0);
                b[i] = ((t + T(i)) * b[i] + (T(q) - t - T(i)) * left) * inv;
            }
        }
    }
    T v = T(0);
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
        v = i == j ? b[i] : v;
    return v;
}
template <typename T> __device__ __forceinline__ T bspline_point(T delta, int s, int m)
{
    return bspline_tri<T>(delta, 2 * m, 2 * m - s);
}
// d/dz M_2m(z) = N_{2m-1}(x) - N_{2m-1}(x - 1) at x = z + m
template <typename T> __device__ __forceinline__ T bspline_point_d(T delta, int s, int m)
{
    return bspline_tri<T>(delta, 2 * m - 1, 2 * m - s) - bspline_tri<T>(delta, 2 * m - 1, 2 * m - s - 1);
}

// Sinc window (the fourth; standard pair): phi(z) = (sin(a z) / (a z))^(2m) with
// a = pi (2 - 1/sigma) / (2m) (peak 1), truncated to the 2m+2-point stencil.
template <typename T> __device__ __forceinline__ T sinc1(T x)
{
    return fabs(x) < T(1e-4) ? T(1) - x * x / T(6) : sin(x) / x;
}
template <typename T> __device__ __forceinline__ T sinc_point(T delta, int s, int m, T a)
{
    const T sc = sinc1<T>(a * (delta - T(s - m)));
    const T r = sc * sc;
    T v = T(1);
    for (int i = 0; i < m; ++i)
        v *= r;
    return v;
}
// d/dx sin(x)/x: for |x| < 1 the power series (the closed form (x cos x - sin x) / x^2
// cancels there), term n+1 = term n * (-x^2 (n+1) / (n (2n+2)(2n+3))); beyond it the closed form
template <typename T> __device__ __forceinline__ T dsinc1(T x)
{
    if (fabs(x) >= T(1))
        return (x * cos(x) - sin(x)) / (x * x);
    T term = -x / T(3), sum = T(0);
#pragma unroll
    for (int n = 1; n < 14; ++n) {
        sum += term;
        term *= -x * x * T(n + 1) / (T(n) * T(2 * n + 2) * T(2 * n + 3));
    }
    return sum;
}
template <typename T> __device__ __forceinline__ T sinc_point_d(T delta, int s, int m, T a)
{
    const T x = a * (delta - T(s - m));
    const T sc = sinc1<T>(x);
    const T ds = dsinc1<T>(x);
    T v = T(2 * m) * ds * a;
    for (int i = 0; i < 2 * m - 1; ++i)
        v *= sc;
    return v;
}

// ------------------------------------------------------------------ parameter blocks

// Geometry of a plan's window kernels.
struct Geom {
    int d;
    int m;
    int W;             // 2m+2
    int WM;            // compiled stencil width (>= W)
    int n[kMaxDim];    // grid lengths (1 for unused dimensions); even, not necessarily powers of two
    int p2;            // 1 when every n_t is a power of two (indices wrap with a mask)
    int lin;           // 1: window factors from the lookup tables (Nodes::lin), not the closed form
    int lgB[kMaxDim];  // log2 of the bin edge per dimension
    int nb[kMaxDim];   // bins per dimension
    int P[kMaxDim];    // padded tile edge B + WM - 1
    int Ptot;          // prod P
    int nbins;
    int window;           // 0 Kaiser-Bessel, 1 Gaussian, 2 B-spline, 3 sinc
    int fold2;            // every grid index is covered by at most 2 tiles per dimension
    double b[kMaxDim];    // window shape per dimension
    double emb[kMaxDim];  // 1 / (factor the device window is divided by): e^{-b m} (Kaiser-Bessel),
                          // (pi b)^{1/2} (Gaussian)
    // Owner-computes spreading (3-D plans, own = 1): the grid is cut into output tiles of
    // oT[0] x oT[1] x oT[2] cells; the node list of a tile is the concatenation of the bins
    // okb[t] .. okb[t] + okn[t] - 1 (relative to the tile's first bin, periodic) per
    // dimension, or of all bins of a dimension when oall[t].
    int own;
    int oT[kMaxDim];
    int ont[kMaxDim];   // tiles per dimension
    int ontiles;
    int okb[kMaxDim];
    int okn[kMaxDim];
    int oall[kMaxDim];
    int ocap;           // node-list entries per work item
    // 3-D plans whose smallest padded tile exceeds the LDS: planes of the tile staged per
    // interpolation slab (0: the whole tile at once)
    int islab;
};

// Window factor of dimension t at stencil point s of a node with offset delta, and its
// derivative with respect to the grid variable, for the plan's window.  AllW = false
// compiles the Kaiser-Bessel and Gaussian windows only: the unrolled B-spline triangle and
// sinc series would otherwise set the register budget of the whole kernel, so kernels that
// evaluate windows are instantiated both ways and launched by window.
template <typename T, bool AllW = true> __device__ __forceinline__ T win_point(const Geom &g, int t, T delta, int s)
{
    if (g.window == 1)
        return gauss_point<T>(delta, s, (T)g.m, (T)g.b[t]);
    if constexpr (AllW) {
        if (g.window == 2)
            return bspline_point<T>(delta, s, g.m);
        if (g.window == 3)
            return sinc_point<T>(delta, s, g.m, (T)g.b[t]);
    }
    return kb_point<T>(delta, s, g.W, (T)g.m, (T)g.b[t], (T)g.emb[t]);
}
template <typename T, bool AllW = true> __device__ __forceinline__ T win_point_d(const Geom &g, int t, T delta, int s)
{
    if (g.window == 1)
        return gauss_point_d<T>(delta, s, (T)g.m, (T)g.b[t]);
    if constexpr (AllW) {
        if (g.window == 2)
            return bspline_point_d<T>(delta, s, g.m);
        if (g.window == 3)
            return sinc_point_d<T>(delta, s, g.m, (T)g.b[t]);
    }
    return kb_point_d<T>(delta, s, g.W, (T)g.m, (T)g.b[t], (T)g.emb[t]);
}
// Whether a plan's window needs the AllW instantiations.
__host__ __device__ inline bool window_needs_all(const Geom &g) { return g.window >= 2; }

// Sorted node data in the workspace (written by the node kernels).
struct Nodes {
    int32_t *u[kMaxDim];   // grid index floor(n x) mod n, sorted order
    void *delta[kMaxDim];  // n x - floor(n x) (float or double), sorted order
    int32_t *perm;         // sorted position -> caller index
    int32_t *key;          // bin of each node, caller order
    int32_t *rank;         // rank of each node inside its bin, caller order
    int32_t *bin_count;    // [nbins]
    int32_t *bin_start;    // [nbins+1]
    int32_t *bin_chunk;    // [nbins+1] first work item of each bin
    int32_t *chunk_bin;    // [max_chunks]
    int32_t *chunk_first;  // [max_chunks] first sorted node
    int32_t *chunk_len;    // [max_chunks]
    int32_t *counters;     // [0] = number of work items, [1] = non-finite node flag
    void *psi;             // window factors per sorted node: [M][d][W] (float or double)
    int32_t *spos;         // d = 2 spreading in registers, else null: per work item, its
                           // nodes in order of tile row as pairs ((offset << 10) | (row << 5)
                           // | column, caller index)
    // owner-computes spreading (Geom::own), else null
    int32_t *tile_count;   // [ontiles] entries (nodes whose stencils reach it) of every output tile
    int32_t *tile_entry;   // [ontiles+1] first entry of every tile
    void *entries;         // int2 (sorted position, packed tile offsets and block mask) per entry
    int32_t *tile_item;    // [ontiles+1] first work item of every tile
    const int32_t *tile_order;  // [ontiles] tiles in Morton order (the order of their items)
    int32_t *item_tile;    // [max items] tile of a work item
    int32_t *item_lo;      // [max items] its slice [lo, hi) of the tile's node list
    int32_t *item_hi;
    const double *x;       // caller node array (only used while setting nodes)
    // window lookup tables (Geom::lin): per dimension, per stencil point s, kLinK + 1 samples
    // of the factor (lin) and of its derivative (lin_d) at delta = i / kLinK (float or double)
    const void *lin[kMaxDim];
    const void *lin_d[kMaxDim];
    int64_t M;
    int chunk_cap;
    int max_chunks;
};

// Window factors from the lookup tables of the PRE_LIN_PSI strategy (Table 3.2): linear
// interpolation in the offset delta between the kLinK + 1 samples of stencil point s.
constexpr int kLinK = 4096;
template <typename T> __device__ __forceinline__ T lin_lookup(const void *tab, int s, T delta)
{
    const T y = delta * T(kLinK);
    int i = (int)y;
    i = i < 0 ? 0 : (i > kLinK - 1 ? kLinK - 1 : i);
    const T f = y - T(i);
    const T *row = static_cast<const T *>(tab) + (int64_t)s * (kLinK + 1);
    const T a = row[i], b = row[i + 1];
    return a + f * (b - a);
}
// Factor and derivative of dimension t at stencil point s: the closed form, or the tables.
template <typename T, bool AllW = true>
__device__ __forceinline__ T win_value(const Geom &g, const Nodes &nd, int t, T delta, int s)
{
    return g.lin ? lin_lookup<T>(nd.lin[t], s, delta) : win_point<T, AllW>(g, t, delta, s);
}
template <typename T, bool AllW = true>
__device__ __forceinline__ T win_value_d(const Geom &g, const Nodes &nd, int t, T delta, int s)
{
    return g.lin ? lin_lookup<T>(nd.lin_d[t], s, delta) : win_point_d<T, AllW>(g, t, delta, s);
}

}  // namespace nfft
