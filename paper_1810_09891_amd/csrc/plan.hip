// Host side of the NFFT library: plan validation and defaults, FP64 tables, workspace
// layout, launch sequences of Algorithm 2.1 / 2.2, and the exported C ABI.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/nfft_mi355x.h"
#include "launch.hpp"
#include "plan_impl.hpp"

using namespace nfft;

namespace {

constexpr size_t kAlign = 256;
constexpr size_t kLdsPreferred = 80 * 1024;  // spreading tiles of one workgroup, d >= 2
constexpr size_t kLdsMax = 160 * 1024;       // LDS per compute unit on gfx950
constexpr int kMaxN = 4096;                  // longest FFT line held in one workgroup
constexpr int kMaxM = 12;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// FFT points per thread of a line group of `pts` points: a power of two >= pts / 256
int vpt_of(int pts)
{
    int v = 1;
    while (v * 256 < pts)
        v *= 2;
    return v;
}

int ilog2(int64_t v)
{
    int r = 0;
    while ((int64_t(1) << (r + 1)) <= v)
        ++r;
    return r;
}

}  // namespace

// ------------------------------------------------------------------ plan construction

namespace nfft {

// Bin edges: the requested ones (req[t] > 0: powers of two no longer than the grid, checked
// against the LDS), else the rule below.
static int choose_bins(nfft_plan_s *p, const int32_t *req)
{
    const int d = p->d;
    const size_t cs = p->dbl ? 16 : 8;
    int B[kMaxDim] = {1, 1, 1};
    // starting edges: long tiles in 1-D, 32x32 in 2-D, 8x8x8 in 3-D
    const int start = d == 1 ? 512 : d == 2 ? 32 : 8;
    // (bin edges are powers of two; with a grid length that is not one, the last bin of a
    // dimension holds the remaining n_t mod B_t cells)
    for (int t = 0; t < d; ++t)
        B[t] = 1 << ilog2(std::min<int64_t>(start, p->n[t]));
    // complex128 2-D plans with even m: 16-row bins, the height at which the spreading kernel
    // that keeps tile columns in registers fits its accumulators
    if (d == 2 && p->dbl && 2 * p->m + 2 == p->WM)
        B[0] = std::min(B[0], 16);
    auto lds_of = [&](const int *b) {
        size_t v = cs;
        for (int t = 0; t < d; ++t)
            v *= (size_t)(b[t] + p->WM - 1);
        return v;
    };
    // Shrink the largest edge (outer dimension first on ties) until the tiles fit: the
    // spreading kernel keeps four tiles per workgroup for d = 1, two for d = 2 and one for
    // d = 3 (at most 80 KB for d >= 2, so that two workgroups share a compute unit); the
    // interpolation kernel keeps one.
    const int minB = 4;
    const size_t ntiles = d == 1 ? 4 : d == 2 ? 2 : 1;
    // (1 KB of LDS is left for the static arrays of the batched kernels)
    size_t budget = (d == 1 ? kLdsMax : kLdsPreferred) - 1024;
    // 2-D and 3-D spreading also keep one dummy complex slot per thread after their tiles
    size_t extra = d >= 2 ? (size_t)kBlock * cs : 0;
    // 3-D plans that spread by output tiles (see setup_owner) keep no padded tile there: the
    // bins need only fit the interpolation kernel's one tile
    bool own3 = d == 3;
    for (int t = 0; t < d && own3; ++t)
        own3 = p->n[t] % kOwnTile12 == 0 && p->n[t] >= kOwnTile12 + p->WM - 1;
    if (own3) {
        budget = kLdsMax - 1024;
        extra = 0;
    }
    const bool requested = req && req[0] > 0;
    if (requested) {
        for (int t = 0; t < d; ++t) {
            if (req[t] < 1 || (req[t] & (req[t] - 1)) || req[t] > (1 << ilog2(p->n[t])))
                return NFFT_ERR_ARG;
            B[t] = req[t];
        }
    }
    while (!requested && ntiles * lds_of(B) + extra > budget) {
        int best = -1;
        for (int t = 0; t < d; ++t)
            if (B[t] > minB && B[t] > 1 && (best < 0 || B[t] > B[best]))
                best = t;
        if (best < 0)
            break;
        B[best] /= 2;
    }
    // When even the smallest tile does not fit, 3-D plans that spread by output tiles stage
    // their interpolation tile in slabs of planes along dimension 0 (8 x 8 x 8 bins, work
    // items of at most kBlock nodes); other plans are refused.
    int islab = 0;
    size_t window_lds = lds_of(B);
    if (ntiles * lds_of(B) + extra > kLdsMax - 1024) {
        if (requested || !own3)
            return NFFT_ERR_UNSUPPORTED;
        for (int t = 0; t < d; ++t)
            B[t] = 1 << ilog2(std::min<int64_t>(8, p->n[t]));
        const size_t plane = cs * (size_t)(B[1] + p->WM - 1) * (size_t)(B[2] + p->WM - 1);
        // slabs of half the LDS: two workgroups per CU, as many as the gather's registers allow
        // (m = 9, 10 on the 32^3 test polynomial: 0.84 / 0.90 ms per transform against 1.23 /
        // 1.31 ms with one slab filling the LDS)
        islab = (int)std::min<size_t>((kLdsMax / 2 - 1024) / plane, (size_t)(B[0] + p->WM - 1));
        if (islab < 1)
            return NFFT_ERR_UNSUPPORTED;
        window_lds = plane * (size_t)islab;
    }
    Geom &g = p->geom;
    g.islab = islab;
    g.Ptot = 1;
    g.nbins = 1;
    for (int t = 0; t < kMaxDim; ++t) {
        if (t < d) {
            g.lgB[t] = ilog2(B[t]);
            g.nb[t] = (int)((p->n[t] + B[t] - 1) / B[t]);  // the last bin may be partial
            g.P[t] = B[t] + p->WM - 1;
        } else {
            g.lgB[t] = 0;
            g.nb[t] = 1;
            g.P[t] = 1;
        }
        g.Ptot *= g.P[t];
        g.nbins *= g.nb[t];
    }
    g.fold2 = 1;
    for (int t = 0; t < d; ++t) {
        const int pairs = fold_max_pairs(g, t);
        if (pairs > kFoldMaxPairs)
            return NFFT_ERR_UNSUPPORTED;
        if (pairs > 2)
            g.fold2 = 0;
    }
    p->lds_window = window_lds;
    return NFFT_OK;
}

// Owner-computes spreading for 3-D plans (kernels_own3.hip): output tiles of 16 x 16 x 16
// cells whose node lists are the bins around them.  Used when every node can reach a tile
// through one periodic image only (n_t >= tile edge + 2m + 1), the stencil width is the
// compiled one (even m) and a tile's list is at most kOwnMaxRanges runs of bins.
static void setup_owner(nfft_plan_s *p)
{
    Geom &g = p->geom;
    g.own = 0;
    p->own_max_items = 0;
    if (p->d != 3 || g.W > g.WM)
        return;
    const int T[3] = {kOwnTile0, kOwnTile12, kOwnTile12};
    int okb[3], okn[3], oall[3];
    int64_t tiles_per_bin = 1, ntiles = 1;
    for (int t = 0; t < 3; ++t) {
        const int B = 1 << g.lgB[t];
        if (p->n[t] % T[t] != 0 || p->n[t] < T[t] + g.W - 1 || T[t] % B != 0)
            return;
        // bins holding nodes whose stencil (cells u - m .. u + m + 1) reaches the cells
        // [i T, i T + T - 1] of a tile: from floor((i T - m - 1) / B) to floor((i T + T - 1 + m) / B)
        okb[t] = -((g.m + 1 + B - 1) / B);
        okn[t] = (T[t] - 1 + g.m) / B - okb[t] + 1;
        const int tiles = (int)(p->n[t] / T[t]);
        if (okn[t] >= g.nb[t]) {
            oall[t] = 1;
            okb[t] = 0;
            okn[t] = g.nb[t];
            tiles_per_bin *= tiles;
        } else {
            oall[t] = 0;
            tiles_per_bin *= (okn[t] - 1) / (T[t] / B) + 1;
        }
        ntiles *= tiles;
    }
    if (okn[0] * okn[1] * 2 > kOwnMaxRanges || ntiles > (1 << 24))
        return;
    const int cap = 2048;
    const int64_t list_max = p->M * tiles_per_bin;
    const int64_t items = ntiles + (list_max + cap - 1) / cap + 1;
    if (list_max >= ((int64_t)1 << 31) || items >= ((int64_t)1 << 31))
        return;
    for (int t = 0; t < 3; ++t) {
        g.oT[t] = T[t];
        g.ont[t] = (int)(p->n[t] / T[t]);
        g.okb[t] = okb[t];
        g.okn[t] = okn[t];
        g.oall[t] = oall[t];
    }
    g.ontiles = (int)ntiles;
    g.ocap = cap;
    // tiles in Morton order: interleave the bits of the three tile indices (dimension 0
    // highest), sort by the interleaved code
    {
        std::vector<std::pair<uint64_t, int32_t>> code((size_t)ntiles);
        for (int64_t t = 0; t < ntiles; ++t) {
            const int64_t i2 = t % g.ont[2], i1 = (t / g.ont[2]) % g.ont[1], i0 = t / ((int64_t)g.ont[1] * g.ont[2]);
            uint64_t c = 0;
            for (int b = 0; b < 21; ++b)
                c |= (((uint64_t)(i0 >> b) & 1) << (3 * b + 2)) | (((uint64_t)(i1 >> b) & 1) << (3 * b + 1)) |
                     (((uint64_t)(i2 >> b) & 1) << (3 * b));
            code[(size_t)t] = {c, (int32_t)t};
        }
        std::sort(code.begin(), code.end());
        p->tile_order.resize((size_t)ntiles);
        for (int64_t t = 0; t < ntiles; ++t)
            p->tile_order[(size_t)t] = code[(size_t)t].second;
    }
    p->own_max_entries = list_max;
    p->own_max_items = (int)items;
    g.own = 1;
}

static void plan_fft_pass(nfft_plan_s *p, int t, bool forward, bool first_or_last, FftPass &fp)
{
    const int d = p->d;
    std::memset(&fp, 0, sizeof(fp));
    fp.d = d;
    fp.t = t;
    fp.L = (int)p->n[t];
    for (int q = 0; q < kMaxDim; ++q) {
        fp.N[q] = q < d ? (int)p->N[q] : 1;
        fp.n[q] = q < d ? (int)p->n[q] : 1;
    }
    int64_t st = 1;
    for (int q = d - 1; q >= 0; --q) {
        fp.stride[q] = st;
        st *= p->n[q];
    }
    fp.sign = forward ? -1 : +1;
    fp.rows = (t == d - 1) ? 1 : 0;
    if (forward) {
        fp.in_mode = first_or_last ? 0 : 1;
        fp.out_mode = 0;
    } else {
        fp.in_mode = 2;
        fp.out_mode = first_or_last ? 2 : 1;
    }
    const int L = fp.L;
    const bool mix = (L & (L - 1)) != 0;
    // points per workgroup: mixed-radix passes (L not a power of two) hold at most 4096, so
    // that their direct odd-radix stages keep 16 outputs per thread in registers
    const int maxPts = (p->dbl || mix) ? 4096 : 8192;
    // Aim for at least 512 line groups (two per compute unit) before packing more lines
    // into a workgroup; column passes keep >= 2 adjacent columns per row segment.
    const int64_t target = 512;
    int nl;
    if (fp.rows) {
        int64_t nrows = 1;
        for (int q = 0; q < d - 1; ++q)
            nrows *= p->N[q];
        fp.nrows = (int)nrows;
        nl = 1;
        while ((int64_t)nl * 2 * L <= maxPts && nl * 2 <= 256 && nrows / (nl * 2) >= target)
            nl *= 2;
        fp.ngroups = (nrows + nl - 1) / nl;
    } else {
        int64_t outer = 1;
        for (int q = 0; q < d - 1; ++q) {
            if (q == t)
                continue;
            outer *= (q < t) ? p->N[q] : p->n[q];
        }
        const int inner = (int)p->n[d - 1];
        nl = std::min<int>(inner, std::max(1, maxPts / L));
        nl = std::min(nl, std::min(256, 16));  // 16 adjacent columns: 128 / 256-byte row segments
        // a power of two that divides n_{d-1} (n_{d-1} is even, so 2 always does)
        {
            int v = 1;
            while (v * 2 <= nl && inner % (v * 2) == 0)
                v *= 2;
            nl = v;
        }
        while (nl > 2 && outer * (inner / nl) < target)
            nl /= 2;
        fp.ncb = inner / nl;
        fp.ngroups = outer * fp.ncb;
    }
    fp.nl = nl;
    // line pitch in LDS: L elements plus one skew element per 32 (and one more for columns)
    fp.pitch = L + (L >> 5) + (fp.rows ? 0 : 1);
    fp.vpt = vpt_of(nl * L);
    fft_choose_buffers(fp, p->dbl ? 16 : 8);
}

}  // namespace nfft

bool plan_repack_pass(const nfft_plan_s *p, const FftPass &tmpl, int factor, FftPass &out)
{
    out = tmpl;
    if (factor == 1)
        return true;
    const bool mix = (tmpl.L & (tmpl.L - 1)) != 0;
    const int maxPts = (p->dbl || mix) ? 4096 : 8192;
    int nl = tmpl.nl * factor;
    if (nl < 1 || nl > 256 || (int64_t)nl * tmpl.L > maxPts)
        return false;
    if (tmpl.rows) {
        if (nl > tmpl.nrows)
            return false;
        out.ngroups = (tmpl.nrows + nl - 1) / nl;
    } else {
        const int inner = (int)p->n[p->d - 1];
        if (nl > inner || nl < 2 || inner % nl != 0)
            return false;
        const int64_t outer = tmpl.ngroups / tmpl.ncb;
        out.ncb = inner / nl;
        out.ngroups = outer * out.ncb;
    }
    out.nl = nl;
    out.vpt = vpt_of(nl * tmpl.L);
    fft_choose_buffers(out, p->dbl ? 16 : 8);
    return true;
}

// Centred cardinal B-spline M_k(u) = N_k(u + k/2) in FP64 (host tables of the sinc window):
// de Boor's triangle over the k values N_q(t + j) nonzero at the fractional part t, all
// terms nonnegative.
static double centred_bspline(int k, double u)
{
    const double x = u + 0.5 * k;
    if (!(x >= 0.0) || x >= (double)k)
        return 0.0;
    const double t = x - std::floor(x);
    const int j = (int)std::floor(x);
    std::vector<double> b((size_t)k + 1, 0.0);
    b[0] = 1.0;
    for (int q = 2; q <= k; ++q)
        for (int i = q - 1; i >= 0; --i) {
            const double left = i > 0 ? b[(size_t)i - 1] : 0.0;
            b[(size_t)i] = ((t + i) * b[(size_t)i] + (q - t - i) * left) / (q - 1);
        }
    return b[(size_t)j];
}

static int build_tables(nfft_plan_s *p)
{
    const double pi = 3.14159265358979323846264338327950288;
    const bool gauss = (p->flags & NFFT_WINDOW_GAUSSIAN) != 0;
    const bool bspline = (p->flags & NFFT_WINDOW_BSPLINE) != 0;
    const bool sinc = (p->flags & NFFT_WINDOW_SINC) != 0;
    p->geom.window = gauss ? 1 : bspline ? 2 : sinc ? 3 : 0;
    for (int t = 0; t < p->d; ++t) {
        // The device evaluates the window divided by lambda and the deconvolution factor is
        // lambda / Phi(k), Phi(k) = n phihat(k) the window's Fourier transform at k / n.
        p->wtab[t].resize((size_t)p->N[t]);
        if (bspline) {
            // Phi(k) = (sin(pi k/n) / (pi k/n))^(2m), lambda = 1
            p->geom.b[t] = 0.0;
            p->geom.emb[t] = 1.0;
            for (int64_t i = 0; i < p->N[t]; ++i) {
                const double a = pi * (double)(i - p->N[t] / 2) / (double)p->n[t];
                const double s = a == 0.0 ? 1.0 : std::sin(a) / a;
                p->wtab[t][(size_t)i] = 1.0 / std::pow(s, 2.0 * p->m);
            }
        } else if (sinc) {
            // a = pi (2 - 1/sigma) / (2m), Phi(k) = (pi/a) M_2m(pi k / (n a)), lambda = 1
            const double a = pi * (2.0 - (double)p->N[t] / (double)p->n[t]) / (2.0 * p->m);
            p->geom.b[t] = a;
            p->geom.emb[t] = 1.0;
            for (int64_t i = 0; i < p->N[t]; ++i) {
                const double u = pi * (double)(i - p->N[t] / 2) / ((double)p->n[t] * a);
                p->wtab[t][(size_t)i] = 1.0 / ((pi / a) * centred_bspline(2 * p->m, u));
            }
        } else if (gauss) {
            // b = 2 sigma m / ((2 sigma - 1) pi), Phi(k) = exp(-b (pi k / n)^2),
            // lambda = (pi b)^{-1/2} (the window's peak)
            const double sigma = (double)p->n[t] / (double)p->N[t];
            const double b = 2.0 * sigma * p->m / ((2.0 * sigma - 1.0) * pi);
            const double lambda = 1.0 / std::sqrt(pi * b);
            p->geom.b[t] = b;
            p->geom.emb[t] = 1.0 / lambda;
            for (int64_t i = 0; i < p->N[t]; ++i) {
                const double a = pi * (double)(i - p->N[t] / 2) / (double)p->n[t];
                p->wtab[t][(size_t)i] = lambda * std::exp(b * a * a);
            }
        } else {
            // b = pi (2 - 1/sigma), Phi(k) = I0(m sqrt(b^2 - (2 pi k/n)^2)), lambda = e^{b m}
            const double b = pi * (2.0 - (double)p->N[t] / (double)p->n[t]);
            p->geom.b[t] = b;
            p->geom.emb[t] = std::exp(-b * p->m);
            for (int64_t i = 0; i < p->N[t]; ++i) {
                const double k = (double)(i - p->N[t] / 2);
                const double w = 2.0 * pi * k / (double)p->n[t];
                const double arg = (double)p->m * std::sqrt(b * b - w * w);
                const double i0 = std::cyl_bessel_i(0.0, arg);
                p->wtab[t][(size_t)i] = std::exp(b * p->m) / i0;
            }
        }
        // twiddles e^{-2 pi i k / n}, k < n, from the exact angle of each k
        p->twd[t].resize((size_t)p->n[t]);
        p->twf[t].resize((size_t)p->n[t]);
        for (int64_t k = 0; k < p->n[t]; ++k) {
            const double a = 2.0 * pi * (double)k / (double)p->n[t];
            double c = std::cos(a), s = -std::sin(a);
            p->twd[t][(size_t)k] = double2{c, s};
            p->twf[t][(size_t)k] = float2{(float)c, (float)s};
        }
    }
    for (int t = p->d; t < kMaxDim; ++t) {
        p->geom.b[t] = 0.0;
        p->geom.emb[t] = 1.0;
    }
    return NFFT_OK;
}

static void layout_workspace(nfft_plan_s *p)
{
    const size_t cs = p->dbl ? 16 : 8;
    const size_t rs = p->dbl ? 8 : 4;
    const int64_t M = p->M;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    int64_t ngrid = 1;
    for (int t = 0; t < p->d; ++t)
        ngrid *= p->n[t];
    p->ngrid = ngrid;
    for (int t = 0; t < p->d; ++t)
        p->off_w[t] = take(sizeof(double) * (size_t)p->N[t]);
    for (int t = 0; t < p->d; ++t)
        p->off_tw[t] = take(cs * (size_t)p->n[t]);
    p->off_grid = take(cs * (size_t)ngrid);
    p->off_grid_adj = (p->flags & NFFT_KEEP_GRID) ? take(cs * (size_t)ngrid) : p->off_grid;
    for (int t = 0; t < p->d; ++t)
        p->off_u[t] = take(4 * (size_t)M);
    for (int t = 0; t < p->d; ++t)
        p->off_delta[t] = take(rs * (size_t)M);
    p->off_perm = take(4 * (size_t)M);
    p->off_key = take(4 * (size_t)M);
    p->off_rank = take(4 * (size_t)M);
    p->off_bin_count = take(4 * (size_t)p->geom.nbins);
    p->off_bin_start = take(4 * (size_t)(p->geom.nbins + 1));
    p->off_bin_chunk = take(4 * (size_t)(p->geom.nbins + 1));
    p->off_chunk_bin = take(4 * (size_t)p->max_chunks);
    p->off_chunk_first = take(4 * (size_t)p->max_chunks);
    p->off_chunk_len = take(4 * (size_t)p->max_chunks);
    p->off_counters = take(64);
    p->off_xcopy = take(sizeof(double) * (size_t)M * p->d);
    // window factors, padded so that reads of WM (>= 2m+2) factors past the last node's
    // record stay inside the workspace
    p->off_psi = take(rs * ((size_t)M * p->d * (size_t)(2 * p->m + 2) + 64));
    for (int t = 0; t < p->d; ++t) {
        const size_t ntab = p->geom.lin ? (size_t)(2 * p->m + 2) * (kLinK + 1) : 0;
        p->off_lin[t] = take(rs * ntab);
        p->off_lin_d[t] = take(rs * ntab);
    }
    // one padded tile per work item for the tile spreading kernels; owner-computes plans
    // need tile lists, work items and one partial tile per item instead
    p->off_scratch = take(p->geom.own ? 0 : cs * (size_t)p->geom.Ptot * (size_t)p->max_chunks);
    if (p->geom.own) {
        const size_t items = (size_t)p->own_max_items;
        const size_t tc = (size_t)p->geom.oT[0] * p->geom.oT[1] * p->geom.oT[2];
        p->off_tile_count = take(4 * (size_t)p->geom.ontiles);
        p->off_tile_order = take(4 * (size_t)p->geom.ontiles);
        p->off_tile_entry = take(4 * ((size_t)p->geom.ontiles + 1));
        p->off_entries = take(8 * (size_t)p->own_max_entries);
        p->off_own_fs = take(cs * (size_t)M);
        p->off_tile_item = take(4 * ((size_t)p->geom.ontiles + 1));
        p->off_item_tile = take(4 * items);
        p->off_item_lo = take(4 * items);
        p->off_item_hi = take(4 * items);
        p->off_own_scratch = take(cs * tc * items);
    }
    p->spos_used = spread_in_registers(p->geom, p->dbl);
    if (p->spos_used)
        p->off_spos = take(8 * (size_t)M);
    p->ws_bytes = off;
}

static int create_plan(nfft_plan_s **out, int d, const int64_t *N, int64_t M, const int64_t *n, int m,
                       nfft_dtype dtype, uint32_t flags, const nfft_plan_params *params)
{
    if (!out || !N || d < 1 || d > kMaxDim || M < 1 || M > (int64_t)0x7fffffff)
        return NFFT_ERR_ARG;
    if (dtype != NFFT_C64 && dtype != NFFT_C128)
        return NFFT_ERR_ARG;
    if (m == 0)
        m = 8;
    if (m < 1)
        return NFFT_ERR_ARG;
    {
        const uint32_t win = flags & (NFFT_WINDOW_GAUSSIAN | NFFT_WINDOW_BSPLINE | NFFT_WINDOW_SINC);
        if (win & (win - 1))
            return NFFT_ERR_ARG;  // more than one window
    }
    int64_t nn[kMaxDim];
    for (int t = 0; t < d; ++t) {
        if (N[t] < 2 || (N[t] & 1))
            return NFFT_ERR_ARG;
        if (n) {
            nn[t] = n[t];
        } else {
            int e = 0;
            while ((int64_t(1) << e) < N[t])
                ++e;
            nn[t] = int64_t(1) << (e + 1);
        }
        if (nn[t] <= N[t] || (nn[t] & 1))
            return NFFT_ERR_ARG;
        if (2 * m + 2 > nn[t])
            return NFFT_ERR_ARG;
    }
    for (int t = 0; t < d; ++t)
        if (nn[t] > kMaxN)
            return NFFT_ERR_UNSUPPORTED;
    if (m > kMaxM)
        return NFFT_ERR_UNSUPPORTED;

    nfft_plan_s *p = new (std::nothrow) nfft_plan_s();
    if (!p)
        return NFFT_ERR_ARG;
    p->d = d;
    p->m = m;
    p->dtype = dtype;
    p->dbl = dtype == NFFT_C128;
    p->flags = flags | NFFT_SORT_NODES;
    p->M = M;
    for (int t = 0; t < kMaxDim; ++t) {
        p->N[t] = t < d ? N[t] : 1;
        p->n[t] = t < d ? nn[t] : 1;
    }
    Geom &g = p->geom;
    std::memset(&g, 0, sizeof(g));
    g.d = d;
    g.m = m;
    g.W = 2 * m + 2;
    g.WM = wm_bucket(m);
    p->WM = g.WM;
    g.lin = (flags & NFFT_PRE_LIN_PSI) ? 1 : 0;
    g.p2 = 1;
    for (int t = 0; t < kMaxDim; ++t) {
        g.n[t] = (int)p->n[t];
        g.p2 = g.p2 && is_pow2(p->n[t]);
    }
    if (params && params->chunk_cap != 0 &&
        (params->chunk_cap < 32 || params->chunk_cap > 1024 || (params->chunk_cap & (params->chunk_cap - 1)))) {
        delete p;
        return NFFT_ERR_ARG;
    }
    int st = choose_bins(p, params ? params->bin : nullptr);
    if (st != NFFT_OK) {
        delete p;
        return st;
    }
    // Work items hold at most chunk_cap nodes of one bin: M / 512 rounded down to a power
    // of two, between 128 and 1024, so that a dense bin of a clustered node set is split
    // over many workgroups while uniform node sets keep about one item per bin.
    p->chunk_cap = 128;
    while (p->chunk_cap < 1024 && (int64_t)p->chunk_cap * 2 * 512 <= M)
        p->chunk_cap *= 2;
    if (params && params->chunk_cap > 0)
        p->chunk_cap = params->chunk_cap;
    if (g.islab > 0) {
        // one node per thread across the slabs
        if (p->chunk_cap > kBlock && params && params->chunk_cap > 0) {
            delete p;
            return NFFT_ERR_UNSUPPORTED;
        }
        p->chunk_cap = std::min(p->chunk_cap, kBlock);
    }
    p->max_chunks = (int)(g.nbins + (M + p->chunk_cap - 1) / p->chunk_cap);
    setup_owner(p);
    if (g.islab > 0 && !g.own) {  // the spreading tile would not fit either
        delete p;
        return NFFT_ERR_UNSUPPORTED;
    }
    build_tables(p);
    // FFT passes
    p->fwd_passes.clear();
    for (int t = d - 1; t >= 0; --t) {
        FftPass fp;
        plan_fft_pass(p, t, true, t == d - 1, fp);
        p->fwd_passes.push_back(fp);
    }
    p->adj_passes.clear();
    for (int t = 0; t < d; ++t) {
        FftPass fp;
        plan_fft_pass(p, t, false, t == d - 1, fp);
        p->adj_passes.push_back(fp);
    }
    layout_workspace(p);
    *out = p;
    return NFFT_OK;
}

// ------------------------------------------------------------------ device views

Nodes plan_node_view(nfft_plan_s *p)
{
    Nodes nd;
    std::memset(&nd, 0, sizeof(nd));
    char *ws = static_cast<char *>(p->ws);
    for (int t = 0; t < p->d; ++t) {
        nd.u[t] = reinterpret_cast<int32_t *>(ws + p->off_u[t]);
        nd.delta[t] = ws + p->off_delta[t];
    }
    nd.perm = reinterpret_cast<int32_t *>(ws + p->off_perm);
    nd.key = reinterpret_cast<int32_t *>(ws + p->off_key);
    nd.rank = reinterpret_cast<int32_t *>(ws + p->off_rank);
    nd.bin_count = reinterpret_cast<int32_t *>(ws + p->off_bin_count);
    nd.bin_start = reinterpret_cast<int32_t *>(ws + p->off_bin_start);
    nd.bin_chunk = reinterpret_cast<int32_t *>(ws + p->off_bin_chunk);
    nd.chunk_bin = reinterpret_cast<int32_t *>(ws + p->off_chunk_bin);
    nd.chunk_first = reinterpret_cast<int32_t *>(ws + p->off_chunk_first);
    nd.chunk_len = reinterpret_cast<int32_t *>(ws + p->off_chunk_len);
    nd.counters = reinterpret_cast<int32_t *>(ws + p->off_counters);
    nd.psi = ws + p->off_psi;
    for (int t = 0; t < kMaxDim; ++t) {
        nd.lin[t] = (p->geom.lin && t < p->d) ? ws + p->off_lin[t] : nullptr;
        nd.lin_d[t] = (p->geom.lin && t < p->d) ? ws + p->off_lin_d[t] : nullptr;
    }
    nd.spos = p->spos_used ? reinterpret_cast<int32_t *>(ws + p->off_spos) : nullptr;
    if (p->geom.own) {
        nd.tile_count = reinterpret_cast<int32_t *>(ws + p->off_tile_count);
        nd.tile_order = reinterpret_cast<const int32_t *>(ws + p->off_tile_order);
        nd.tile_entry = reinterpret_cast<int32_t *>(ws + p->off_tile_entry);
        nd.entries = ws + p->off_entries;
        nd.tile_item = reinterpret_cast<int32_t *>(ws + p->off_tile_item);
        nd.item_tile = reinterpret_cast<int32_t *>(ws + p->off_item_tile);
        nd.item_lo = reinterpret_cast<int32_t *>(ws + p->off_item_lo);
        nd.item_hi = reinterpret_cast<int32_t *>(ws + p->off_item_hi);
    }
    nd.M = p->M;
    nd.chunk_cap = p->chunk_cap;
    nd.max_chunks = p->max_chunks;
    return nd;
}

FftPass plan_bind_pass(nfft_plan_s *p, const FftPass &tmpl, void *grid, const void *fin, void *fout)
{
    FftPass fp = tmpl;
    char *ws = static_cast<char *>(p->ws);
    fp.grid = grid;
    fp.fin = fin;
    fp.fout = fout;
    for (int t = 0; t < kMaxDim; ++t)
        fp.w[t] = t < p->d ? reinterpret_cast<const double *>(ws + p->off_w[t]) : nullptr;
    fp.tw = ws + p->off_tw[tmpl.t];
    fp.mul = nullptr;
    return fp;
}

// ------------------------------------------------------------------ profiling

static void prof_begin(nfft_plan_s *p, hipStream_t s)
{
    if (!p->prof_on)
        return;
    hipEvent_t e;
    if (p->ev_pool.empty()) {
        if (hipEventCreate(&e) != hipSuccess)
            return;
    } else {
        e = p->ev_pool.back();
        p->ev_pool.pop_back();
    }
    (void)hipEventRecord(e, s);
    p->ev_open = e;
}

static void prof_end(nfft_plan_s *p, hipStream_t s, const char *name)
{
    if (!p->prof_on || !p->ev_open)
        return;
    hipEvent_t e;
    if (p->ev_pool.empty()) {
        if (hipEventCreate(&e) != hipSuccess)
            return;
    } else {
        e = p->ev_pool.back();
        p->ev_pool.pop_back();
    }
    (void)hipEventRecord(e, s);
    p->ev_pending.push_back({name, p->ev_open, e});
    p->ev_open = nullptr;
}

#define LAUNCH(p, s, name, call)                                                                      \
    do {                                                                                              \
        prof_begin(p, s);                                                                             \
        hipError_t e_ = (call);                                                                       \
        prof_end(p, s, name);                                                                         \
        if (e_ != hipSuccess) {                                                                       \
            p->last_hip_error = e_;                                                                   \
            return NFFT_ERR_HIP;                                                                      \
        }                                                                                             \
    } while (0)

// ------------------------------------------------------------------ launch sequences

static int grid_blocks(nfft_plan_s *p)
{
    // work items are visited with a grid-stride loop; one workgroup per item up to the bound
    return std::max(1, std::min(p->max_chunks, 1 << 20));
}

static int run_forward_grid(nfft_plan_s *p, const void *fhat, void *grid, hipStream_t s)
{
    for (size_t i = 0; i < p->fwd_passes.size(); ++i) {
        FftPass fp = plan_bind_pass(p, p->fwd_passes[i], grid, fhat, nullptr);
        int blocks = (int)std::min<int64_t>(fp.ngroups, 1 << 20);
        LAUNCH(p, s, i == 0 ? "fft_fwd_deconv" : "fft_fwd", launch_fft_pass(fp, p->dbl, blocks, s));
    }
    return NFFT_OK;
}

static int run_adjoint_coeffs(nfft_plan_s *p, void *grid, void *hhat, hipStream_t s, const void *mul = nullptr)
{
    for (size_t i = 0; i < p->adj_passes.size(); ++i) {
        FftPass fp = plan_bind_pass(p, p->adj_passes[i], grid, nullptr, hhat);
        if (i + 1 == p->adj_passes.size())
            fp.mul = mul;
        int blocks = (int)std::min<int64_t>(fp.ngroups, 1 << 20);
        LAUNCH(p, s, i + 1 == p->adj_passes.size() ? "fft_adj_deconv" : "fft_adj",
               launch_fft_pass(fp, p->dbl, blocks, s));
    }
    return NFFT_OK;
}

static int run_interp(nfft_plan_s *p, const void *grid, void *f, hipStream_t s)
{
    Nodes nd = plan_node_view(p);
    LAUNCH(p, s, "interp",
           launch_interp(p->geom, nd, p->dbl, grid, f, grid_blocks(p), interp_lds_bytes(p->geom, p->dbl), s));
    return NFFT_OK;
}

static int run_spread(nfft_plan_s *p, const void *f, void *grid, hipStream_t s)
{
    Nodes nd = plan_node_view(p);
    if (p->geom.own) {
        void *own = static_cast<char *>(p->ws) + p->off_own_scratch;
        void *fs = static_cast<char *>(p->ws) + p->off_own_fs;
        LAUNCH(p, s, "spread_own",
               launch_spread_own(p->geom, nd, p->dbl, f, fs, grid, own, p->own_max_items, s));
        LAUNCH(p, s, "spread_own_fold", launch_own_fold(p->geom, nd, p->dbl, own, grid, s));
        return NFFT_OK;
    }
    void *scratch = static_cast<char *>(p->ws) + p->off_scratch;
    LAUNCH(p, s, "spread_tiles",
           launch_spread_tiles(p->geom, nd, p->dbl, f, scratch, grid_blocks(p),
                               spread_lds_bytes(p->geom, p->dbl), s));
    LAUNCH(p, s, "spread_fold", launch_fold(p->geom, nd, p->dbl, scratch, grid, s));
    return NFFT_OK;
}

static int ensure_tables(nfft_plan_s *p, hipStream_t s)
{
    if (p->tables_on_device)
        return NFFT_OK;
    char *ws = static_cast<char *>(p->ws);
    for (int t = 0; t < p->d; ++t) {
        if (hipMemcpyAsync(ws + p->off_w[t], p->wtab[t].data(), sizeof(double) * p->wtab[t].size(),
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return NFFT_ERR_HIP;
        const void *src = p->dbl ? (const void *)p->twd[t].data() : (const void *)p->twf[t].data();
        size_t bytes = (p->dbl ? 16 : 8) * (size_t)p->n[t];
        if (hipMemcpyAsync(ws + p->off_tw[t], src, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
            return NFFT_ERR_HIP;
    }
    if (p->geom.own && hipMemcpyAsync(ws + p->off_tile_order, p->tile_order.data(), 4 * p->tile_order.size(),
                                      hipMemcpyHostToDevice, s) != hipSuccess)
        return NFFT_ERR_HIP;
    if (p->geom.lin)
        for (int t = 0; t < p->d; ++t)
            if (launch_fill_lin(p->geom, t, p->dbl, ws + p->off_lin[t], ws + p->off_lin_d[t], s) != hipSuccess)
                return NFFT_ERR_HIP;
    // the host tables stay alive in the plan; wait so a later destroy cannot race the copy
    if (hipStreamSynchronize(s) != hipSuccess)
        return NFFT_ERR_HIP;
    p->tables_on_device = true;
    return NFFT_OK;
}

// ------------------------------------------------------------------ exported ABI

extern "C" {

const char *nfft_status_string(int status)
{
    switch (status) {
    case NFFT_OK: return "ok";
    case NFFT_ERR_ARG: return "invalid argument";
    case NFFT_ERR_STATE: return "call out of order";
    case NFFT_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case NFFT_ERR_HIP: return "HIP call failed";
    case NFFT_ERR_UNSUPPORTED: return "not supported by this library";
    default: return "unknown status";
    }
}

int nfft_plan_create(nfft_plan *out, int d, const int64_t *N, int64_t M, const int64_t *n, int m,
                     nfft_dtype dtype, uint32_t flags)
{
    if (!out)
        return NFFT_ERR_ARG;
    nfft_plan_s *p = nullptr;
    int st = create_plan(&p, d, N, M, n, m, dtype, flags, nullptr);
    if (st == NFFT_OK)
        *out = p;
    return st;
}

int nfft_plan_create_params(nfft_plan *out, int d, const int64_t *N, int64_t M, const int64_t *n, int m,
                            nfft_dtype dtype, uint32_t flags, const nfft_plan_params *params)
{
    if (!out)
        return NFFT_ERR_ARG;
    nfft_plan_s *p = nullptr;
    int st = create_plan(&p, d, N, M, n, m, dtype, flags, params);
    if (st == NFFT_OK)
        *out = p;
    return st;
}

int nfft_plan_destroy(nfft_plan p)
{
    if (!p)
        return NFFT_ERR_ARG;
    for (auto &pe : p->ev_pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    for (auto e : p->ev_pool)
        (void)hipEventDestroy(e);
    delete p;
    return NFFT_OK;
}

int nfft_plan_get_info(nfft_plan p, nfft_plan_info *info)
{
    if (!p || !info)
        return NFFT_ERR_ARG;
    std::memset(info, 0, sizeof(*info));
    info->d = p->d;
    info->m = p->m;
    info->dtype = p->dtype;
    info->flags = p->flags;
    info->M = p->M;
    for (int t = 0; t < kMaxDim; ++t) {
        info->N[t] = p->N[t];
        info->n[t] = p->n[t];
        info->bin[t] = (int64_t)1 << p->geom.lgB[t];
    }
    info->nbins = p->geom.nbins;
    info->chunk_cap = p->chunk_cap;
    info->max_chunks = p->max_chunks;
    info->workspace_bytes = p->ws_bytes;
    info->lds_bytes = p->lds_window;
    double sc = 1.0;
    for (int t = 0; t < p->d; ++t)
        sc /= p->geom.emb[t];
    info->grid_scale = sc;
    info->window = p->geom.window;
    info->own_tiles = p->geom.own ? p->geom.ontiles : 0;
    for (int t = 0; t < kMaxDim; ++t)
        info->own_tile[t] = p->geom.own ? p->geom.oT[t] : 0;
    return NFFT_OK;
}

int nfft_workspace_bytes(nfft_plan p, size_t *bytes)
{
    if (!p || !bytes)
        return NFFT_ERR_ARG;
    *bytes = p->ws_bytes;
    return NFFT_OK;
}

int nfft_set_workspace(nfft_plan p, void *ws, size_t bytes)
{
    if (!p)
        return NFFT_ERR_ARG;
    if (!ws || bytes < p->ws_bytes || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
        return NFFT_ERR_WORKSPACE;
    p->ws = ws;
    p->tables_on_device = false;
    p->nodes_set = false;
    p->grid_valid = false;
    return NFFT_OK;
}

int nfft_set_nodes(nfft_plan p, const double *x, hipStream_t s)
{
    if (!p || !x)
        return NFFT_ERR_ARG;
    if (!p->ws)
        return NFFT_ERR_WORKSPACE;
    int st = ensure_tables(p, s);
    if (st != NFFT_OK)
        return st;
    Nodes nd = plan_node_view(p);
    nd.x = x;
    double *xcopy = reinterpret_cast<double *>(static_cast<char *>(p->ws) + p->off_xcopy);
    p->nodes_set = false;
    p->grid_valid = false;
    LAUNCH(p, s, "nodes_reset", launch_node_reset(p->geom, nd, s));
    LAUNCH(p, s, "nodes_key", launch_node_key(p->geom, nd, xcopy, s));
    LAUNCH(p, s, "nodes_scan", launch_node_scan(p->geom, nd, s));
    LAUNCH(p, s, "nodes_scatter", launch_node_scatter(p->geom, nd, p->dbl, s));
    if (p->geom.own)
        LAUNCH(p, s, "nodes_tiles", launch_own_items(p->geom, nd, s));
    p->nodes_set = true;
    return NFFT_OK;
}

int nfft_nodes_finite(nfft_plan p, int *all_finite, hipStream_t s)
{
    if (!p || !all_finite)
        return NFFT_ERR_ARG;
    if (!p->ws)
        return NFFT_ERR_WORKSPACE;
    if (!p->nodes_set)
        return NFFT_ERR_STATE;
    const int32_t *counters = reinterpret_cast<const int32_t *>(static_cast<char *>(p->ws) + p->off_counters);
    int32_t flag = 0;
    if (hipMemcpyAsync(&flag, counters + 1, sizeof(flag), hipMemcpyDeviceToHost, s) != hipSuccess)
        return NFFT_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess)
        return NFFT_ERR_HIP;
    *all_finite = flag ? 0 : 1;
    return NFFT_OK;
}

static int check_ready(nfft_plan p)
{
    if (!p)
        return NFFT_ERR_ARG;
    if (!p->ws)
        return NFFT_ERR_WORKSPACE;
    if (!p->nodes_set)
        return NFFT_ERR_STATE;
    return NFFT_OK;
}

int nfft_trafo(nfft_plan p, const void *fhat, void *f, hipStream_t s)
{
    int st = check_ready(p);
    if (st != NFFT_OK)
        return st;
    if (!fhat || !f)
        return NFFT_ERR_ARG;
    void *grid = static_cast<char *>(p->ws) + p->off_grid;
    if ((st = run_forward_grid(p, fhat, grid, s)) != NFFT_OK)
        return st;
    if ((st = run_interp(p, grid, f, s)) != NFFT_OK)
        return st;
    p->grid_valid = true;
    return NFFT_OK;
}

int nfft_adjoint(nfft_plan p, const void *f, void *hhat, hipStream_t s)
{
    int st = check_ready(p);
    if (st != NFFT_OK)
        return st;
    if (!f || !hhat)
        return NFFT_ERR_ARG;
    void *grid = static_cast<char *>(p->ws) + p->off_grid_adj;
    if ((st = run_spread(p, f, grid, s)) != NFFT_OK)
        return st;
    if ((st = run_adjoint_coeffs(p, grid, hhat, s)) != NFFT_OK)
        return st;
    if (p->off_grid_adj == p->off_grid)
        p->grid_valid = false;
    return NFFT_OK;
}

int nfft_fastsum(nfft_plan px, nfft_plan py, const void *bhat, const void *alpha, void *g, void *coef_work,
                 hipStream_t s)
{
    int st = check_ready(px);
    if (st != NFFT_OK)
        return st;
    if ((st = check_ready(py)) != NFFT_OK)
        return st;
    if (!bhat || !alpha || !g || !coef_work)
        return NFFT_ERR_ARG;
    if (px->d != py->d || px->dtype != py->dtype)
        return NFFT_ERR_ARG;
    for (int t = 0; t < px->d; ++t)
        if (px->N[t] != py->N[t])
            return NFFT_ERR_ARG;
    // coefficients of the kernel sum: bhat (.) A_x^H alpha, the product taken in the
    // adjoint's last pass
    void *gx = static_cast<char *>(px->ws) + px->off_grid_adj;
    if ((st = run_spread(px, alpha, gx, s)) != NFFT_OK)
        return st;
    if ((st = run_adjoint_coeffs(px, gx, coef_work, s, bhat)) != NFFT_OK)
        return st;
    if (px->off_grid_adj == px->off_grid)
        px->grid_valid = false;
    // g = A_y coef
    void *gy = static_cast<char *>(py->ws) + py->off_grid;
    if ((st = run_forward_grid(py, coef_work, gy, s)) != NFFT_OK)
        return st;
    if ((st = run_interp(py, gy, g, s)) != NFFT_OK)
        return st;
    py->grid_valid = true;
    return NFFT_OK;
}

int nfft_step_grid(nfft_plan p, const void *fhat, void *g, hipStream_t s)
{
    if (!p || !fhat || !g)
        return NFFT_ERR_ARG;
    if (!p->ws)
        return NFFT_ERR_WORKSPACE;
    int st = ensure_tables(p, s);
    if (st != NFFT_OK)
        return st;
    return run_forward_grid(p, fhat, g, s);
}

int nfft_step_interp(nfft_plan p, const void *g, void *f, hipStream_t s)
{
    int st = check_ready(p);
    if (st != NFFT_OK)
        return st;
    if (!g || !f)
        return NFFT_ERR_ARG;
    return run_interp(p, g, f, s);
}

int nfft_step_spread(nfft_plan p, const void *f, void *g, hipStream_t s)
{
    int st = check_ready(p);
    if (st != NFFT_OK)
        return st;
    if (!g || !f)
        return NFFT_ERR_ARG;
    return run_spread(p, f, g, s);
}

int nfft_step_coeffs(nfft_plan p, const void *g, void *hhat, hipStream_t s)
{
    if (!p || !g || !hhat)
        return NFFT_ERR_ARG;
    if (!p->ws)
        return NFFT_ERR_WORKSPACE;
    int st = ensure_tables(p, s);
    if (st != NFFT_OK)
        return st;
    // the passes work in place: transform a copy held in the workspace grid
    void *grid = static_cast<char *>(p->ws) + p->off_grid_adj;
    if (hipMemcpyAsync(grid, g, (p->dbl ? 16 : 8) * (size_t)p->ngrid, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return NFFT_ERR_HIP;
    if (p->off_grid_adj == p->off_grid)
        p->grid_valid = false;
    return run_adjoint_coeffs(p, grid, hhat, s);
}

static int run_ndft(nfft_plan p, const void *in, void *out, bool adjoint, hipStream_t s)
{
    int st = check_ready(p);
    if (st != NFFT_OK)
        return st;
    if (!in || !out)
        return NFFT_ERR_ARG;
    NdftArgs a;
    std::memset(&a, 0, sizeof(a));
    a.d = p->d;
    a.K = 1;
    for (int t = 0; t < kMaxDim; ++t) {
        a.N[t] = (int)p->N[t];
        if (t < p->d)
            a.K *= p->N[t];
    }
    a.M = p->M;
    a.x = reinterpret_cast<const double *>(static_cast<char *>(p->ws) + p->off_xcopy);
    a.in = in;
    a.out = out;
    LAUNCH(p, s, adjoint ? "ndft_adjoint" : "ndft_trafo", launch_ndft(a, p->dbl, adjoint, s));
    return NFFT_OK;
}

int ndft_trafo(nfft_plan p, const void *fhat, void *f, hipStream_t s) { return run_ndft(p, fhat, f, false, s); }

int ndft_adjoint(nfft_plan p, const void *f, void *hhat, hipStream_t s) { return run_ndft(p, f, hhat, true, s); }

int nfft_grad_x(nfft_plan p, const void *v, void *grad_x, hipStream_t s)
{
    int st = check_ready(p);
    if (st != NFFT_OK)
        return st;
    if (!v || !grad_x)
        return NFFT_ERR_ARG;
    if (!(p->flags & NFFT_KEEP_GRID) || !p->grid_valid)
        return NFFT_ERR_STATE;
    Nodes nd = plan_node_view(p);
    const void *grid = static_cast<char *>(p->ws) + p->off_grid;
    LAUNCH(p, s, "grad_x",
           launch_grad_x(p->geom, nd, p->dbl, grid, v, grad_x, grid_blocks(p), interp_lds_bytes(p->geom, p->dbl),
                         s));
    return NFFT_OK;
}

int nfft_profile_enable(nfft_plan p, int on)
{
    if (!p)
        return NFFT_ERR_ARG;
    p->prof_on = on != 0;
    return NFFT_OK;
}

int nfft_profile_read(nfft_plan p, const char **names, double *total_ms, int64_t *launches, int cap, int *count)
{
    if (!p || !count)
        return NFFT_ERR_ARG;
    std::map<std::string, std::pair<double, int64_t>> acc;
    for (auto &pe : p->ev_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pe.a, pe.b) == hipSuccess) {
            auto &slot = acc[pe.name];
            slot.first += ms;
            slot.second += 1;
        }
        p->ev_pool.push_back(pe.a);
        p->ev_pool.push_back(pe.b);
    }
    p->ev_pending.clear();
    int i = 0;
    for (auto &kv : acc) {
        if (i < cap) {
            // names point at the static strings passed to LAUNCH
            names[i] = p->intern(kv.first);
            total_ms[i] = kv.second.first;
            launches[i] = kv.second.second;
        }
        ++i;
    }
    *count = i;
    return NFFT_OK;
}

}  // extern "C"
