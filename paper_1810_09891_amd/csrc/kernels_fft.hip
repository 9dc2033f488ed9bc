// The d-variate FFT of Algorithm 2.1 step 2 (sign -) and Algorithm 2.2 step 2 (sign +),
// unnormalised, as one kernel pass per dimension over the oversampled grid, in place.
//
// A workgroup loads `nl` lines of length L = n_t into LDS, transforms them with a
// Stockham autosort FFT (radix 8, 4 and 2 stages, in place between barriers) and writes
// them back.  Only nonzero data is read and only needed data is written:
//  * forward, dimension d-1 first: the deconvolution of Algorithm 2.1 step 1 (eq. (2.9))
//    is fused into the load -- the pass reads the coefficient rows, multiplies them by
//    the FP64 factors prod_t w_t[k_t] = prod_t e^{b_t m} / I0(...), and zero-pads them
//    onto the n_{d-1} line at positions k mod n; only the prod_{q<d-1} N_q rows holding
//    coefficients are transformed;
//  * forward, later passes over dimension t read only the N_t nonzero entries of each
//    line and transform only lines whose indices in dimensions q < t are in I_N;
//  * adjoint passes run t = 0, 1, ..., d-1 and keep only the N_t entries with k in I_N;
//    the last pass applies the deconvolution of Algorithm 2.2 step 3 and writes the
//    centred coefficient array.
#include "batch_desc.hpp"

namespace nfft {

namespace {

// multiplication by SIGN * i
template <typename C, int SIGN> __device__ __forceinline__ C rot(C z)
{
    return SIGN < 0 ? C{z.y, -z.x} : C{-z.y, z.x};
}

template <typename C, int SIGN> __device__ __forceinline__ void dft2(C *v)
{
    C a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename C, int SIGN> __device__ __forceinline__ void dft4(C &a0, C &a1, C &a2, C &a3)
{
    C t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = rot<C, SIGN>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <typename C, int SIGN> __device__ __forceinline__ void dft4v(C *v) { dft4<C, SIGN>(v[0], v[1], v[2], v[3]); }

// X_k = E_k + W8^k O_k, X_{k+4} = E_k - W8^k O_k with E, O the 4-point DFTs of the even
// and odd inputs, W8 = e^{SIGN 2 pi i / 8}.
template <typename C, int SIGN> __device__ __forceinline__ void dft8v(C *v)
{
    using T = decltype(v[0].x);
    const T h = T(0.707106781186547524400844362104849039);
    C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<C, SIGN>(e0, e1, e2, e3);
    dft4<C, SIGN>(o0, o1, o2, o3);
    // W8^1 z = h (z + SIGN i z); W8^2 z = SIGN i z; W8^3 z = h (SIGN i z - z)
    C r1 = rot<C, SIGN>(o1);
    o1 = cscale(cadd(o1, r1), h);
    o2 = rot<C, SIGN>(o2);
    C r3 = rot<C, SIGN>(o3);
    o3 = cscale(csub(r3, o3), h);
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

template <typename C, int SIGN, int R> __device__ __forceinline__ void dftR(C *v)
{
    if constexpr (R == 2)
        dft2<C, SIGN>(v);
    else if constexpr (R == 4)
        dft4v<C, SIGN>(v);
    else
        dft8v<C, SIGN>(v);
}

// LDS position of line element i: one padding element after every 32, so the strided
// accesses of the early Stockham stages (stride R, R^2, ...) spread over the banks.
__device__ __forceinline__ int skew(int i) { return i + (i >> 5); }

// One radix-R Stockham stage over nl lines of length L held in LDS (pitch elements per
// line).  Ns = product of the radices of the earlier stages.  Job (line, j), j < L/R,
// reads x[j + r L/R], multiplies input r by w^{(j mod Ns) r / (Ns R)} with
// w = e^{SIGN 2 pi i}, transforms, and writes y[(j / Ns) Ns R + (j mod Ns) + r Ns].
template <typename T, int VPT, int SIGN, int R>
__device__ __forceinline__ void fft_stage(const Cplx<T> *src, Cplx<T> *dst_buf, int L, int lgL, int nl, int pitch,
                                          int lgNs, const Cplx<T> *tw /* in LDS */)
{
    using C = Cplx<T>;
    constexpr int J = VPT >= R ? VPT / R : 1;
    constexpr int lgR = R == 8 ? 3 : R == 4 ? 2 : 1;
    const int lgJobs = lgL - lgR;  // jobs per line = L / R
    const int jobs = nl << lgJobs;
    const int Ns = 1 << lgNs;
    const int twStep = lgL - lgNs - lgR;  // L / (Ns R) = 2^twStep
    C v[J][R];
    int base[J];
#pragma unroll
    for (int q = 0; q < J; ++q) {
        int b = threadIdx.x + q * kBlock;
        base[q] = -1;
        if (b < jobs) {
            int line = b >> lgJobs;
            int j = b & ((1 << lgJobs) - 1);
            const C *row = src + line * pitch;
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[q][r] = row[skew(j + (r << lgJobs))];
            int jm = j & (Ns - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C w = tw[(jm * r) << twStep];
                if (SIGN > 0)
                    w.y = -w.y;
                v[q][r] = cmul(v[q][r], w);
            }
            dftR<C, SIGN, R>(v[q]);
            base[q] = ((j >> lgNs) << (lgNs + lgR)) + jm;  // position in the line
            base[q] |= line << 24;                            // line index in the high bits
        }
    }
    if (src == dst_buf)  // in place: every read is done before the first write (uniform)
        __syncthreads();
#pragma unroll
    for (int q = 0; q < J; ++q) {
        if (base[q] >= 0) {
            C *dst = dst_buf + (base[q] >> 24) * pitch;
            const int pos = base[q] & 0xffffff;
#pragma unroll
            for (int r = 0; r < R; ++r)
                dst[skew(pos + r * Ns)] = v[q][r];
        }
    }
    __syncthreads();
}

// The same radix-R stage (R = 2, 4, 8) for a line length L that is not a power of two
// (L = 2^a times odd factors): positions and twiddle steps by division instead of shifts.
template <typename T, int VPT, int SIGN, int R>
__device__ __forceinline__ void fft_stage_mixed(const Cplx<T> *src, Cplx<T> *dst_buf, int L, int nl, int pitch, int Ns,
                                                const Cplx<T> *tw /* in LDS */)
{
    using C = Cplx<T>;
    constexpr int J = VPT >= R ? VPT / R : 1;
    const int LR = L / R;  // jobs per line
    const int jobs = nl * LR;
    const int twStep = LR / Ns;  // L / (Ns R)
    C v[J][R];
    int pos[J], lin[J];
#pragma unroll
    for (int q = 0; q < J; ++q) {
        const int b = threadIdx.x + q * kBlock;
        lin[q] = -1;
        if (b < jobs) {
            const int line = b / LR;
            const int j = b - line * LR;
            const C *row = src + line * pitch;
#pragma unroll
            for (int r = 0; r < R; ++r)
                v[q][r] = row[skew(j + r * LR)];
            const int jh = j / Ns;
            const int jm = j - jh * Ns;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                C w = tw[jm * r * twStep];
                if (SIGN > 0)
                    w.y = -w.y;
                v[q][r] = cmul(v[q][r], w);
            }
            dftR<C, SIGN, R>(v[q]);
            pos[q] = jh * Ns * R + jm;
            lin[q] = line;
        }
    }
    if (src == dst_buf)  // in place: every read is done before the first write (uniform)
        __syncthreads();
#pragma unroll
    for (int q = 0; q < J; ++q) {
        if (lin[q] >= 0) {
            C *dst = dst_buf + lin[q] * pitch;
#pragma unroll
            for (int r = 0; r < R; ++r)
                dst[skew(pos[q] + r * Ns)] = v[q][r];
        }
    }
    __syncthreads();
}

// A Stockham stage of odd radix p (any odd factor of L) as direct p-point sums.  Output
// (j, k) of a line, j < L/p, k < p, is sum_r x[j + r L/p] w^{r e} with w = e^{SIGN 2 pi i / L}
// and e = (j mod Ns) L / (Ns p) + k L / p < L: the stage twiddle and the p-point DFT kernel
// combined into one table index r e mod L.  It is written to (j / Ns) Ns p + (j mod Ns) + k Ns.
// A thread computes VPT outputs (VPT kBlock >= nl L), all before the first write.
template <typename T, int VPT, int SIGN>
__device__ __forceinline__ void fft_stage_odd(const Cplx<T> *src, Cplx<T> *dst_buf, int L, int nl, int pitch, int Ns,
                                              int p, const Cplx<T> *tw /* in LDS */)
{
    using C = Cplx<T>;
    const int Lp = L / p;
    const int twStep = Lp / Ns;  // L / (Ns p)
    const int outs = nl * L;
    auto split = [&](int b, int &line, int &j, int &k) {
        line = b / L;
        const int rem = b - line * L;
        k = rem / Lp;
        j = rem - k * Lp;
    };
    C acc[VPT];
    int lb[VPT], jj[VPT], e[VPT], ex[VPT];
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
        int line, j, k;
        split(min((int)threadIdx.x + q * kBlock, outs - 1), line, j, k);
        lb[q] = line * pitch;
        jj[q] = j;
        e[q] = (j % Ns) * twStep + k * Lp;
        ex[q] = 0;
        acc[q] = C{T(0), T(0)};
    }
    for (int r = 0; r < p; ++r) {
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const C x = src[lb[q] + skew(jj[q] + r * Lp)];
            C w = tw[ex[q]];
            if (SIGN > 0)
                w.y = -w.y;
            const C t = cmul(x, w);
            acc[q].x += t.x;
            acc[q].y += t.y;
            ex[q] += e[q];
            ex[q] -= ex[q] >= L ? L : 0;
        }
    }
    __syncthreads();  // every read is done before the first write (in place or not)
#pragma unroll
    for (int q = 0; q < VPT; ++q) {
        const int b = (int)threadIdx.x + q * kBlock;
        if (b < outs) {
            int line, j, k;
            split(b, line, j, k);
            const int jh = j / Ns;
            dst_buf[line * pitch + skew(jh * Ns * p + (j - jh * Ns) + k * Ns)] = acc[q];
        }
    }
    __syncthreads();
}

// Position of centred coefficient index p (k = p - N/2) on a line of length n.
__device__ __forceinline__ int coef_to_pos(int p, int N, int n) { return p < N / 2 ? p - N / 2 + n : p - N / 2; }
// Inverse: centred index of line position i, or -1 when k = i (mod n) is not in I_N.
__device__ __forceinline__ int pos_to_coef(int i, int N, int n)
{
    if (i < N / 2)
        return i + N / 2;
    if (i >= n - N / 2)
        return i - n + N / 2;
    return -1;
}

// a[i] for a runtime i < 3 without indexing the array dynamically (keeps descriptor
// fields in registers instead of private memory)
template <typename A> __device__ __forceinline__ A pick3(const A (&a)[kMaxDim], int i)
{
    return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]);
}

// Per-line data of a line group, computed once per group by the first nl threads.
// Rows (t = d-1): row index r over the pruned dimensions q < d-1.  Columns (t < d-1):
// outer index over dimensions q not in {t, d-1} (pruned when q < t), times a block of
// nl consecutive positions of dimension d-1.  gbase < 0 marks a line past the end.
__device__ __forceinline__ void line_info(const FftPass &p, int g, int c, int64_t &gbase, int &cbase,
                                          double &fac)
{
    gbase = 0;
    cbase = 0;
    fac = 1.0;
    if (p.rows) {
        int r = g * p.nl + c;
        if (r >= p.nrows) {
            gbase = -1;
            return;
        }
        cbase = r * pick3(p.N, p.d - 1);
        int rr = r;
#pragma unroll
        for (int q = kMaxDim - 2; q >= 0; --q) {
            if (q > p.d - 2)
                continue;
            int pq = rr % p.N[q];
            rr /= p.N[q];
            gbase += (int64_t)coef_to_pos(pq, p.N[q], p.n[q]) * p.stride[q];
            if (p.in_mode == 0 || p.out_mode == 2)
                fac *= p.w[q][pq];
        }
        return;
    }
    int o = g / p.ncb;
    int cb = g - o * p.ncb;
    gbase = (int64_t)cb * p.nl + c;  // stride of dimension d-1 is 1
#pragma unroll
    for (int q = kMaxDim - 2; q >= 0; --q) {
        if (q > p.d - 2 || q == p.t)
            continue;
        int ext = q < p.t ? p.N[q] : p.n[q];
        int iq = o % ext;
        o /= ext;
        if (q < p.t)
            iq = coef_to_pos(iq, p.N[q], p.n[q]);
        gbase += (int64_t)iq * p.stride[q];
    }
}

constexpr int kMaxLines = 256;

// One line group g of a pass: load (with the deconvolution when in_mode == 0), transform
// in LDS, store (with the deconvolution when out_mode == 2).  MIX: the line length need not
// be a power of two (radix 8/4/2 stages by division, then one direct stage per odd prime
// factor); this is a separate instantiation so that the power-of-two passes keep their
// register budget.
template <typename T, int VPT, int SIGN, bool MIX>
__device__ __forceinline__ void fft_group(const FftPass &p, const void *fin_ptr, void *fout_ptr, int g,
                                          Cplx<T> *lds, int64_t *s_gbase, int *s_cbase, double *s_fac)
{
    using C = Cplx<T>;
    const int L = p.L, nl = p.nl, pitch = p.pitch;
    // line buffers (a second one when the pass alternates buffers), then the twiddles
    C *buf_a = lds;
    C *buf_b = p.pp ? lds + nl * pitch : lds;
    C *tw = lds + (p.pp ? 2 : 1) * nl * pitch;
    if (threadIdx.x >= 64) {
        // waves 1-3 copy the twiddles (four loads in flight per thread before their LDS
        // stores) while wave 0 sets up the lines below, so the two latencies overlap
        constexpr int kCopy = kBlock - 64;
        const int tid = threadIdx.x - 64;
        const C *twg = static_cast<const C *>(p.tw);
        for (int b = 0; b < L; b += 4 * kCopy) {
            C tv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = b + tid + q * kCopy;
                tv[q] = twg[i < L ? i : 0];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = b + tid + q * kCopy;
                if (i < L)
                    tw[i] = tv[q];
            }
        }
    }
    C *grid = static_cast<C *>(p.grid);
    const int lgL = 31 - __clz(L);
    const int lgnl = 31 - __clz(nl);
    const int total = nl * L;
    const int t = p.t;
    const int Nt = pick3(p.N, t);
    const int64_t st = pick3(p.stride, t);
    const double *wt = pick3(p.w, t);
    const C *fin = static_cast<const C *>(fin_ptr);
    C *fout = static_cast<C *>(fout_ptr);
    const C *mul = static_cast<const C *>(p.mul);
    if (threadIdx.x < nl)
        line_info(p, g, threadIdx.x, s_gbase[threadIdx.x], s_cbase[threadIdx.x], s_fac[threadIdx.x]);
    __syncthreads();
    // Elements idx = base + threadIdx.x + k kBlock, k < SUB, of the nl lines: all loads of a
    // thread are issued before the first of them is used, so their latencies overlap.
    constexpr int SUB = VPT < 8 ? VPT : 8;
    auto line_pos = [&](int idx, int &c, int &i) {
        if (p.rows) {
            if constexpr (MIX) {
                c = idx / L;
                i = idx - c * L;
            } else {
                c = idx >> lgL;
                i = idx & (L - 1);
            }
        } else {
            c = idx & (nl - 1);
            i = idx >> lgnl;
        }
    };
    // ---------------- load (every load is issued, from a clamped valid address, and masked
    // afterwards, so that no branch separates the loads of a thread)
    for (int base = 0; base < total; base += SUB * kBlock) {
        C a[SUB];
        int dst[SUB];
        bool ok[SUB];
        if (p.in_mode == 0) {
            // coefficients times the deconvolution factor (FP64 product, rounded once)
            double wv[SUB], fc[SUB];
#pragma unroll
            for (int k = 0; k < SUB; ++k) {
                const int idx = base + threadIdx.x + k * kBlock;
                int c, i;
                line_pos(min(idx, total - 1), c, i);
                dst[k] = idx < total ? c * pitch + skew(i) : -1;
                const int pc = pos_to_coef(i, Nt, L);
                ok[k] = idx < total && s_gbase[c] >= 0 && pc >= 0;
                const int pcc = ok[k] ? pc : 0;
                a[k] = fin[ok[k] ? s_cbase[c] + pc : 0];
                wv[k] = wt[pcc];
                fc[k] = s_fac[c];
            }
#pragma unroll
            for (int k = 0; k < SUB; ++k) {
                const double f = fc[k] * wv[k];
                a[k] = ok[k] ? C{(T)((double)a[k].x * f), (T)((double)a[k].y * f)} : C{T(0), T(0)};
            }
        } else {
#pragma unroll
            for (int k = 0; k < SUB; ++k) {
                const int idx = base + threadIdx.x + k * kBlock;
                int c, i;
                line_pos(min(idx, total - 1), c, i);
                dst[k] = idx < total ? c * pitch + skew(i) : -1;
                const int64_t gb = s_gbase[c];
                ok[k] = idx < total && gb >= 0 && (p.in_mode == 2 || pos_to_coef(i, Nt, L) >= 0);
                a[k] = grid[ok[k] ? gb + i * st : 0];
            }
#pragma unroll
            for (int k = 0; k < SUB; ++k)
                if (!ok[k])
                    a[k] = C{T(0), T(0)};
        }
#pragma unroll
        for (int k = 0; k < SUB; ++k)
            if (dst[k] >= 0)
                lds[dst[k]] = a[k];
    }
    __syncthreads();

    // ---------------- transform: radix 8 stages, then one radix 4 or 2 stage (and, for
    // other lengths, one direct stage per odd prime factor, smallest first)
    C *cur = buf_a, *nxt = buf_b;
    auto flip = [&]() {
        C *t2 = cur;
        cur = nxt;
        nxt = t2;
    };
    if constexpr (MIX) {
        int Ns = 1, rem = L;
        while (rem % 8 == 0) {
            fft_stage_mixed<T, VPT, SIGN, 8>(cur, nxt, L, nl, pitch, Ns, tw);
            Ns *= 8;
            rem /= 8;
            flip();
        }
        if (rem % 4 == 0) {
            fft_stage_mixed<T, VPT, SIGN, 4>(cur, nxt, L, nl, pitch, Ns, tw);
            Ns *= 4;
            rem /= 4;
            flip();
        } else if (rem % 2 == 0) {
            fft_stage_mixed<T, VPT, SIGN, 2>(cur, nxt, L, nl, pitch, Ns, tw);
            Ns *= 2;
            rem /= 2;
            flip();
        }
        for (int f = 3; rem > 1; f += 2) {
            while (rem % f == 0) {
                fft_stage_odd<T, VPT, SIGN>(cur, nxt, L, nl, pitch, Ns, f, tw);
                Ns *= f;
                rem /= f;
                flip();
            }
        }
    } else {
        int lgNs = 0;
        while (lgL - lgNs >= 3) {
            fft_stage<T, VPT, SIGN, 8>(cur, nxt, L, lgL, nl, pitch, lgNs, tw);
            lgNs += 3;
            flip();
        }
        if (lgL - lgNs == 2) {
            fft_stage<T, VPT, SIGN, 4>(cur, nxt, L, lgL, nl, pitch, lgNs, tw);
            flip();
        } else if (lgL - lgNs == 1) {
            fft_stage<T, VPT, SIGN, 2>(cur, nxt, L, lgL, nl, pitch, lgNs, tw);
            flip();
        }
    }

    // ---------------- store
    if (p.out_mode != 2) {
        for (int idx = threadIdx.x; idx < total; idx += kBlock) {
            int c, i;
            line_pos(idx, c, i);
            const int64_t gb = s_gbase[c];
            if (gb < 0 || (p.out_mode == 1 && pos_to_coef(i, Nt, L) < 0))
                continue;
            grid[gb + i * st] = cur[c * pitch + skew(i)];
        }
    } else {
        // coefficients times the deconvolution factor (and the product coefficients when
        // given): the factor loads of a thread are issued before the first is used
        for (int base = 0; base < total; base += SUB * kBlock) {
            C val[SUB], mv[SUB];
            double wv[SUB], fc[SUB];
            int dst[SUB];
#pragma unroll
            for (int k = 0; k < SUB; ++k) {
                const int idx = base + threadIdx.x + k * kBlock;
                int c, i;
                line_pos(min(idx, total - 1), c, i);
                const int pc = pos_to_coef(i, Nt, L);
                const bool ok = idx < total && s_gbase[c] >= 0 && pc >= 0;
                dst[k] = ok ? s_cbase[c] + pc : -1;
                val[k] = cur[c * pitch + skew(i)];
                wv[k] = wt[ok ? pc : 0];
                fc[k] = s_fac[c];
                mv[k] = mul ? mul[ok ? dst[k] : 0] : C{T(1), T(0)};
            }
#pragma unroll
            for (int k = 0; k < SUB; ++k) {
                if (dst[k] < 0)
                    continue;
                const double f = fc[k] * wv[k];
                C o = C{(T)((double)val[k].x * f), (T)((double)val[k].y * f)};
                if (mul)
                    o = cmul(o, mv[k]);
                fout[dst[k]] = o;
            }
        }
    }
    __syncthreads();
}

template <typename T, int VPT, int SIGN, bool MIX> __global__ __launch_bounds__(kBlock) void k_fft_pass(FftPass p)
{
    using C = Cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int64_t s_gbase[kMaxLines];
    __shared__ int s_cbase[kMaxLines];
    __shared__ double s_fac[kMaxLines];
    C *lds = reinterpret_cast<C *>(smem_raw);
    for (int g = xcd_local_id(blockIdx.x, gridDim.x); g < (int)p.ngroups; g += gridDim.x)
        fft_group<T, VPT, SIGN, MIX>(p, p.fin, p.fout, g, lds, s_gbase, s_cbase, s_fac);
}

// Pass `pass` (forward or adjoint) of every plan of a batch in one launch.
template <typename T, int VPT, int SIGN, bool MIX>
__global__ __launch_bounds__(kBlock) void k_fft_batch(const PlanDev *__restrict__ plans, int count, int pass,
                                                      BatchPtrs ptrs)
{
    using C = Cplx<T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int64_t s_gbase[kMaxLines];
    __shared__ int s_cbase[kMaxLines];
    __shared__ double s_fac[kMaxLines];
    __shared__ int s_cnt[kMaxBatch];
    __shared__ int s_prefix[kMaxBatch + 1];
    C *lds = reinterpret_cast<C *>(smem_raw);
    if ((int)threadIdx.x < count) {
        const PlanDev &pd = plans[threadIdx.x];
        s_cnt[threadIdx.x] = (int)(SIGN < 0 ? pd.fwd[pass].ngroups : pd.adj[pass].ngroups);
    }
    __syncthreads();
    batch_prefix(s_prefix, count, s_cnt);
    const int total = s_prefix[count];
    for (int it = xcd_local_id(blockIdx.x, gridDim.x); it < total; it += gridDim.x) {
        const int pi = batch_find(s_prefix, count, it);
        const PlanDev &pd = plans[pi];
        const FftPass &fp = SIGN < 0 ? pd.fwd[pass] : pd.adj[pass];
        // the caller's arrays of this call: coefficients in (first forward pass) or out
        // (last adjoint pass)
        const void *fin = (SIGN < 0 && pass == 0) ? ptrs.in[pi] : fp.fin;
        void *fout = (SIGN > 0 && pass == pd.nfft - 1) ? ptrs.out[pi] : fp.fout;
        fft_group<T, VPT, SIGN, MIX>(fp, fin, fout, it - s_prefix[pi], lds, s_gbase, s_cbase, s_fac);
    }
}

template <typename T, int SIGN, bool MIX> hipError_t launch_typed(const FftPass &p, int blocks, hipStream_t s)
{
    size_t lds = fft_lds_bytes(p, sizeof(Cplx<T>));
    dim3 grid(blocks), block(kBlock);
#define NFFT_FFT_CALL(V)                                                                               \
    {                                                                                                  \
        auto kf = k_fft_pass<T, V, SIGN, MIX>;                                                         \
        (void)hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL(kf, grid, block, lds, s, p);                                                \
    }
    switch (p.vpt) {
    case 1: NFFT_FFT_CALL(1); break;
    case 2: NFFT_FFT_CALL(2); break;
    case 4: NFFT_FFT_CALL(4); break;
    case 8: NFFT_FFT_CALL(8); break;
    case 16: NFFT_FFT_CALL(16); break;
    case 32:
        if constexpr (MIX)
            return hipErrorInvalidValue;  // mixed-radix passes hold at most 4096 points
        else
            NFFT_FFT_CALL(32);
        break;
    default: return hipErrorInvalidValue;
    }
#undef NFFT_FFT_CALL
    return hipGetLastError();
}

}  // namespace

template <typename T, int SIGN, bool MIX>
hipError_t launch_batch_typed(const PlanDev *plans, int count, int pass, const BatchPtrs &ptrs, int vpt, int blocks,
                              size_t lds, hipStream_t s)
{
    dim3 grid(blocks), block(kBlock);
#define NFFT_FFT_CALL(V)                                                                               \
    {                                                                                                  \
        auto kf = k_fft_batch<T, V, SIGN, MIX>;                                                        \
        (void)hipFuncSetAttribute((const void *)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
        hipLaunchKernelGGL(kf, grid, block, lds, s, plans, count, pass, ptrs);                         \
    }
    switch (vpt) {
    case 1: NFFT_FFT_CALL(1); break;
    case 2: NFFT_FFT_CALL(2); break;
    case 4: NFFT_FFT_CALL(4); break;
    case 8: NFFT_FFT_CALL(8); break;
    case 16: NFFT_FFT_CALL(16); break;
    case 32:
        if constexpr (MIX)
            return hipErrorInvalidValue;
        else
            NFFT_FFT_CALL(32);
        break;
    default: return hipErrorInvalidValue;
    }
#undef NFFT_FFT_CALL
    return hipGetLastError();
}

hipError_t launch_fft_batch(const PlanDev *plans, int count, int pass, bool forward, const BatchPtrs &ptrs,
                            bool dbl, bool mix, int vpt, int blocks, size_t lds, hipStream_t s)
{
    if (mix) {
        if (dbl)
            return forward ? launch_batch_typed<double, -1, true>(plans, count, pass, ptrs, vpt, blocks, lds, s)
                           : launch_batch_typed<double, 1, true>(plans, count, pass, ptrs, vpt, blocks, lds, s);
        return forward ? launch_batch_typed<float, -1, true>(plans, count, pass, ptrs, vpt, blocks, lds, s)
                       : launch_batch_typed<float, 1, true>(plans, count, pass, ptrs, vpt, blocks, lds, s);
    }
    if (dbl)
        return forward ? launch_batch_typed<double, -1, false>(plans, count, pass, ptrs, vpt, blocks, lds, s)
                       : launch_batch_typed<double, 1, false>(plans, count, pass, ptrs, vpt, blocks, lds, s);
    return forward ? launch_batch_typed<float, -1, false>(plans, count, pass, ptrs, vpt, blocks, lds, s)
                   : launch_batch_typed<float, 1, false>(plans, count, pass, ptrs, vpt, blocks, lds, s);
}

hipError_t launch_fft_pass(const FftPass &p, bool dbl, int blocks, hipStream_t s)
{
    if ((p.L & (p.L - 1)) != 0) {
        if (dbl)
            return p.sign < 0 ? launch_typed<double, -1, true>(p, blocks, s) : launch_typed<double, 1, true>(p, blocks, s);
        return p.sign < 0 ? launch_typed<float, -1, true>(p, blocks, s) : launch_typed<float, 1, true>(p, blocks, s);
    }
    if (dbl)
        return p.sign < 0 ? launch_typed<double, -1, false>(p, blocks, s) : launch_typed<double, 1, false>(p, blocks, s);
    return p.sign < 0 ? launch_typed<float, -1, false>(p, blocks, s) : launch_typed<float, 1, false>(p, blocks, s);
}

}  // namespace nfft
