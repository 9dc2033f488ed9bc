// Measured choice of a plan's work decomposition (bin edges and work-item cap): the
// analogue, for the window steps, of the measured FFT plans and wisdom the paper's library
// uses (Sec. 3.1).  Candidates are timed through the library's own entry points on the
// caller's node set; results are kept in a text file keyed by the plan shape.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <fstream>
#include <limits>
#include <sstream>
#include <string>
#include <vector>

#include "nfft_mi355x.h"

namespace {

std::string shape_key(int d, const nfft_plan_info &info, int64_t M)
{
    int mb = 0;
    while (((int64_t)2 << mb) <= M)
        ++mb;
    std::ostringstream k;
    k << "plan-d" << d << "-n";
    for (int t = 0; t < d; ++t)
        k << (t ? "x" : "") << info.n[t];
    k << "-M2^" << mb << "-m" << info.m << "-c" << (info.dtype == NFFT_C128 ? 128 : 64) << "-w" << info.window;
    return k.str();
}

bool cache_lookup(const char *path, const std::string &key, nfft_plan_params &out)
{
    if (!path)
        return false;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        if (line.empty() || line[0] == '#')
            continue;
        std::istringstream ls(line);
        std::string k;
        nfft_plan_params p{};
        if ((ls >> k >> p.bin[0] >> p.bin[1] >> p.bin[2] >> p.chunk_cap) && k == key) {
            out = p;
            return true;
        }
    }
    return false;
}

bool cache_append(const char *path, const std::string &key, const nfft_plan_params &p, double ms)
{
    if (!path)
        return true;
    bool fresh = false;
    {
        std::ifstream in(path);
        fresh = !in.good();
    }
    std::ofstream o(path, std::ios::app);
    if (!o)
        return false;
    if (fresh)
        o << "# NFFT plan parameters: key bin0 bin1 bin2 chunk_cap ms_per_trafo_adjoint\n";
    o << key << " " << p.bin[0] << " " << p.bin[1] << " " << p.bin[2] << " " << p.chunk_cap << " " << ms << "\n";
    return (bool)o;
}

// One candidate: plan, workspace, nodes, one warm-up pair and three timed trafo + adjoint
// pairs on zero stand-in data (the kernels' work does not depend on the values).  Returns
// the time of one pair in ms, infinity when the candidate is not accepted.
double time_candidate(int d, const int64_t *N, int64_t M, const int64_t *n, int m, nfft_dtype dtype, uint32_t flags,
                      const nfft_plan_params &par, const double *x, hipStream_t s, int &status)
{
    const double inf = std::numeric_limits<double>::infinity();
    nfft_plan p = nullptr;
    status = nfft_plan_create_params(&p, d, N, M, n, m, dtype, flags, &par);
    if (status != NFFT_OK)
        return inf;
    size_t ws_bytes = 0;
    nfft_workspace_bytes(p, &ws_bytes);
    int64_t ncoef = 1;
    for (int t = 0; t < d; ++t)
        ncoef *= N[t];
    const size_t cs = dtype == NFFT_C128 ? 16 : 8;
    void *ws = nullptr, *fhat = nullptr, *f = nullptr;
    double ms = inf;
    hipEvent_t a = nullptr, b = nullptr;
    bool ok = hipMalloc(&ws, ws_bytes) == hipSuccess && hipMalloc(&fhat, cs * (size_t)ncoef) == hipSuccess &&
              hipMalloc(&f, cs * (size_t)M) == hipSuccess && hipEventCreate(&a) == hipSuccess &&
              hipEventCreate(&b) == hipSuccess;
    ok = ok && hipMemsetAsync(fhat, 0, cs * (size_t)ncoef, s) == hipSuccess &&
         hipMemsetAsync(f, 0, cs * (size_t)M, s) == hipSuccess;
    ok = ok && nfft_set_workspace(p, ws, ws_bytes) == NFFT_OK && nfft_set_nodes(p, x, s) == NFFT_OK;
    ok = ok && nfft_trafo(p, fhat, f, s) == NFFT_OK && nfft_adjoint(p, f, fhat, s) == NFFT_OK;
    if (ok) {
        constexpr int kReps = 3;
        ok = hipEventRecord(a, s) == hipSuccess;
        for (int r = 0; ok && r < kReps; ++r)
            ok = nfft_trafo(p, fhat, f, s) == NFFT_OK && nfft_adjoint(p, f, fhat, s) == NFFT_OK;
        ok = ok && hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
        float e = 0;
        if (ok && hipEventElapsedTime(&e, a, b) == hipSuccess)
            ms = e / kReps;
    }
    if (!ok)
        status = NFFT_ERR_HIP;
    (void)hipStreamSynchronize(s);
    if (a)
        (void)hipEventDestroy(a);
    if (b)
        (void)hipEventDestroy(b);
    (void)hipFree(ws);
    (void)hipFree(fhat);
    (void)hipFree(f);
    nfft_plan_destroy(p);
    return ms;
}

}  // namespace

// a candidate replaces the best so far only when it is faster by more than the run-to-run
// spread of short timings (about 3% here), so that noise does not pick a decomposition
constexpr double kMargin = 0.95;
constexpr double kMinTuneMs = 0.1;

extern "C" {

int nfft_plan_tune(int d, const int64_t *N, int64_t M, const int64_t *n, int m, nfft_dtype dtype, uint32_t flags,
                   const double *x, const char *cache, hipStream_t s, nfft_plan_params *out, double *best_ms)
{
    if (!out || !x)
        return NFFT_ERR_ARG;
    // the default decomposition (also validates the shape)
    nfft_plan p0 = nullptr;
    int st = nfft_plan_create_params(&p0, d, N, M, n, m, dtype, flags, nullptr);
    if (st != NFFT_OK)
        return st;
    nfft_plan_info info{};
    nfft_plan_get_info(p0, &info);
    nfft_plan_destroy(p0);
    const std::string key = shape_key(d, info, M);
    if (best_ms)
        *best_ms = 0.0;
    if (cache_lookup(cache, key, *out))
        return NFFT_OK;
    nfft_plan_params def{};
    for (int t = 0; t < 3; ++t)
        def.bin[t] = t < d ? (int32_t)info.bin[t] : 1;
    def.chunk_cap = (int32_t)info.chunk_cap;

    nfft_plan_params best = def;
    int cst = NFFT_OK;
    double best_t = time_candidate(d, N, M, n, m, dtype, flags, def, x, s, cst);
    if (cst == NFFT_ERR_HIP)
        return cst;
    // work-item caps with the default bins (plans whose transform pair takes less than
    // kMinTuneMs keep the defaults: their time is launch latency, which no decomposition
    // changes, and the differences measured are noise)
    for (int cap = 128; cap <= 1024 && best_t >= kMinTuneMs; cap *= 2) {
        if (cap == def.chunk_cap)
            continue;
        nfft_plan_params c = def;
        c.chunk_cap = cap;
        const double t = time_candidate(d, N, M, n, m, dtype, flags, c, x, s, cst);
        if (cst == NFFT_ERR_HIP)
            return cst;
        if (t < kMargin * best_t) {
            best_t = t;
            best = c;
        }
    }
    // bin edges halved or doubled per dimension, and halved in every dimension, with that cap
    std::vector<nfft_plan_params> bins;
    for (int t = 0; t < d; ++t) {
        for (int f : {-1, +1}) {
            nfft_plan_params c = best;
            c.bin[t] = f < 0 ? def.bin[t] / 2 : def.bin[t] * 2;
            for (int q = 0; q < d; ++q)
                if (q != t)
                    c.bin[q] = def.bin[q];
            if (c.bin[t] >= 1)
                bins.push_back(c);
        }
    }
    if (d > 1) {
        nfft_plan_params c = best;
        for (int t = 0; t < d; ++t)
            c.bin[t] = def.bin[t] / 2;
        bins.push_back(c);
    }
    if (!(best_t >= kMinTuneMs))
        bins.clear();
    for (const nfft_plan_params &c : bins) {
        const double t = time_candidate(d, N, M, n, m, dtype, flags, c, x, s, cst);
        if (cst == NFFT_ERR_HIP)
            return cst;
        if (t < kMargin * best_t) {
            best_t = t;
            best = c;
        }
    }
    if (!std::isfinite(best_t))
        return NFFT_ERR_UNSUPPORTED;
    *out = best;
    if (best_ms)
        *best_ms = best_t;
    if (!cache_append(cache, key, best, best_t))
        return NFFT_ERR_ARG;
    return NFFT_OK;
}

}  // extern "C"
