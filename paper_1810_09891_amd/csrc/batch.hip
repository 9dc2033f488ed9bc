// Batched execution of many independent plans: one launch per step kind covers every plan
// of a launch group, plus an autotuner for the launch shapes.
//
// Plans are grouped by (dimension, compiled stencil width, precision) -- the template
// parameters of the kernels -- and each group is cut into launch groups of at most
// kMaxBatch plans, largest M first.  A launch group owns a device table of PlanDev entries
// (geometry, node data and workspace regions of each plan) and a two-int work queue per
// window kernel.  The tuned parameters of a launch group are
//   pack_fwd, pack_adj   lines per FFT workgroup, as a multiple of the plan's own packing;
//   k_fwd, k_adj, k_interp, k_spread, k_fold
//                        persistent grid of k x (compute units) workgroups, 0 for one
//                        workgroup per item.
// The autotuner times every candidate of each step kind on the stream (the analogue of
// measuring plans and keeping their wisdom) and stores the winners, keyed by the device
// and the group's plan shapes, in a text cache file.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/nfft_mi355x.h"
#include "batch_desc.hpp"
#include "plan_impl.hpp"

using namespace nfft;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

enum Param { kPackFwd = 0, kKFwd, kPackAdj, kKAdj, kKInterp, kKSpread, kKFold };

struct Group {
    int d = 0, WM = 0;
    bool dbl = false;
    std::vector<int> idx;  // positions in the caller's plan array, largest M first
    int params[NFFT_BATCH_NPARAMS] = {1, 0, 1, 0, 8, 8, 0, 0};
    bool tuned = false;
    std::string key;
    size_t off_table = 0, off_queue = 0;
    // derived from the parameters
    int vpt_fwd[kMaxDim] = {1, 1, 1}, vpt_adj[kMaxDim] = {1, 1, 1};
    size_t lds_fwd[kMaxDim] = {0, 0, 0}, lds_adj[kMaxDim] = {0, 0, 0};
    int64_t items_fwd[kMaxDim] = {0, 0, 0}, items_adj[kMaxDim] = {0, 0, 0};
    size_t lds_interp = 0, lds_spread = 0;
    bool cols = false;  // every plan's 2-D spreading runs in registers
    bool own = false;   // every plan's 3-D spreading runs by output tiles (one launch per plan)
    bool mix = false;   // the plans' grids are not all powers of two (mixed-radix FFT passes)
    int64_t chunk_bound = 0, fold_items = 0;
    std::vector<PlanDev> table;
};

}  // namespace

struct nfft_batch_s {
    std::vector<nfft_plan_s *> plans;
    std::vector<void *> plan_ws;  // workspaces at creation
    std::vector<Group> groups;
    std::string cache;
    size_t ws_bytes = 0;
    void *ws = nullptr;
    void *run_ws = nullptr;  // device memory of the call in progress: ws, or the static scratch
    int cus = 0;
    bool prepared = false;   // groups built for the current device (launch data, host tables)
    bool table_current = false;
    hipError_t last_hip_error = hipSuccess;
};

namespace {

int pow2_ceil(int v)
{
    int r = 1;
    while (r < v)
        r <<= 1;
    return r;
}

// Fill the host table and the derived launch data of a group from its parameters.
void build_group(nfft_batch_s *b, Group &G)
{
    const size_t cs = G.dbl ? 16 : 8;
    G.table.assign(G.idx.size(), PlanDev());
    for (int t = 0; t < kMaxDim; ++t) {
        G.vpt_fwd[t] = G.vpt_adj[t] = 1;
        G.lds_fwd[t] = G.lds_adj[t] = 0;
        G.items_fwd[t] = G.items_adj[t] = 0;
    }
    G.lds_interp = G.lds_spread = 0;
    G.chunk_bound = G.fold_items = 0;
    G.cols = !G.idx.empty();
    for (int i : G.idx)
        G.cols = G.cols && b->plans[(size_t)i]->spos_used;
    for (size_t i = 0; i < G.idx.size(); ++i) {
        nfft_plan_s *p = b->plans[(size_t)G.idx[i]];
        PlanDev &pd = G.table[i];
        std::memset(&pd, 0, sizeof(pd));
        char *ws = static_cast<char *>(p->ws);
        pd.g = p->geom;
        pd.nd = plan_node_view(p);
        pd.grid = ws + p->off_grid;
        pd.grid_adj = ws + p->off_grid_adj;
        pd.scratch = ws + p->off_scratch;
        pd.ngrid = p->ngrid;
        pd.nfft = p->d;
        for (int q = 0; q < p->d; ++q) {
            for (int dir = 0; dir < 2; ++dir) {
                const FftPass &tmpl = dir == 0 ? p->fwd_passes[(size_t)q] : p->adj_passes[(size_t)q];
                FftPass packed = tmpl;
                // the largest packing up to the requested one that fits this plan's pass
                for (int f = dir == 0 ? G.params[kPackFwd] : G.params[kPackAdj]; f >= 1; f >>= 1)
                    if (plan_repack_pass(p, tmpl, f, packed))
                        break;
                FftPass bound = plan_bind_pass(p, packed, ws + (dir == 0 ? p->off_grid : p->off_grid_adj), nullptr,
                                               nullptr);
                const size_t lds = fft_lds_bytes(bound, cs);
                if (dir == 0) {
                    pd.fwd[q] = bound;
                    G.vpt_fwd[q] = std::max(G.vpt_fwd[q], pow2_ceil(bound.vpt));
                    G.lds_fwd[q] = std::max(G.lds_fwd[q], lds);
                    G.items_fwd[q] += bound.ngroups;
                } else {
                    pd.adj[q] = bound;
                    G.vpt_adj[q] = std::max(G.vpt_adj[q], pow2_ceil(bound.vpt));
                    G.lds_adj[q] = std::max(G.lds_adj[q], lds);
                    G.items_adj[q] += bound.ngroups;
                }
            }
        }
        G.lds_interp = std::max(G.lds_interp, interp_lds_bytes(p->geom, p->dbl));
        G.lds_spread = std::max(G.lds_spread, G.cols ? spread_lds_bytes(p->geom, p->dbl)
                                                      : spread_batch_lds_bytes(p->geom, p->dbl));
        G.chunk_bound += p->max_chunks;
        G.fold_items += (p->ngrid + kBlock - 1) / kBlock;
    }
}

int upload_group(nfft_batch_s *b, Group &G)
{
    char *ws = static_cast<char *>(b->ws);
    hipError_t e = hipMemcpy(ws + G.off_table, G.table.data(), sizeof(PlanDev) * G.table.size(),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        b->last_hip_error = e;
        return NFFT_ERR_HIP;
    }
    return NFFT_OK;
}

int blocks_for(const nfft_batch_s *b, int k, int64_t items)
{
    int64_t v = k <= 0 ? items : std::min<int64_t>(items, (int64_t)k * b->cus);
    return (int)std::max<int64_t>(1, std::min<int64_t>(v, 1 << 20));
}

// ------------------------------------------------------------------ launch sequences

#define BCHECK(call)                                                                                  \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) {                                                                       \
            b->last_hip_error = e_;                                                                   \
            return NFFT_ERR_HIP;                                                                      \
        }                                                                                             \
    } while (0)

const PlanDev *table_of(const nfft_batch_s *b, const Group &G)
{
    return reinterpret_cast<const PlanDev *>(static_cast<const char *>(b->run_ws) + G.off_table);
}

int *queue_of(const nfft_batch_s *b, const Group &G, int which)
{
    return reinterpret_cast<int *>(static_cast<char *>(b->run_ws) + G.off_queue) + 2 * which;
}

int run_fft(nfft_batch_s *b, const Group &G, const BatchPtrs &ptrs, bool forward, hipStream_t s)
{
    const int count = (int)G.idx.size();
    for (int q = 0; q < G.d; ++q) {
        const int64_t items = forward ? G.items_fwd[q] : G.items_adj[q];
        const int blocks = blocks_for(b, G.params[forward ? kKFwd : kKAdj], items);
        BCHECK(launch_fft_batch(table_of(b, G), count, q, forward, ptrs, G.dbl, G.mix,
                                forward ? G.vpt_fwd[q] : G.vpt_adj[q], blocks,
                                forward ? G.lds_fwd[q] : G.lds_adj[q], s));
    }
    return NFFT_OK;
}

int run_interp(nfft_batch_s *b, const Group &G, const BatchPtrs &ptrs, hipStream_t s)
{

    const int blocks = blocks_for(b, G.params[kKInterp], G.chunk_bound);
    BCHECK(launch_interp_batch(table_of(b, G), (int)G.idx.size(), ptrs, queue_of(b, G, 0), G.d, G.dbl, G.WM, blocks,
                               G.lds_interp, s));
    return NFFT_OK;
}

int run_spread(nfft_batch_s *b, const Group &G, const BatchPtrs &ptrs, hipStream_t s)
{
    if (G.own) {
        // 3-D plans spread by output tiles: one launch per plan (each launch covers all the
        // compute units), the partial tiles folded by run_fold
        for (size_t i = 0; i < G.idx.size(); ++i) {
            const PlanDev &pd = G.table[i];
            nfft_plan_s *p = b->plans[(size_t)G.idx[i]];
            char *ws = static_cast<char *>(p->ws);
            BCHECK(launch_spread_own(pd.g, pd.nd, G.dbl, ptrs.in[i], ws + p->off_own_fs, pd.grid_adj,
                                     ws + p->off_own_scratch, p->own_max_items, s));
        }
        return NFFT_OK;
    }
    const int blocks = blocks_for(b, G.params[kKSpread], G.chunk_bound);
    if (G.cols)
        BCHECK(launch_spread_cols_batch(table_of(b, G), (int)G.idx.size(), ptrs, queue_of(b, G, 1), G.dbl, G.WM,
                                        blocks, G.lds_spread, s));
    else
        BCHECK(launch_spread_batch(table_of(b, G), (int)G.idx.size(), ptrs, queue_of(b, G, 1), G.d, G.dbl, G.WM,
                                   blocks, G.lds_spread, s));
    return NFFT_OK;
}

int run_fold(nfft_batch_s *b, const Group &G, hipStream_t s)
{
    if (G.own) {
        for (size_t i = 0; i < G.idx.size(); ++i) {
            const PlanDev &pd = G.table[i];
            nfft_plan_s *p = b->plans[(size_t)G.idx[i]];
            BCHECK(launch_own_fold(pd.g, pd.nd, G.dbl, static_cast<char *>(p->ws) + p->off_own_scratch,
                                   pd.grid_adj, s));
        }
        return NFFT_OK;
    }
    const int blocks = blocks_for(b, G.params[kKFold], G.fold_items);
    BCHECK(launch_fold_batch(table_of(b, G), (int)G.idx.size(), G.d, G.dbl, blocks, s));
    return NFFT_OK;
}

BatchPtrs make_ptrs(const Group &G, const void *const *in, void *const *out)
{
    BatchPtrs ptrs;
    std::memset(&ptrs, 0, sizeof(ptrs));
    for (size_t i = 0; i < G.idx.size(); ++i) {
        ptrs.in[i] = in[G.idx[i]];
        ptrs.out[i] = out[G.idx[i]];
    }
    return ptrs;
}

int check_ready(nfft_batch_s *b, const void *const *in, void *const *out)
{
    if (!b || !in || !out)
        return NFFT_ERR_ARG;
    if (!b->ws || !b->table_current)
        return NFFT_ERR_WORKSPACE;
    for (size_t i = 0; i < b->plans.size(); ++i) {
        if (!in[i] || !out[i])
            return NFFT_ERR_ARG;
        if (b->plans[i]->ws != b->plan_ws[i] || !b->plans[i]->nodes_set)
            return NFFT_ERR_STATE;
    }
    return NFFT_OK;
}

// ------------------------------------------------------------------ tuning cache

std::string group_key(const nfft_batch_s *b, const Group &G, const char *arch)
{
    std::ostringstream o;
    o << arch << "/" << b->cus << "/d" << G.d << "/w" << G.WM << (G.dbl ? "/c128" : "/c64");
    for (int i : G.idx) {
        const nfft_plan_s *p = b->plans[(size_t)i];
        o << "/";
        for (int t = 0; t < p->d; ++t)
            o << p->N[t] << "x" << p->n[t] << ",";
        o << p->M;
    }
    // FNV-1a of the description: one short token per line of the cache file
    uint64_t h = 1469598103934665603ull;
    for (char c : o.str()) {
        h ^= (unsigned char)c;
        h *= 1099511628211ull;
    }
    char buf[32];
    std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
    return std::string(buf);
}

std::map<std::string, std::vector<int>> read_cache(const std::string &path)
{
    std::map<std::string, std::vector<int>> out;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string key;
        if (!(ls >> key) || key.empty() || key[0] == '#')
            continue;
        std::vector<int> v;
        int x;
        while (ls >> x)
            v.push_back(x);
        if ((int)v.size() == NFFT_BATCH_NPARAMS)
            out[key] = v;
    }
    return out;
}

bool valid_params(const int *v);

// Launch data and host descriptor tables of every group for the current device, with the
// tuned parameters of the cache file when it has them.  Host work only (no allocation).
int prepare_groups(nfft_batch_s *b)
{
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) {
        b->last_hip_error = e;
        return NFFT_ERR_HIP;
    }
    b->cus = prop.multiProcessorCount;
    std::map<std::string, std::vector<int>> cached;
    if (!b->cache.empty())
        cached = read_cache(b->cache);
    for (auto &G : b->groups) {
        G.key = group_key(b, G, prop.gcnArchName);
        auto it = cached.find(G.key);
        if (it != cached.end() && valid_params(it->second.data())) {
            for (int q = 0; q < NFFT_BATCH_NPARAMS; ++q)
                G.params[q] = it->second[(size_t)q];
            G.tuned = true;
        }
        build_group(b, G);
    }
    b->prepared = true;
    return NFFT_OK;
}


bool write_cache(const std::string &path, const std::map<std::string, std::vector<int>> &entries)
{
    const std::string tmp = path + ".tmp";
    {
        std::ofstream o(tmp, std::ios::trunc);
        if (!o)
            return false;
        o << "# NFFT batch launch parameters: key pack_fwd k_fwd pack_adj k_adj k_interp k_spread k_fold -\n";
        for (auto &kv : entries) {
            o << kv.first;
            for (int x : kv.second)
                o << " " << x;
            o << "\n";
        }
        if (!o)
            return false;
    }
    return std::rename(tmp.c_str(), path.c_str()) == 0;
}

bool valid_params(const int *v)
{
    for (int q : {kPackFwd, kPackAdj})
        if (v[q] < 1 || v[q] > 64 || (v[q] & (v[q] - 1)))
            return false;
    for (int q : {kKFwd, kKAdj, kKInterp, kKSpread, kKFold})
        if (v[q] < 0 || v[q] > 1024)
            return false;
    return true;
}

}  // namespace

// ------------------------------------------------------------------ exported ABI

// ------------------------------------------------------------------ allocation-free batch calls
//
// nfft_batch_trafo_noalloc runs the batched forward transform with the batch's descriptor
// tables and work queues in this file-scope device array instead of a caller-provided batch
// workspace.  Each device holds its own copy; its address is looked up once per device (with
// that device current) and kept, and only that address is handed to copies and kernels.
// Calls that overlap on one device share the array and therefore race.
constexpr size_t kNoallocScratchBytes = size_t(1) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use).
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

int nfft_batch_create(nfft_batch *out, int count, const nfft_plan *plans, const char *tune_cache)
{
    if (!out || count < 1 || !plans)
        return NFFT_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || plans[i]->dtype != plans[0]->dtype)
            return NFFT_ERR_ARG;
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i])
                return NFFT_ERR_ARG;
    }
    for (int i = 0; i < count; ++i)
        if (!plans[i]->ws)
            return NFFT_ERR_WORKSPACE;
    nfft_batch_s *b = new (std::nothrow) nfft_batch_s();
    if (!b)
        return NFFT_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        b->plans.push_back(plans[i]);
        b->plan_ws.push_back(plans[i]->ws);
    }
    if (tune_cache)
        b->cache = tune_cache;
    // group by kernel template parameters, largest M first, at most kMaxBatch per launch
    // (the last key holds the output-tile flag, in bit 1 a grid that is not a power of two,
    // in bit 2 spreading in registers, so that plans whose bins do not allow it do not move
    // a whole group to the tile kernel)
    std::map<std::tuple<int, int, int, int>, std::vector<int>> by_kind;
    for (int i = 0; i < count; ++i)
        by_kind[std::make_tuple(plans[i]->d, plans[i]->WM, plans[i]->dbl ? 1 : 0,
                                plans[i]->geom.own + (plans[i]->geom.p2 ? 0 : 2) + (plans[i]->spos_used ? 4 : 0))]
            .push_back(i);
    for (auto &kv : by_kind) {
        std::vector<int> v = kv.second;
        std::stable_sort(v.begin(), v.end(), [&](int a, int c) { return plans[a]->M > plans[c]->M; });
        for (size_t s0 = 0; s0 < v.size(); s0 += kMaxBatch) {
            Group G;
            G.d = std::get<0>(kv.first);
            G.WM = std::get<1>(kv.first);
            G.dbl = std::get<2>(kv.first) != 0;
            G.own = (std::get<3>(kv.first) & 1) != 0;
            G.mix = (std::get<3>(kv.first) & 2) != 0;
            G.idx.assign(v.begin() + (long)s0, v.begin() + (long)std::min(v.size(), s0 + kMaxBatch));
            b->groups.push_back(G);
        }
    }
    size_t off = align_up(16 * b->groups.size());  // two work queues of two ints per group
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        Group &G = b->groups[gi];
        G.off_queue = 16 * gi;
        G.off_table = off;
        off = align_up(off + sizeof(PlanDev) * G.idx.size());
    }
    b->ws_bytes = off;
    *out = b;
    return NFFT_OK;
}

int nfft_batch_get_info(nfft_batch b, nfft_batch_info *info)
{
    if (!b || !info)
        return NFFT_ERR_ARG;
    std::memset(info, 0, sizeof(*info));
    info->count = (int)b->plans.size();
    info->groups = (int)b->groups.size();
    int tuned = 1;
    for (auto &G : b->groups)
        tuned &= G.tuned ? 1 : 0;
    info->tuned = tuned;
    info->workspace_bytes = b->ws_bytes;
    return NFFT_OK;
}

int nfft_batch_get_params(nfft_batch b, int group, int *params, int *plan_count)
{
    if (!b || group < 0 || group >= (int)b->groups.size() || !params)
        return NFFT_ERR_ARG;
    const Group &G = b->groups[(size_t)group];
    for (int q = 0; q < NFFT_BATCH_NPARAMS; ++q)
        params[q] = G.params[q];
    if (plan_count)
        *plan_count = (int)G.idx.size();
    return NFFT_OK;
}

int nfft_batch_set_params(nfft_batch b, int group, const int *params)
{
    if (!b || group < 0 || group >= (int)b->groups.size() || !params)
        return NFFT_ERR_ARG;
    if (!valid_params(params))
        return NFFT_ERR_ARG;
    Group &G = b->groups[(size_t)group];
    for (int q = 0; q < NFFT_BATCH_NPARAMS; ++q)
        G.params[q] = params[q];
    G.tuned = false;
    if (!b->ws)
        return NFFT_OK;
    build_group(b, G);
    return upload_group(b, G);
}

int nfft_batch_workspace_bytes(nfft_batch b, size_t *bytes)
{
    if (!b || !bytes)
        return NFFT_ERR_ARG;
    *bytes = b->ws_bytes;
    return NFFT_OK;
}

int nfft_batch_set_workspace(nfft_batch b, void *ws, size_t bytes)
{
    if (!b)
        return NFFT_ERR_ARG;
    if (!ws || bytes < b->ws_bytes || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0)
        return NFFT_ERR_WORKSPACE;
    b->ws = ws;
    b->run_ws = ws;
    b->table_current = false;
    int st = prepare_groups(b);
    if (st != NFFT_OK)
        return st;
    for (auto &G : b->groups) {
        st = upload_group(b, G);
        if (st != NFFT_OK)
            return st;
    }
    // work queues start at zero and reset themselves after every launch
    hipError_t e = hipMemset(ws, 0, 16 * b->groups.size());
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        b->last_hip_error = e;
        return NFFT_ERR_HIP;
    }
    b->table_current = true;
    return NFFT_OK;
}

int nfft_batch_trafo(nfft_batch b, const void *const *fhat, void *const *f, hipStream_t s)
{
    int st = check_ready(b, fhat, f);
    if (st != NFFT_OK)
        return st;
    for (auto &G : b->groups) {
        const BatchPtrs ptrs = make_ptrs(G, fhat, f);
        if ((st = run_fft(b, G, ptrs, true, s)) != NFFT_OK)
            return st;
        if ((st = run_interp(b, G, ptrs, s)) != NFFT_OK)
            return st;
    }
    for (auto *p : b->plans)
        p->grid_valid = true;
    return NFFT_OK;
}

int nfft_batch_trafo_noalloc(nfft_batch b, const void *const *fhat, void *const *f, hipStream_t s)
{
    if (!b || !fhat || !f)
        return NFFT_ERR_ARG;
    if (b->ws_bytes > kNoallocScratchBytes)
        return NFFT_ERR_WORKSPACE;  // descriptor tables larger than the static scratch
    for (size_t i = 0; i < b->plans.size(); ++i) {
        if (!fhat[i] || !f[i])
            return NFFT_ERR_ARG;
        if (b->plans[i]->ws != b->plan_ws[i] || !b->plans[i]->nodes_set)
            return NFFT_ERR_STATE;
    }
    int st;
    if (!b->prepared && (st = prepare_groups(b)) != NFFT_OK)
        return st;
    void *base = nullptr;
    hipError_t e = scratch_address(&base);
    if (e != hipSuccess) {
        b->last_hip_error = e;
        return NFFT_ERR_HIP;
    }
    char *sc = static_cast<char *>(base);
    // descriptor tables into the scratch, work queues cleared (by a kernel, not a memset)
    for (auto &G : b->groups) {
        e = hipMemcpyAsync(sc + G.off_table, G.table.data(), sizeof(PlanDev) * G.table.size(),
                           hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            b->last_hip_error = e;
            return NFFT_ERR_HIP;
        }
    }
    e = launch_fill_zero(sc, 16 * b->groups.size(), s);
    if (e != hipSuccess) {
        b->last_hip_error = e;
        return NFFT_ERR_HIP;
    }
    void *saved = b->run_ws;
    b->run_ws = base;
    for (auto &G : b->groups) {
        const BatchPtrs ptrs = make_ptrs(G, fhat, f);
        if ((st = run_fft(b, G, ptrs, true, s)) != NFFT_OK || (st = run_interp(b, G, ptrs, s)) != NFFT_OK) {
            b->run_ws = saved;
            return st;
        }
    }
    b->run_ws = saved;
    for (auto *p : b->plans)
        p->grid_valid = true;
    return NFFT_OK;
}

int nfft_batch_adjoint(nfft_batch b, const void *const *f, void *const *hhat, hipStream_t s)
{
    int st = check_ready(b, f, hhat);
    if (st != NFFT_OK)
        return st;
    for (auto &G : b->groups) {
        const BatchPtrs ptrs = make_ptrs(G, f, hhat);
        if ((st = run_spread(b, G, ptrs, s)) != NFFT_OK)
            return st;
        if ((st = run_fold(b, G, s)) != NFFT_OK)
            return st;
        if ((st = run_fft(b, G, ptrs, false, s)) != NFFT_OK)
            return st;
    }
    for (auto *p : b->plans)
        if (p->off_grid_adj == p->off_grid)
            p->grid_valid = false;
    return NFFT_OK;
}

int nfft_batch_autotune(nfft_batch b, hipStream_t s)
{
    if (!b)
        return NFFT_ERR_ARG;
    if (!b->ws || !b->table_current)
        return NFFT_ERR_WORKSPACE;
    for (size_t i = 0; i < b->plans.size(); ++i)
        if (b->plans[i]->ws != b->plan_ws[i] || !b->plans[i]->nodes_set)
            return NFFT_ERR_STATE;
    // stand-in coefficient and value arrays (zeros), freed before returning
    const size_t cs = b->plans[0]->dbl ? 16 : 8;
    std::vector<size_t> off_c(b->plans.size()), off_v(b->plans.size());
    size_t total = 0;
    for (size_t i = 0; i < b->plans.size(); ++i) {
        int64_t K = 1;
        for (int t = 0; t < b->plans[i]->d; ++t)
            K *= b->plans[i]->N[t];
        off_c[i] = total;
        total = align_up(total + cs * (size_t)K);
        off_v[i] = total;
        total = align_up(total + cs * (size_t)b->plans[i]->M);
    }
    char *tmp = nullptr;
    hipError_t e = hipMalloc(&tmp, total);
    if (e != hipSuccess) {
        b->last_hip_error = e;
        return NFFT_ERR_HIP;
    }
    std::vector<const void *> cin(b->plans.size());
    std::vector<void *> cout(b->plans.size()), vout(b->plans.size());
    for (size_t i = 0; i < b->plans.size(); ++i) {
        cin[i] = tmp + off_c[i];
        cout[i] = tmp + off_c[i];
        vout[i] = tmp + off_v[i];
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = NFFT_OK;
    if ((e = hipMemsetAsync(tmp, 0, total, s)) != hipSuccess || (e = hipEventCreate(&e0)) != hipSuccess ||
        (e = hipEventCreate(&e1)) != hipSuccess) {
        b->last_hip_error = e;
        st = NFFT_ERR_HIP;
    }
    constexpr int kReps = 4;
    // mean time of one run of `fn` on the stream (one untimed run first), or -1 on error
    auto time_ms = [&](auto fn) -> double {
        if (fn() != NFFT_OK)
            return -1.0;
        if (hipEventRecord(e0, s) != hipSuccess)
            return -1.0;
        for (int r = 0; r < kReps; ++r)
            if (fn() != NFFT_OK)
                return -1.0;
        float ms = 0.f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            return -1.0;
        return ms / kReps;
    };
    std::map<std::string, std::vector<int>> cached;
    if (st == NFFT_OK && !b->cache.empty())
        cached = read_cache(b->cache);
    const int packs[] = {1, 2, 4, 8};
    const int ks_fft[] = {0, 1, 2, 4, 8};
    const int ks_win[] = {0, 1, 2, 4, 8, 16};
    for (size_t gi = 0; st == NFFT_OK && gi < b->groups.size(); ++gi) {
        Group &G = b->groups[gi];
        const BatchPtrs fwd_ptrs = make_ptrs(G, cin.data(), vout.data());
        const BatchPtrs adj_ptrs = make_ptrs(G, (const void *const *)vout.data(), cout.data());
        int best[NFFT_BATCH_NPARAMS];
        std::memcpy(best, G.params, sizeof(best));
        // FFT passes: packing x grid size, forward and adjoint
        for (int dir = 0; dir < 2 && st == NFFT_OK; ++dir) {
            double tbest = 1e30;
            for (int pk : packs) {
                int trial[NFFT_BATCH_NPARAMS];
                std::memcpy(trial, best, sizeof(trial));
                trial[dir == 0 ? kPackFwd : kPackAdj] = pk;
                std::memcpy(G.params, trial, sizeof(trial));
                build_group(b, G);
                if ((st = upload_group(b, G)) != NFFT_OK)
                    break;
                for (int k : ks_fft) {
                    G.params[dir == 0 ? kKFwd : kKAdj] = k;
                    const double ms = time_ms([&] { return run_fft(b, G, dir == 0 ? fwd_ptrs : adj_ptrs, dir == 0, s); });
                    if (ms < 0) {
                        st = NFFT_ERR_HIP;
                        break;
                    }
                    if (ms < tbest) {
                        tbest = ms;
                        best[dir == 0 ? kPackFwd : kPackAdj] = pk;
                        best[dir == 0 ? kKFwd : kKAdj] = k;
                    }
                }
                if (st != NFFT_OK)
                    break;
            }
        }
        if (st != NFFT_OK)
            break;
        std::memcpy(G.params, best, sizeof(best));
        build_group(b, G);
        if ((st = upload_group(b, G)) != NFFT_OK)
            break;
        // window kernels and fold: grid size
        struct Kind {
            Param q;
            int which;
        };
        for (Kind kd : {Kind{kKInterp, 0}, Kind{kKSpread, 1}, Kind{kKFold, 2}}) {
            double tbest = 1e30;
            for (int k : ks_win) {
                G.params[kd.q] = k;
                const double ms = time_ms([&] {
                    if (kd.which == 0)
                        return run_interp(b, G, fwd_ptrs, s);
                    if (kd.which == 1)
                        return run_spread(b, G, adj_ptrs, s);
                    return run_fold(b, G, s);
                });
                if (ms < 0) {
                    st = NFFT_ERR_HIP;
                    break;
                }
                if (ms < tbest) {
                    tbest = ms;
                    best[kd.q] = k;
                }
            }
            G.params[kd.q] = best[kd.q];
            if (st != NFFT_OK)
                break;
        }
        if (st != NFFT_OK)
            break;
        std::memcpy(G.params, best, sizeof(best));
        G.tuned = true;
        cached[G.key] = std::vector<int>(best, best + NFFT_BATCH_NPARAMS);
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (hipStreamSynchronize(s) != hipSuccess && st == NFFT_OK)
        st = NFFT_ERR_HIP;
    (void)hipFree(tmp);
    if (st != NFFT_OK)
        return st;
    if (!b->cache.empty() && !write_cache(b->cache, cached))
        return NFFT_ERR_ARG;
    return NFFT_OK;
}

int nfft_batch_destroy(nfft_batch b)
{
    if (!b)
        return NFFT_ERR_ARG;
    delete b;
    return NFFT_OK;
}

}  // extern "C"
