// Host-side plan object behind the opaque nfft_plan handle.
#pragma once

#include <set>
#include <string>
#include <vector>

#include "../../include/nfft_mi355x.h"
#include "launch.hpp"

struct nfft_prof_pair {
    const char *name;
    hipEvent_t a, b;
};

struct nfft_plan_s {
    int d = 0, m = 0, WM = 0;
    nfft_dtype dtype = NFFT_C64;
    bool dbl = false;
    uint32_t flags = 0;
    int64_t N[nfft::kMaxDim] = {1, 1, 1};
    int64_t n[nfft::kMaxDim] = {1, 1, 1};
    int64_t M = 0;
    int64_t ngrid = 0;
    nfft::Geom geom;
    int chunk_cap = 0;
    int max_chunks = 0;
    size_t lds_window = 0;

    // FP64 deconvolution factors (centred index) and twiddles per dimension
    std::vector<double> wtab[nfft::kMaxDim];
    std::vector<double2> twd[nfft::kMaxDim];
    std::vector<float2> twf[nfft::kMaxDim];

    std::vector<nfft::FftPass> fwd_passes, adj_passes;

    // workspace layout (byte offsets)
    size_t off_w[nfft::kMaxDim] = {0, 0, 0}, off_tw[nfft::kMaxDim] = {0, 0, 0};
    size_t off_grid = 0, off_grid_adj = 0;
    size_t off_u[nfft::kMaxDim] = {0, 0, 0}, off_delta[nfft::kMaxDim] = {0, 0, 0};
    size_t off_perm = 0, off_key = 0, off_rank = 0;
    size_t off_bin_count = 0, off_bin_start = 0, off_bin_chunk = 0;
    size_t off_chunk_bin = 0, off_chunk_first = 0, off_chunk_len = 0;
    size_t off_counters = 0, off_xcopy = 0, off_scratch = 0, off_psi = 0;
    size_t off_lin[nfft::kMaxDim] = {0, 0, 0}, off_lin_d[nfft::kMaxDim] = {0, 0, 0};  // NFFT_PRE_LIN_PSI tables
    size_t off_spos = 0;  // only when 2-D spreading runs in registers (spos_used)
    bool spos_used = false;
    // owner-computes 3-D spreading (geom.own): tile lists, work items, partial-tile slots
    size_t off_tile_count = 0, off_tile_entry = 0, off_entries = 0, off_tile_item = 0, off_item_tile = 0;
    size_t off_item_lo = 0, off_item_hi = 0, off_own_scratch = 0, off_own_fs = 0;
    int own_max_items = 0;
    size_t off_tile_order = 0;
    std::vector<int32_t> tile_order;  // output tiles in Morton order (uploaded with the tables)
    int64_t own_max_entries = 0;
    size_t ws_bytes = 0;

    void *ws = nullptr;
    bool tables_on_device = false;
    bool nodes_set = false;
    bool grid_valid = false;
    hipError_t last_hip_error = hipSuccess;

    // kernel timing
    bool prof_on = false;
    hipEvent_t ev_open = nullptr;
    std::vector<hipEvent_t> ev_pool;
    std::vector<nfft_prof_pair> ev_pending;
    std::set<std::string> names;
    const char *intern(const std::string &s) { return names.insert(s).first->c_str(); }
};

// Device views of a plan with a workspace attached (shared with the batch code).
nfft::Nodes plan_node_view(nfft_plan_s *p);
nfft::FftPass plan_bind_pass(nfft_plan_s *p, const nfft::FftPass &tmpl, void *grid, const void *fin, void *fout);
// FFT pass `tmpl` with `factor` times as many lines per workgroup (factor 1: unchanged);
// false when the packing does not fit the pass.
bool plan_repack_pass(const nfft_plan_s *p, const nfft::FftPass &tmpl, int factor, nfft::FftPass &out);
