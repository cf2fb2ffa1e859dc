// bsde_internal.h -- library-internal declarations shared by the C ABI
// (bsde_host.cpp) and the request server (bsde_server.cpp).
#pragma once

#include "../../include/bsde.h"
#include "bsde_common.h"

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

struct bsde_problem_s {
    // parameters
    int d = 0, eta = 0, M = 0, N = 0, K_it = 0, precision = 0;
    double q = 1.0, omega = 0.0;
    bsde::PathParams base{};
    // sizes
    int n = 0, n_spatial = 0, p = 0, C = 0;
    // grid: kind, nodes, redraw flag and the iteration whose points are on
    // the device (with redraw)
    int grid_kind = 0, n_t = 0, n_x = 0, redraw = 0, pts_k = 0;
    int q10 = 10;                // index-set kernel: q in tenths (10 = total degree)
    std::vector<int> act;        // active multi-indices (hyperbolic set)
    std::vector<int8_t> nu;      // p x (d+1), kernel order
    std::vector<char> active;    // in the hyperbolic set
    std::vector<double> pts;     // n x (d+1)
    std::vector<double> lo, hi;
    // d x p sparse rows (column, value) of d/dx_j on the basis, columns ascending
    std::vector<std::vector<std::vector<std::pair<int, double>>>> Dx;
    int n_live = 0;              // entries of the packed channel table
    // device
    double *d_pts = nullptr, *d_W = nullptr, *d_vals = nullptr,
           *d_alpha = nullptr, *d_beta = nullptr, *d_g64 = nullptr,
           *d_partial = nullptr, *d_c = nullptr, *d_var = nullptr;
    float *d_g32 = nullptr;
    // the channel update as a sparse matrix over the packed table: entry e
    // is sum_k vals[k] alpha[cols[k]], k in rowptr[e] .. rowptr[e+1]-1
    int *d_rowptr = nullptr, *d_cols = nullptr;
    // d_pts, d_vals, d_alpha, d_g64, d_g32, d_rowptr, d_cols and d_ktab live in
    // this one allocation
    void *d_block = nullptr;
    // kernel operator of Section 3.2 (kop): bandwidth and the path kernel's
    // table of rows {z_0, .., z_d, y} (FP32 or FP64 as the paths); d_alpha
    // then holds the point values y (p = n)
    bool kop = false;
    void *d_ktab = nullptr;
    size_t partial_cap = 0;
    // state
    int k_done = 0;
    bool have_alpha = false;
    std::vector<double> alpha_hist; // (K_it + 1) x p, host mirror
    int groups = 0, ppl = 0;       // tiling (0 = automatic)
    double timings[5] = {0, 0, 0, 0, 0};
    int timing = 1; // event level of bsde_solve (bsde_set_timing)
};


namespace bsde {
// records msg as the thread's last error and returns s
bsde_status fail(bsde_status s, const std::string &msg);
// runs `steps` Picard iterations (steps_each[q] for problem q when given;
// at most the remaining ones) of every problem with the batched kernels;
// copies coefficient histories back when copy_back is set; the descriptor
// tables and tile counters go to workspace (device memory of
// workspace_bytes) when given, else to memory from the library's pool;
// ms (may be null) receives the GPU time; with parallel, launches of
// different kernel signatures in a step run on the library's side streams
// (parallel branches), else all on s; the persistent grids leave
// cu_reserve compute units' worth of workgroup slots free for other work
bsde_status run_batch(bsde_problem *probs, int count, hipStream_t s, int steps,
                      bool graph, bool copy_back, double *ms,
                      const int *steps_each = nullptr, void *workspace = nullptr,
                      size_t workspace_bytes = 0, bool parallel = true,
                      int cu_reserve = 0);
// copies the latest coefficients of a finished problem back to the host
bsde_status fetch_coefficients(bsde_problem h);
// device bytes a problem with these parameters allocates (pool size classes)
size_t problem_device_bytes(int d, const bsde_grid *grid, int M, int K_it);
} // namespace bsde
