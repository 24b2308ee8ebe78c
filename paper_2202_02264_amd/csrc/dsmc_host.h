// Host-side pieces shared by the plan path (dsmc_api.cpp) and the serving
// engine (dsmc_server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "dsmc.h"
#include "dsmc_internal.h"
#include "dsmc_launch.h"

// Device-resident model (dsmc_model_create).
struct dsmc_model {
  void* dmem = nullptr;  // DevModel header followed by its arrays
  dsmc::DevModel* dev = nullptr;
  dsmc::DevModel hdr{};  // host copy of the header (device array pointers)
  int K = 0, dx = 0, dy = 0, obs_kind = 0, prop_kind = 0;
  void* pit_ws = nullptr;  // workspace of dsmc_model_gaussian_proposals
  size_t pit_bytes = 0;
};

namespace dsmc {

// Records a thread-local error message (dsmc_last_error) and returns `code`.
int fail(int code, const char* fmt, ...);

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return ::dsmc::fail(e_ == hipErrorOutOfMemory ? DSMC_ENOMEM : DSMC_EDEVICE,  \
                          "%s: %s", #expr, hipGetErrorString(e_));                 \
  } while (0)

// Rows-kernel tile: rows per lane, waves per workgroup, column splits.
struct TileChoice {
  int RPL, W, CS;
};

int padded_dx(int dx);
int pick_cs(int nodes, int N, int Nc, int rpl, int W);
TileChoice heuristic_tile(int nodes, int N, int Nc, bool split_ok);
void set_tile(LevelLaunch& L, TileChoice tc);
int check_output(const dsmc_output* o);

// Algorithm 6 for one series of K points whose combines get ids
// node_base + (0 .. K-2), ordered by level; `series` is its index in the
// series table and row_base the first time row.  Appends the combines to
// `nodes`, writes per-level offsets/counts (relative to node_base), the
// consumer of every single-point block (leaf_cons[t], t < K; -1 if none) and
// the id of the root combine (-1 when K == 1).
void build_series_schedule(int K, int series, int node_base, std::vector<NodeDesc>& nodes,
                           std::vector<int>& lvl_off, std::vector<int>& lvl_cnt,
                           std::vector<int32_t>& leaf_cons, int* root);

// Size of the per-combine / per-time-row device buffers of a pool.
struct PoolSizes {
  size_t per_row;   // bytes per time row (particles, weights, ancestry, per-combine data)
  size_t per_node;  // bytes per combine of one launch slice (chunk sums, row sums)
};
PoolSizes pool_sizes(int N, int DX, int dx_alloc, size_t rsz);

}  // namespace dsmc
