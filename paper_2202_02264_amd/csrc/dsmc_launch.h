// Host-side launch interface between the plan code and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "dsmc_internal.h"

namespace dsmc {

// Optional per-launch HIP-event timing, grouped by kernel class
// (0 leaves, 1 prep, 2 rows, 3 sample, 4 gather, 5 output).
struct Timer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<int> cls;               // class of each recorded pair
  std::vector<hipEvent_t> beg, fin;   // recorded pairs
  hipEvent_t pending = nullptr;

  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void reset() {
    used = 0;
    cls.clear();
    beg.clear();
    fin.clear();
  }
  void begin(int c, hipStream_t st) {
    if (!on) return;
    pending = take();
    if (pending) hipEventRecord(pending, st);
    cls.push_back(c);
    beg.push_back(pending);
  }
  void end(int, hipStream_t st) {
    if (!on) return;
    hipEvent_t e = take();
    if (e) hipEventRecord(e, st);
    fin.push_back(e);
  }
  ~Timer() {
    for (auto e : pool) hipEventDestroy(e);
  }
};

struct LevelLaunch {
  bool fp64;
  int DX;
  int nodes;            // combines in this launch
  int N, Npad, Nc;      // particles, padded columns, chunks per row
  int RB, CS, KC;       // row blocks, column splits, chunks per split
  int totalK;
  const NodeDesc* d_nodes;
  const SeriesDesc* d_series;
  const void* leafX;
  const void* leafW;
  const int32_t* sigma;
  void* col;
  void* row;
  double* nscal;
  void* P;
};

struct LeafLaunch {
  bool fp64;
  int DX;
  int N, totalK;
  const SeriesDesc* d_series;
  const int32_t* d_series_of_t;
  void* leafX;
  void* leafW;
  double* leafL;
  int32_t* sigma;
};

int launch_leaves(const LeafLaunch& L, hipStream_t st, Timer* tm);
int launch_level(const LevelLaunch& L, hipStream_t st, Timer* tm);
void launch_gather(const NodeDesc* d_nodes, const SeriesDesc* d_series, int nodes,
                   int rows_per_node, int N, int32_t* sigma, hipStream_t st, Timer* tm);
void launch_output(const LeafLaunch& L, int B, int dx, hipStream_t st, Timer* tm);
void launch_clear_status(const SeriesDesc* d_series, int B, hipStream_t st);

}  // namespace dsmc
