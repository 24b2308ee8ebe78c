// Host-side launch interface between the plan code and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "dsmc_internal.h"

namespace dsmc {

// Optional per-launch HIP-event timing, grouped by kernel class
// (0 leaves, 1 rows, 2 sample, 3 output).
struct Timer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<int> cls;               // class of each recorded pair
  std::vector<hipEvent_t> beg, fin;   // recorded pairs

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
    hipEvent_t e = take();
    if (e) (void)hipEventRecord(e, st);
    cls.push_back(c);
    beg.push_back(e);
  }
  void end(int, hipStream_t st) {
    if (!on) return;
    hipEvent_t e = take();
    if (e) (void)hipEventRecord(e, st);
    fin.push_back(e);
  }
  ~Timer() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct LevelLaunch {
  bool fp64;
  bool bf16;            // pair rows on bf16 matrix cores (DX 16 or 32, fp32 otherwise)
  int DX;
  const int32_t* node_list;  // device list of combine ids, or null: ids node0 .. node0+nodes-1
  int node0;            // id of the first combine of this launch (without a list)
  int nodes;            // combines in this launch
  int N, Npad, Nc, NcP; // particles, padded columns, chunks per row, chunk-row stride
  int RPL, W, RB;       // rows kernel: rows per lane, waves per workgroup, row blocks per combine
  int CS, KC;           // rows kernel: column splits per combine, chunks per split
  int DS;               // sample kernel: workgroups per combine
  int SB;               // sample kernel: threads per workgroup
  int lazy;             // 0 exact draws; 1 Metropolis-Hastings, 2 rejection (no pair-row pass)
  int lazy_param;       // MH steps, or the rejection proposal cap
  int totalK;
  const NodeDesc* d_nodes;
  const SeriesDesc* d_series;
  const void* leafX;
  const double* bmerged;
  void* P;
  void* Pr;             // chunk sums of rescued rows (same layout as P)
  double* Rsum;
  float* Rshift;        // per-row shifts of the row sums (DX >= 8), like Rsum
  double* Gs;           // per row of the slice: sums of its groups of kGroup chunks
                        // (group_stride(NcP) per row), written with column splits
  bool force_rescue;    // testing aid: every row takes the rescue path
  unsigned long long* rescue_count;  // rescued rows are added here when non-null
  NodeBufs nb;
};

struct LeafLaunch {
  bool fp64;
  int DX;
  int N, Npad, totalK; // totalK: length (stride) of the packed time axis
  int row0, rows;       // time rows [row0, row0 + rows) of this launch
  const SeriesDesc* d_series;
  const int32_t* d_series_of_t;
  const int32_t* d_leaf_cons;
  const NodeDesc* d_nodes;
  void* leafX;
  void* leafW;
  double* leafL;
  double* bmerged;
  NodeBufs nb;
};

// Row stride of the chunk-group sums (NcP / kGroup groups, at least 4, even).
inline int group_stride(int NcP) {
  const int g = NcP / kGroup;
  return g <= 4 ? 4 : (g + 1) / 2 * 2;
}

// Threads per workgroup of the sampling kernel and of the small-d_x leaf kernel
// for N particles: one wave for N <= 256, two for N <= 512, else kBlock.  A
// function of N alone, so that every path (plan, batch, server, static) sums
// the fp64 CDFs and the leaf normalisers in the same order.
inline int sample_block(int N) { return N <= 256 ? 64 : (N <= 512 ? 128 : kBlock); }
inline int leaf_block(int N) { return sample_block(N); }

// LDS of the sampling kernel before its optional column data (layout in
// k_sample): the fp64 row CDF and rescue chunk sums, the fp32 row shifts (with
// row shifts), the row weights, two row bit masks and the rescue list.
inline size_t sample_lds(int Npad, int Nc, size_t threads, bool row_shift, size_t real) {
  return (size_t)Npad * 8 + (size_t)Nc * 8 + (row_shift ? (size_t)Npad * 4 : 0) +
         (size_t)Npad * real + 2 * (size_t)(Npad / 32) * 4 + threads * 4;
}

// Shape of a level's sampling launch (needs L.N, L.DX, L.nodes and L.lazy):
// sample_block(N) threads per workgroup, and several workgroups per combine
// (each computes the combine's CDF and takes a share of its draws) when a level
// has few combines.  Where a draw is dear against that repeated CDF pass
// (N <= 1024, or padded d_x >= 8 with its d_x-dimensional chunk recompute),
// exact draws aim at about 1024 workgroups, four per compute unit, to hide
// their dependent loads: one workgroup per combine at 256 combines (N = 1024)
// took 42 us, against 25 us for 128 combines in 512 workgroups.  Elsewhere
// (exact draws at N = 4096, d_x = 1: 8 % slower with the wider split; the
// lazy chains) the target is 512.  Results do not depend on the split.
inline void set_sample_shape(LevelLaunch& L) {
  const int nodes = L.nodes < 1 ? 1 : L.nodes;
  L.SB = sample_block(L.N);
  const bool wide = !L.lazy && (L.N <= 1024 || L.DX >= 8);
  const int target = wide ? 1024 : 512;      // workgroups per launch
  const int one_each = wide ? 1024 : 256;    // combines from which one workgroup each
  const int ds_max = (L.N + 127) / 128 < 1 ? 1 : (L.N + 127) / 128;
  const int spread = (target + nodes - 1) / nodes;
  L.DS = nodes >= one_each ? 1 : (ds_max < spread ? ds_max : spread);
}

int launch_leaves(const LeafLaunch& L, hipStream_t st, Timer* tm);
int launch_level(const LevelLaunch& L, hipStream_t st, Timer* tm);
void launch_output(const LeafLaunch& L, int s0, int B, int dx, hipStream_t st, Timer* tm);
// The output by tree levels from the roots down (schedules whose combines are
// numbered level by level, level l at [level_off[l], + level_cnt[l])); map is
// N int32 per combine of scratch, which the levels' sampling no longer needs.
void launch_output_levels(const LeafLaunch& L, const int* level_off, const int* level_cnt,
                          int levels, int32_t* map, int B, int dx, hipStream_t st, Timer* tm);
void launch_clear_status(const SeriesDesc* d_series, int s0, int B, hipStream_t st);
// Fills a model's leaf records (rec = its leafrec array, padded dimension DX).
void launch_leaf_records(const DevModel* dev, double* rec, int K, int DX, hipStream_t st);

}  // namespace dsmc
