// HIP kernels of the dSMC combine tree for gfx950: the launch entry points,
// which dispatch on the padded state dimension to the instantiations of
// dsmc_kernels_dx*.hip (kernel templates in dsmc_kernels_impl.h), and the
// output kernels, which do not depend on it.
//
//   k_output   once per call: each output entry follows the ancestry from the
//              root combine down to its leaf (the gather of Algorithm 1, done
//              once instead of per level), and log L^N per series.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dsmc.h"
#include "dsmc_device.h"
#include "dsmc_launch.h"

namespace dsmc {

#define DSMC_DECLARE(DX, SUF)                                                    \
  int launch_level_dx##DX##SUF(const LevelLaunch& L, hipStream_t st, Timer* tm);  \
  void launch_leaves_dx##DX##SUF(const LeafLaunch& L, hipStream_t st, Timer* tm);
#define DSMC_DECLARE_DX(DX) DSMC_DECLARE(DX, _f32) DSMC_DECLARE(DX, _f64)
DSMC_DECLARE_DX(1)
DSMC_DECLARE_DX(2)
DSMC_DECLARE_DX(4)
DSMC_DECLARE_DX(8)
DSMC_DECLARE_DX(16)
DSMC_DECLARE_DX(32)

// =============================================================== output
// Output entry n of time t of a series: the particle idx of leaf t (trajectory
// value), and the per-leaf diagnostics when requested.
template <typename R>
__device__ __forceinline__ void emit_leaf(const SeriesDesc& sd, int t, int n, int idx, int totalK,
                                          int N, int dx, const R* __restrict__ leafX,
                                          const R* __restrict__ leafW,
                                          const double* __restrict__ leafL) {
  const int g = sd.base + t, K = sd.K;
  R* lw = (R*)sd.leaf_logw;
  // coordinate i of a leaf row lies totalK N elements after coordinate i - 1,
  // of an output row K N after; eight loads are issued before their stores
  const size_t ss = (size_t)totalK * N, ds = (size_t)K * N;
  auto copy = [&](R* dst, const R* src) __attribute__((always_inline)) {
    int i = 0;
    for (; i + 8 <= dx; i += 8) {
      R v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = src[(size_t)(i + j) * ss];
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[(size_t)(i + j) * ds] = v[j];
    }
    for (; i < dx; ++i) dst[(size_t)i * ds] = src[(size_t)i * ss];
  };
  copy((R*)sd.traj + (size_t)t * N + n, leafX + (size_t)g * N + idx);
  if (sd.leaf_x) copy((R*)sd.leaf_x + (size_t)t * N + n, leafX + (size_t)g * N + n);
  if (lw) lw[(size_t)t * N + n] = leafW[(size_t)g * N + n];
  if (sd.index) sd.index[(size_t)t * N + n] = idx;
  if (n == 0 && sd.leaf_logL) sd.leaf_logL[t] = leafL[g];
}

// One workgroup per time row: each output entry follows the ancestry from
// the root combine down to its leaf.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_output_rows(
    const SeriesDesc* __restrict__ series, const int32_t* __restrict__ series_of_t,
    const NodeDesc* __restrict__ nodes, int row0, int totalK, int N, int dx,
    const R* __restrict__ leafX, const R* __restrict__ leafW, const double* __restrict__ leafL) {
  const int g = row0 + blockIdx.x;
  const SeriesDesc& sd = series[series_of_t[g]];
  const int t = g - sd.base;
  for (int n = threadIdx.x; n < N; n += kBlock) {
    int idx = n;
    int cur = sd.root;
    // a tree over K <= 2^31 points has at most 31 levels
    for (int depth = 0; cur >= 0 && depth < 32; ++depth) {
      const NodeDesc nd = nodes[cur];
      const bool right = t >= nd.c;
      idx = sd.anc[(size_t)(nd.c - 1) * 2 * N + (right ? N : 0) + idx];
      cur = right ? nd.rchild : nd.lchild;
    }
    emit_leaf<R>(sd, t, n, idx, totalK, N, dx, leafX, leafW, leafL);
  }
}

// The same output level by level from the roots down, for schedules whose
// combines are numbered by level: map[node][n] is the draw index that output
// entry n takes at that combine (n at a series' root); a combine hands its
// children the indices its draw took, and writes the entries of a child
// block that is a single leaf.  One gather per entry and level instead of
// one per entry and tree depth at every time.  Workgroups are dealt to the
// eight XCDs in turn, so workgroup b is renumbered to give each XCD a
// contiguous range of combines: the leaf rows a combine gathers from are
// then fetched into one XCD's L2 only.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_output_down(
    const SeriesDesc* __restrict__ series, const NodeDesc* __restrict__ nodes, int node0,
    int per_node, int totalK, int N, int dx, const R* __restrict__ leafX,
    const R* __restrict__ leafW, const double* __restrict__ leafL, int32_t* __restrict__ map) {
  const unsigned q = gridDim.x / 8, rem = gridDim.x % 8, x = blockIdx.x % 8;
  const unsigned v = x * q + min(x, rem) + blockIdx.x / 8;
  const int node = node0 + (int)(v / per_node);
  const int n = (int)(v % per_node) * kBlock + threadIdx.x;
  if (n >= N) return;
  const NodeDesc nd = nodes[node];
  const SeriesDesc& sd = series[nd.series];
  const int m = (node == sd.root) ? n : map[(size_t)node * N + n];
  const int32_t* anc = sd.anc + (size_t)(nd.c - 1) * 2 * N;
  const int l = anc[m], r = anc[N + m];
  if (nd.lchild >= 0) map[(size_t)nd.lchild * N + n] = l;
  else emit_leaf<R>(sd, nd.a, n, l, totalK, N, dx, leafX, leafW, leafL);
  if (nd.rchild >= 0) map[(size_t)nd.rchild * N + n] = r;
  else emit_leaf<R>(sd, nd.c, n, r, totalK, N, dx, leafX, leafW, leafL);
}

// One workgroup per series: log Z = sum_t log L_t + sum_c Z_c (fixed
// reduction order), and the output log-weights.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_output_series(const SeriesDesc* __restrict__ series,
                                                          int s0, int N, int totalK, int dx,
                                                          int single_leaves,
                                                          const R* __restrict__ leafX,
                                                          const R* __restrict__ leafW,
                                                          const double* __restrict__ leafL) {
  __shared__ double red[kMaxWaves];
  const SeriesDesc& sd = series[s0 + blockIdx.x];
  const int K = sd.K;
  if (single_leaves && K == 1)  // no combine: the leaf itself (after k_output_down)
    for (int n = threadIdx.x; n < N; n += kBlock)
      emit_leaf<R>(sd, 0, n, n, totalK, N, dx, leafX, leafW, leafL);
  double s = 0.0;
  for (int t = threadIdx.x; t < K; t += kBlock) s += leafL[sd.base + t];
  for (int c = threadIdx.x; c < K - 1; c += kBlock) s += sd.zinc[c];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *sd.log_Z = s;
  if (sd.logw) {
    R* lw = (R*)sd.logw;
    const R uni = (R)(-log((double)N));
    for (int n = threadIdx.x; n < N; n += kBlock)
      lw[n] = (K == 1) ? leafW[(size_t)sd.base * N + n] : uni;
  }
}

__global__ void k_clear_status(const SeriesDesc* __restrict__ series, int s0, int B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) *series[s0 + i].status = 0;
}

// ============================================================ launchers
int launch_level(const LevelLaunch& L, hipStream_t st, Timer* tm) {
  switch (L.DX) {
    case 1: return L.fp64 ? launch_level_dx1_f64(L, st, tm) : launch_level_dx1_f32(L, st, tm);
    case 2: return L.fp64 ? launch_level_dx2_f64(L, st, tm) : launch_level_dx2_f32(L, st, tm);
    case 4: return L.fp64 ? launch_level_dx4_f64(L, st, tm) : launch_level_dx4_f32(L, st, tm);
    case 8: return L.fp64 ? launch_level_dx8_f64(L, st, tm) : launch_level_dx8_f32(L, st, tm);
    case 16: return L.fp64 ? launch_level_dx16_f64(L, st, tm) : launch_level_dx16_f32(L, st, tm);
    case 32: return L.fp64 ? launch_level_dx32_f64(L, st, tm) : launch_level_dx32_f32(L, st, tm);
  }
  return -1;
}

int launch_leaves(const LeafLaunch& L, hipStream_t st, Timer* tm) {
  switch (L.DX) {
    case 1: L.fp64 ? launch_leaves_dx1_f64(L, st, tm) : launch_leaves_dx1_f32(L, st, tm); return 0;
    case 2: L.fp64 ? launch_leaves_dx2_f64(L, st, tm) : launch_leaves_dx2_f32(L, st, tm); return 0;
    case 4: L.fp64 ? launch_leaves_dx4_f64(L, st, tm) : launch_leaves_dx4_f32(L, st, tm); return 0;
    case 8: L.fp64 ? launch_leaves_dx8_f64(L, st, tm) : launch_leaves_dx8_f32(L, st, tm); return 0;
    case 16: L.fp64 ? launch_leaves_dx16_f64(L, st, tm) : launch_leaves_dx16_f32(L, st, tm); return 0;
    case 32: L.fp64 ? launch_leaves_dx32_f64(L, st, tm) : launch_leaves_dx32_f32(L, st, tm); return 0;
  }
  return -1;
}

// Leaf records (layout at leafrec_stride) of one model: one workgroup per time
// t, and workgroup K for the time-invariant matrices.
__global__ __launch_bounds__(kBlock) void k_leaf_records(const DevModel* __restrict__ Mp,
                                                         double* __restrict__ rec, int DX) {
  const DevModel& M = *Mp;
  const int K = M.K, dx = M.dx, dy = M.dy, t = blockIdx.x;
  const int S = leafrec_stride(DX);
  const bool lg_obs = M.obs_kind == 0 && dy <= DX;
  if (t == K) {
    double* inv = rec + (size_t)K * S;
    for (int e = threadIdx.x; e < DX * DX; e += blockDim.x) {
      const int i = e / DX, j = e - (e / DX) * DX;
      const bool in = i < dx && j < dx;
      inv[e] = (in && j <= i) ? M.Wcol[i * dx + j] : 0.0;
      inv[DX * DX + e] = in ? M.Wrow[i * dx + j] : 0.0;
      inv[2 * DX * DX + e] = (lg_obs && i < dy && j < dx) ? M.H[i * dx + j] : 0.0;
    }
    return;
  }
  double* r = rec + (size_t)t * S;
  const double* qc = M.q_chol + (size_t)t * dx * dx;
  const double* qi = M.q_inv + (size_t)t * dx * dx;
  const double* qm = M.q_mean + (size_t)t * dx;
  for (int e = threadIdx.x; e < DX * DX; e += blockDim.x) {
    const int i = e / DX, j = e - (e / DX) * DX;
    const bool in = i < dx && j <= i;
    r[e] = in ? qc[i * dx + j] : 0.0;
    r[DX * DX + e] = in ? qi[i * dx + j] : 0.0;
  }
  for (int i = threadIdx.x; i < S - 2 * DX * DX; i += blockDim.x) {
    double v = 0.0;
    if (i < DX) {  // q_mean[t]
      v = i < dx ? qm[i] : 0.0;
    } else if (i < 2 * DX) {  // row offset of boundary t + 1
      const int k = i - DX;
      if (k < dx && t + 1 < K) {
        v = M.wcol_off[k];
        for (int j = 0; j < dx; ++j)
          v += M.Wrow[k * dx + j] * qm[j] - M.Wcol[k * dx + j] * qm[dx + j];
      }
    } else if (i < 3 * DX) {  // whitened y_t - H q_mean[t]
      const int k = i - 2 * DX;
      if (lg_obs && k < dy) {
        v = M.y[(size_t)t * dy + k];
        for (int j = 0; j < dx; ++j) v -= M.H[k * dx + j] * qm[j];
      }
    }
    r[2 * DX * DX + i] = v;
  }
}

void launch_leaf_records(const DevModel* dev, double* rec, int K, int DX, hipStream_t st) {
  k_leaf_records<<<K + 1, kBlock, 0, st>>>(dev, rec, DX);
}

void launch_clear_status(const SeriesDesc* d_series, int s0, int B, hipStream_t st) {
  k_clear_status<<<(B + kBlock - 1) / kBlock, kBlock, 0, st>>>(d_series, s0, B);
}

template <typename R>
static void launch_output_t(const LeafLaunch& L, int s0, int B, int dx, hipStream_t st, Timer* tm) {
  tm->begin(3, st);
  k_output_rows<R><<<L.rows, kBlock, 0, st>>>(L.d_series, L.d_series_of_t, L.d_nodes, L.row0,
                                              L.totalK, L.N, dx, (const R*)L.leafX,
                                              (const R*)L.leafW, L.leafL);
  k_output_series<R><<<B, kBlock, 0, st>>>(L.d_series, s0, L.N, L.totalK, dx, 0,
                                           (const R*)L.leafX, (const R*)L.leafW, L.leafL);
  tm->end(3, st);
}

void launch_output(const LeafLaunch& L, int s0, int B, int dx, hipStream_t st, Timer* tm) {
  if (L.fp64) launch_output_t<double>(L, s0, B, dx, st, tm);
  else launch_output_t<float>(L, s0, B, dx, st, tm);
}

template <typename R>
static void launch_output_levels_t(const LeafLaunch& L, const int* level_off, const int* level_cnt,
                                   int levels, int32_t* map, int B, int dx, hipStream_t st,
                                   Timer* tm) {
  tm->begin(3, st);
  const int per_node = (L.N + kBlock - 1) / kBlock;
  for (int l = levels - 1; l >= 0; --l)
    if (level_cnt[l] > 0)
      k_output_down<R><<<(unsigned)level_cnt[l] * per_node, kBlock, 0, st>>>(
          L.d_series, L.d_nodes, level_off[l], per_node, L.totalK, L.N, dx, (const R*)L.leafX,
          (const R*)L.leafW, L.leafL, map);
  k_output_series<R><<<B, kBlock, 0, st>>>(L.d_series, 0, L.N, L.totalK, dx, 1,
                                           (const R*)L.leafX, (const R*)L.leafW, L.leafL);
  tm->end(3, st);
}

void launch_output_levels(const LeafLaunch& L, const int* level_off, const int* level_cnt,
                          int levels, int32_t* map, int B, int dx, hipStream_t st, Timer* tm) {
  if (L.fp64) launch_output_levels_t<double>(L, level_off, level_cnt, levels, map, B, dx, st, tm);
  else launch_output_levels_t<float>(L, level_off, level_cnt, levels, map, B, dx, st, tm);
}

}  // namespace dsmc
