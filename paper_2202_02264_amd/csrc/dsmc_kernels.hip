// HIP kernels of the dSMC combine tree for gfx950 (wave64, fp32/fp64 VALU).
//
// Per level of the tree (Algorithm 5) four kernels run over all combine
// nodes of the level (of every series in the launch):
//   k_prep    per node: whitened coordinates and log-weights of the two
//             boundary particle sets (O(N d_x^2)).
//   k_rows    the N x N pair-weight matrix of every node, never stored: one
//             lane per row, columns streamed through scalar registers, the
//             exp2 of each entry summed per chunk of 32 columns.  Output: the
//             chunk sums P[node][m][k].
//   k_sample  per node: row sums -> row marginal CDF (fp64 scan) -> left index
//             by binary search; right index by a scan over that row's chunk
//             sums and a recomputation of one 32-column chunk (Algorithm 1's
//             multinomial resampling, in two stages).
//   k_gather  in-place gather of the composed ancestry sigma[t][n] (leaf index
//             of trajectory n at time t) for every time row of the merged blocks.
// Leaves (Algorithm 2) and the output pass run once per call.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dsmc_device.h"
#include "dsmc_launch.h"

namespace dsmc {

// ================================================================ leaves
// One workgroup per time row g of the packed time axis: draw X_g^n ~ q_t from
// the Philox normals, store it (rounded to R), weight the rounded particle
// (Algorithm 2 with the t = 0 weight of Proposition 2.2), normalise.
template <typename R, int DX>
__global__ __launch_bounds__(kBlock) void k_leaves(const SeriesDesc* __restrict__ series,
                                                   const int32_t* __restrict__ series_of_t,
                                                   int totalK, int N, R* __restrict__ leafX,
                                                   R* __restrict__ leafW,
                                                   double* __restrict__ leafL,
                                                   int32_t* __restrict__ sigma) {
  extern __shared__ double ell[];  // [N]
  __shared__ double red[kBlock / 64];
  __shared__ int redi[kBlock / 64];
  const int g = blockIdx.x;
  const SeriesDesc& sd = series[series_of_t[g]];
  const DevModel& M = *sd.model;
  const int t = g - sd.base;
  const int dx = M.dx;
  int bad = 0;
  for (int n = threadIdx.x; n < N; n += kBlock) {
    double z[DX + 3];
#pragma unroll
    for (int j = 0; j < (DX + 3) / 4; ++j) {
      const Words4 w = philox4x64_10((uint64_t)n, (uint64_t)t, kPurposeLeaf, (uint64_t)j,
                                     sd.seed, kKey1);
      box_muller(w.w0, w.w1, z[4 * j], z[4 * j + 1]);
      box_muller(w.w2, w.w3, z[4 * j + 2], z[4 * j + 3]);
    }
    const double* qm = M.q_mean + (size_t)t * dx;
    const double* qc = M.q_chol + (size_t)t * dx * dx;
    double x[DX];
#pragma unroll
    for (int i = 0; i < DX; ++i) {
      double xi = 0.0;
      if (i < dx) {
        xi = qm[i];
#pragma unroll
        for (int j = 0; j <= i; ++j) xi += qc[i * dx + j] * z[j];
        const R xr = (R)xi;
        leafX[((size_t)i * totalK + g) * N + n] = xr;
        xi = (double)xr;  // weights are those of the stored particle
      }
      x[i] = xi;
    }
    double l;
    if (t == 0) {
      l = log_potential<DX>(M, 0, x) + log_prior<DX>(M, x) - log_proposal<DX>(M, 0, x);
    } else if (M.weighting == 0) {
      l = log_potential<DX>(M, t, x);
    } else {
      l = 0.0;
    }
    if (isnan(l)) bad = kFlagNumeric;
    ell[n] = l;
    sigma[(size_t)g * N + n] = n;
  }
  __syncthreads();
  double mx = -INFINITY;
  for (int n = threadIdx.x; n < N; n += kBlock) mx = fmax(mx, ell[n]);
  mx = block_max(mx, red);
  double s = 0.0;
  if (mx > -INFINITY)
    for (int n = threadIdx.x; n < N; n += kBlock) s += exp(ell[n] - mx);
  s = block_sum(s, red);
  const double lse = mx + log(s);
  const bool degenerate = !(mx > -INFINITY);
  for (int n = threadIdx.x; n < N; n += kBlock)
    leafW[(size_t)g * N + n] = degenerate ? (R)(-log((double)N)) : (R)(ell[n] - lse);
  bad = block_or_i(bad, redi);
  if (threadIdx.x == 0) {
    leafL[g] = degenerate ? -INFINITY : lse - log((double)N);
    const int flags = bad | (degenerate ? kFlagDegenerate : 0);
    if (flags) atomicOr(sd.status, flags);
  }
}

// ================================================================= prep
// One workgroup per node.  Column data (right block, time c):
//   u_n   = Wcol (x_R[n] - q_mean[c])                        (DX values)
//   beta_n = log2e (b_n - B*),  b_n = w_R[n] - log q_c(x_R[n]) [+ log h_c(x_R[n])]
// Row data (left block, time c-1):
//   v_m   = Wrow x_L[m] + wcol_off - Wcol q_mean[c]
// so that ||u_n - v_m||^2 = (log2 e / 2) ||Q^{-1/2}(x_R - F x_L - f)||^2 and
// exp2(beta_n - ||u_n - v_m||^2) = exp(b_n - B* + log p(x_R|x_L) - trans_lognorm).
// Centering both sets on the proposal mean keeps the fp32 coordinates small.
// Scalars: nscal[node] = {A* = max_m a_m, B*, trans_lognorm, 0}.
template <typename R, int DX>
__global__ __launch_bounds__(kBlock) void k_prep(const NodeDesc* __restrict__ nodes,
                                                 const SeriesDesc* __restrict__ series,
                                                 int totalK, int N, int Npad,
                                                 const R* __restrict__ leafX,
                                                 const R* __restrict__ leafW,
                                                 const int32_t* __restrict__ sigma,
                                                 R* __restrict__ col, R* __restrict__ row,
                                                 double* __restrict__ nscal) {
  extern __shared__ double bsh[];  // [N]
  __shared__ double red[kBlock / 64];
  __shared__ int redi[kBlock / 64];
  const NodeDesc nd = nodes[blockIdx.x];
  const SeriesDesc& sd = series[nd.series];
  const DevModel& M = *sd.model;
  const int c = nd.c, dx = M.dx;
  const bool left_leaf = (c - nd.a) == 1, right_leaf = (nd.b - c) == 1;
  const int gL = sd.base + c - 1, gR = sd.base + c;
  const double logN = log((double)N);
  R* colp = col + (size_t)blockIdx.x * Npad * (DX + 1);
  R* rowp = row + (size_t)blockIdx.x * Npad * DX;
  const double* qmc = M.q_mean + (size_t)c * dx;
  int bad = 0;
  // centre: Wcol q_mean[c] (each side subtracts it)
  double cen[DX];
#pragma unroll
  for (int i = 0; i < DX; ++i) {
    double s = 0.0;
    if (i < dx)
      for (int j = 0; j < dx; ++j) s += M.Wcol[i * dx + j] * qmc[j];
    cen[i] = s;
  }
  double bmax = -INFINITY;
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const int src = sigma[(size_t)gR * N + n];
    double x[DX];
#pragma unroll
    for (int i = 0; i < DX; ++i)
      x[i] = (i < dx) ? (double)leafX[((size_t)i * totalK + gR) * N + src] : 0.0;
    double b = (right_leaf ? (double)leafW[(size_t)gR * N + src] : -logN) -
               log_proposal<DX>(M, c, x);
    if (M.weighting == 1) b += log_potential<DX>(M, c, x);
    if (isnan(b)) bad = kFlagNumeric;
    bsh[n] = b;
    bmax = fmax(bmax, b);
#pragma unroll
    for (int i = 0; i < DX; ++i) {
      double u = 0.0;
      if (i < dx) {
        for (int j = 0; j < dx; ++j) u += M.Wcol[i * dx + j] * (x[j] - qmc[j]);
      }
      colp[(size_t)n * (DX + 1) + i] = (R)u;
    }
  }
  for (int n = N + threadIdx.x; n < Npad; n += kBlock) {
#pragma unroll
    for (int i = 0; i < DX; ++i) colp[(size_t)n * (DX + 1) + i] = (R)0;
    colp[(size_t)n * (DX + 1) + DX] = (R)(-INFINITY);
  }
  double amax = -INFINITY;
  for (int m = threadIdx.x; m < N; m += kBlock) {
    const int src = sigma[(size_t)gL * N + m];
    double x[DX];
#pragma unroll
    for (int i = 0; i < DX; ++i)
      x[i] = (i < dx) ? (double)leafX[((size_t)i * totalK + gL) * N + src] : 0.0;
    const double a = left_leaf ? (double)leafW[(size_t)gL * N + src] : -logN;
    amax = fmax(amax, a);
#pragma unroll
    for (int i = 0; i < DX; ++i) {
      double v = 0.0;
      if (i < dx) {
        v = M.wcol_off[i] - cen[i];
        for (int j = 0; j < dx; ++j) v += M.Wrow[i * dx + j] * x[j];
      }
      rowp[(size_t)m * DX + i] = (R)v;
    }
  }
  bmax = block_max(bmax, red);  // contains a __syncthreads: bsh is complete
  amax = block_max(amax, red);
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const double beta = (bmax > -INFINITY) ? (bsh[n] - bmax) * kLog2e : -INFINITY;
    colp[(size_t)n * (DX + 1) + DX] = (R)beta;
  }
  bad = block_or_i(bad, redi);
  if (threadIdx.x == 0) {
    double* ns = nscal + (size_t)blockIdx.x * 4;
    ns[0] = amax;
    ns[1] = bmax;
    ns[2] = M.trans_lognorm;
    ns[3] = 0.0;
    if (bad) atomicOr(sd.status, bad);
  }
}

// ================================================================= rows
// Tile = (node, 256-row block, range of KC column chunks).  Lane m of the
// workgroup owns row m; all lanes walk the same columns, whose (u, beta) are
// wave-uniform and so are read into scalar registers.  Per pair:
// DX x (sub, fma) + exp2 + add.
template <typename R, int DX>
__global__ __launch_bounds__(kBlock) void k_rows(const R* __restrict__ col,
                                                 const R* __restrict__ row,
                                                 R* __restrict__ P, int N, int Npad, int Nc,
                                                 int RB, int CS, int KC) {
  const int tiles = RB * CS;
  const int node = blockIdx.x / tiles;
  const int tile = blockIdx.x - node * tiles;
  const int rb = tile / CS, cs = tile - rb * CS;
  const int m = rb * kBlock + threadIdx.x;
  const R* __restrict__ colp = col + (size_t)node * Npad * (DX + 1);
  R v[DX];
  const int mm = m < N ? m : N - 1;
#pragma unroll
  for (int i = 0; i < DX; ++i) v[i] = row[((size_t)node * Npad + mm) * DX + i];
  const int k0 = cs * KC;
  const int k1 = min(Nc, k0 + KC);
  R* __restrict__ Pm = P + ((size_t)node * N + mm) * Nc;
  for (int k = k0; k < k1; ++k) {
    const R* __restrict__ cp = colp + (size_t)k * kChunk * (DX + 1);
    R acc = (R)0;
#pragma unroll
    for (int jj = 0; jj < kChunk; ++jj) {
      R u[DX];
#pragma unroll
      for (int i = 0; i < DX; ++i) u[i] = cp[jj * (DX + 1) + i];
      acc += Real<R>::exp2(pair_log2w<R, DX>(u, cp[jj * (DX + 1) + DX], v));
    }
    if (m < N) Pm[k] = acc;
  }
}

// =============================================================== sample
// One workgroup per node (Algorithm 1: normalise, draw N index pairs).
//   R_m  = sum_k P[m][k]                         (fp64, k ascending)
//   w_m  = exp(a_m - A*) R_m,   C_m = sum_{i<=m} w_i   (fp64 scan)
//   Z_c  = A* + B* + trans_lognorm + log C_{N-1}
//   l_n  = first m with C_m > u1 C_{N-1}
//   r_n  = first j with  cumulative row-l weight > u2 R_l, found by a scan
//          over the chunk sums of row l and one recomputed chunk.
// Rows whose R_m underflows fp32 range (< kTiny) are recomputed with their
// exact maximum as shift and drawn from by a full-row scan.
template <typename R, int DX>
__global__ __launch_bounds__(kBlock) void k_sample(
    const NodeDesc* __restrict__ nodes, const SeriesDesc* __restrict__ series, int totalK,
    int N, int Npad, int Nc, const R* __restrict__ leafW, const int32_t* __restrict__ sigma,
    const R* __restrict__ col, const R* __restrict__ row, const R* __restrict__ P,
    const double* __restrict__ nscal) {
  extern __shared__ double smem[];
  double* cdf = smem;                          // [Npad]
  double* rs = smem + Npad;                    // [Npad]
  float* shift = (float*)(smem + 2 * Npad);    // [Npad]
  __shared__ double red[kBlock / 64];
  __shared__ int redi[kBlock / 64];
  const int node = blockIdx.x;
  const NodeDesc nd = nodes[node];
  const SeriesDesc& sd = series[nd.series];
  const int c = nd.c;
  const bool left_leaf = (c - nd.a) == 1;
  const int gL = sd.base + c - 1;
  const double logN = log((double)N);
  const double* ns = nscal + (size_t)node * 4;
  const double Astar = ns[0], Bstar = ns[1], c0 = ns[2];
  const R* __restrict__ colp = col + (size_t)node * Npad * (DX + 1);
  const R* __restrict__ rowp = row + (size_t)node * Npad * DX;
  const R* __restrict__ Pn = P + (size_t)node * N * Nc;

  // ---- row sums and log row weights (thread owns a contiguous segment of rows)
  //   rho_m = a_m - A* + shift_m ln 2 + ln R_m;  w_m = exp(rho_m - G), G = max rho
  const int per = (N + kBlock - 1) / kBlock;
  const int m0 = threadIdx.x * per, m1 = min(N, m0 + per);
  double gmax = -INFINITY;
  bool row_nan = false;
  for (int m = m0; m < m1; ++m) {
    double Rm = 0.0;
    const R* Pm = Pn + (size_t)m * Nc;
    for (int k = 0; k < Nc; ++k) Rm += (double)Pm[k];
    float sh = 0.0f;
    if (!(Rm >= Real<R>::kTiny) && !isnan(Rm)) {
      // underflow rescue: exact row maximum as shift, full-row fp64 sum
      R v[DX];
#pragma unroll
      for (int i = 0; i < DX; ++i) v[i] = rowp[(size_t)m * DX + i];
      R smax = (R)(-INFINITY);
      for (int j = 0; j < N; ++j) {
        R u[DX];
#pragma unroll
        for (int i = 0; i < DX; ++i) u[i] = colp[(size_t)j * (DX + 1) + i];
        smax = fmax(smax, pair_log2w<R, DX>(u, colp[(size_t)j * (DX + 1) + DX], v));
      }
      if (smax > (R)(-INFINITY)) {
        Rm = 0.0;
        for (int j = 0; j < N; ++j) {
          R u[DX];
#pragma unroll
          for (int i = 0; i < DX; ++i) u[i] = colp[(size_t)j * (DX + 1) + i];
          Rm += (double)Real<R>::exp2(pair_log2w<R, DX>(u, colp[(size_t)j * (DX + 1) + DX], v) -
                                      smax);
        }
        sh = (float)smax;  // < 0 since the row sum was tiny
      } else {
        Rm = 0.0;
      }
    }
    rs[m] = Rm;
    shift[m] = sh;
    const double a = left_leaf ? (double)leafW[(size_t)gL * N + sigma[(size_t)gL * N + m]] : -logN;
    double rho = -INFINITY;
    if (Astar > -INFINITY && Rm > 0.0) rho = a - Astar + (double)sh * kLn2 + log(Rm);
    if (isnan(Rm) || isnan(a)) row_nan = true;
    cdf[m] = rho;  // log row weight for now
    gmax = fmax(gmax, rho);
  }
  gmax = block_max(gmax, red);
  double seg = 0.0;
  int lastpos = -1;
  for (int m = m0; m < m1; ++m) {
    const double w = (gmax > -INFINITY) ? exp(cdf[m] - gmax) : 0.0;
    if (w > 0.0) lastpos = m;
    seg += w;
    cdf[m] = seg;  // segment-local inclusive prefix for now
  }
  // ---- workgroup exclusive scan of the segment totals
  {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double incl = seg;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    __syncthreads();
    if (lane == 63) red[wid] = incl;
    __syncthreads();
    double off = incl - seg;
    for (int i = 0; i < wid; ++i) off += red[i];
    for (int m = m0; m < m1; ++m) cdf[m] += off;
  }
  lastpos = block_max_i(lastpos, redi);  // also orders the cdf writes
  __syncthreads();
  const int any_nan = block_or_i(row_nan ? 1 : 0, redi);
  const double T = cdf[N - 1];
  const bool nan_total = isnan(T) || any_nan;
  const bool degenerate = !(T > 0.0);
  if (threadIdx.x == 0) {
    sd.zinc[c - 1] = degenerate ? -INFINITY : Astar + Bstar + c0 + gmax + log(T);
    const int flags = (degenerate ? kFlagDegenerate : 0) | (nan_total ? kFlagNumeric : 0);
    if (flags) atomicOr(sd.status, flags);
  }
  if (sd.row_lse) {
    double* rl = sd.row_lse + (size_t)(c - 1) * N;
    for (int m = threadIdx.x; m < N; m += kBlock) {
      const double a = left_leaf ? (double)leafW[(size_t)gL * N + sigma[(size_t)gL * N + m]] : -logN;
      rl[m] = a + Bstar + c0 + log(rs[m]) + (double)shift[m] * kLn2;
    }
  }
  // ---- N draws
  int32_t* ancL = sd.anc + (size_t)(c - 1) * 2 * N;
  int32_t* ancR = ancL + N;
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const Words4 w = philox4x64_10((uint64_t)n, (uint64_t)c, kPurposeCombine, 0ull, sd.seed, kKey1);
    const double u1 = unif53(w.w0), u2 = unif53(w.w1);
    int l, r;
    if (degenerate) {
      l = min((int)(u1 * N), N - 1);
      r = min((int)(u2 * N), N - 1);
    } else {
      const double target = u1 * T;
      int lo = 0, hi = N;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cdf[mid] > target) hi = mid; else lo = mid + 1;
      }
      l = lo < N ? lo : (lastpos >= 0 ? lastpos : 0);
      R v[DX];
#pragma unroll
      for (int i = 0; i < DX; ++i) v[i] = rowp[(size_t)l * DX + i];
      const double target2 = u2 * rs[l];
      const float sh = shift[l];
      r = -1;
      if (sh != 0.0f) {
        // rescued row: full scan with the row shift
        double acc = 0.0;
        int lastj = 0;
        for (int j = 0; j < N && r < 0; ++j) {
          R u[DX];
#pragma unroll
          for (int i = 0; i < DX; ++i) u[i] = colp[(size_t)j * (DX + 1) + i];
          const double e = (double)Real<R>::exp2(
              pair_log2w<R, DX>(u, colp[(size_t)j * (DX + 1) + DX], v) - (R)sh);
          acc += e;
          if (e > 0.0) lastj = j;
          if (target2 < acc) r = j;
        }
        if (r < 0) r = lastj;
      } else {
        const R* Pl = Pn + (size_t)l * Nc;
        double pref = 0.0, pref_last = 0.0;
        int k = -1, klast = 0;
        for (int kk = 0; kk < Nc; ++kk) {
          const double p = (double)Pl[kk];
          if (p > 0.0) { klast = kk; pref_last = pref; }
          if (target2 < pref + p) { k = kk; break; }
          pref += p;
        }
        if (k < 0) { k = klast; pref = pref_last; }
        const double rem = target2 - pref;
        const R* cp = colp + (size_t)k * kChunk * (DX + 1);
        R acc = (R)0;
        int lastj = 0;
#pragma unroll
        for (int jj = 0; jj < kChunk; ++jj) {
          R u[DX];
#pragma unroll
          for (int i = 0; i < DX; ++i) u[i] = cp[jj * (DX + 1) + i];
          const R e = Real<R>::exp2(pair_log2w<R, DX>(u, cp[jj * (DX + 1) + DX], v));
          acc += e;
          if (e > (R)0) lastj = jj;
          if (r < 0 && rem < (double)acc) r = jj;
        }
        if (r < 0) r = lastj;
        r += k * kChunk;
      }
      if (r >= N) r = N - 1;  // only reachable through NaN weights
    }
    ancL[n] = l;
    ancR[n] = r;
  }
}

// =============================================================== gather
// In place: sigma[t][n] <- sigma[t][l_n] (t in the left block) or
// sigma[t][r_n] (right block).  One workgroup per time row; the whole row is
// read before any of it is written.
constexpr int kGatherPer = 4096 / kBlock;
__global__ __launch_bounds__(kBlock) void k_gather(const NodeDesc* __restrict__ nodes,
                                                   const SeriesDesc* __restrict__ series, int N,
                                                   int rows_per_node, int32_t* __restrict__ sigma) {
  const int node = blockIdx.x / rows_per_node;
  const int rr = blockIdx.x - node * rows_per_node;
  const NodeDesc nd = nodes[node];
  const int t = nd.a + rr;
  if (t >= nd.b) return;  // uniform over the workgroup
  const SeriesDesc& sd = series[nd.series];
  const int32_t* __restrict__ idx = sd.anc + (size_t)(nd.c - 1) * 2 * N + (t < nd.c ? 0 : N);
  int32_t* srow = sigma + (size_t)(sd.base + t) * N;
  int32_t vals[kGatherPer];
#pragma unroll
  for (int i = 0; i < kGatherPer; ++i) {
    const int n = threadIdx.x + i * kBlock;
    if (n < N) vals[i] = srow[idx[n]];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kGatherPer; ++i) {
    const int n = threadIdx.x + i * kBlock;
    if (n < N) srow[n] = vals[i];
  }
}

// =============================================================== output
// One workgroup per time row: traj[d][t][n] = leafX[d][g][sigma[g][n]] and the
// optional diagnostic copies.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_output_rows(const SeriesDesc* __restrict__ series,
                                                        const int32_t* __restrict__ series_of_t,
                                                        int totalK, int N, int dx,
                                                        const R* __restrict__ leafX,
                                                        const R* __restrict__ leafW,
                                                        const double* __restrict__ leafL,
                                                        const int32_t* __restrict__ sigma) {
  const int g = blockIdx.x;
  const SeriesDesc& sd = series[series_of_t[g]];
  const int t = g - sd.base, K = sd.K;
  R* traj = (R*)sd.traj;
  R* lx = (R*)sd.leaf_x;
  R* lw = (R*)sd.leaf_logw;
  for (int n = threadIdx.x; n < N; n += kBlock) {
    const int src = sigma[(size_t)g * N + n];
    for (int i = 0; i < dx; ++i) {
      traj[((size_t)i * K + t) * N + n] = leafX[((size_t)i * totalK + g) * N + src];
      if (lx) lx[((size_t)i * K + t) * N + n] = leafX[((size_t)i * totalK + g) * N + n];
    }
    if (lw) lw[(size_t)t * N + n] = leafW[(size_t)g * N + n];
    if (sd.index) sd.index[(size_t)t * N + n] = src;
  }
  if (threadIdx.x == 0 && sd.leaf_logL) sd.leaf_logL[t] = leafL[g];
}

// One workgroup per series: log Z = sum_t log L_t + sum_c Z_c (fixed
// reduction order), and the output log-weights.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_output_series(const SeriesDesc* __restrict__ series,
                                                          int N, const R* __restrict__ leafW,
                                                          const double* __restrict__ leafL) {
  __shared__ double red[kBlock / 64];
  const SeriesDesc& sd = series[blockIdx.x];
  const int K = sd.K;
  double s = 0.0;
  for (int t = threadIdx.x; t < K; t += kBlock) s += leafL[sd.base + t];
  for (int c = threadIdx.x; c < K - 1; c += kBlock) s += sd.zinc[c];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *sd.log_Z = s;
  if (sd.logw) {
    R* lw = (R*)sd.logw;
    for (int n = threadIdx.x; n < N; n += kBlock)
      lw[n] = (K == 1) ? leafW[(size_t)sd.base * N + n] : (R)(-log((double)N));
  }
}

__global__ void k_clear_status(const SeriesDesc* __restrict__ series, int B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) *series[i].status = 0;
}

// ============================================================ launchers
template <typename R, int DX>
static void launch_level_t(const LevelLaunch& L, hipStream_t st, Timer* tm) {
  const size_t lds_prep = (size_t)L.N * sizeof(double);
  tm->begin(1, st);
  k_prep<R, DX><<<L.nodes, kBlock, lds_prep, st>>>(
      L.d_nodes, L.d_series, L.totalK, L.N, L.Npad, (const R*)L.leafX, (const R*)L.leafW,
      L.sigma, (R*)L.col, (R*)L.row, L.nscal);
  tm->end(1, st);
  tm->begin(2, st);
  k_rows<R, DX><<<(unsigned)L.nodes * L.RB * L.CS, kBlock, 0, st>>>(
      (const R*)L.col, (const R*)L.row, (R*)L.P, L.N, L.Npad, L.Nc, L.RB, L.CS, L.KC);
  tm->end(2, st);
  const size_t lds_samp = (size_t)L.Npad * (2 * sizeof(double) + sizeof(float));
  tm->begin(3, st);
  k_sample<R, DX><<<L.nodes, kBlock, lds_samp, st>>>(
      L.d_nodes, L.d_series, L.totalK, L.N, L.Npad, L.Nc, (const R*)L.leafW, L.sigma,
      (const R*)L.col, (const R*)L.row, (const R*)L.P, L.nscal);
  tm->end(3, st);
}

template <typename R>
static int launch_level_r(const LevelLaunch& L, hipStream_t st, Timer* tm) {
  switch (L.DX) {
    case 1: launch_level_t<R, 1>(L, st, tm); return 0;
    case 2: launch_level_t<R, 2>(L, st, tm); return 0;
    case 4: launch_level_t<R, 4>(L, st, tm); return 0;
    case 8: launch_level_t<R, 8>(L, st, tm); return 0;
    case 16: launch_level_t<R, 16>(L, st, tm); return 0;
    case 32: launch_level_t<R, 32>(L, st, tm); return 0;
  }
  return -1;
}

int launch_level(const LevelLaunch& L, hipStream_t st, Timer* tm) {
  return L.fp64 ? launch_level_r<double>(L, st, tm) : launch_level_r<float>(L, st, tm);
}

void launch_gather(const NodeDesc* d_nodes, const SeriesDesc* d_series, int nodes,
                   int rows_per_node, int N, int32_t* sigma, hipStream_t st, Timer* tm) {
  tm->begin(4, st);
  k_gather<<<(unsigned)nodes * rows_per_node, kBlock, 0, st>>>(d_nodes, d_series, N,
                                                               rows_per_node, sigma);
  tm->end(4, st);
}

template <typename R, int DX>
static void launch_leaves_t(const LeafLaunch& L, hipStream_t st, Timer* tm) {
  tm->begin(0, st);
  k_leaves<R, DX><<<L.totalK, kBlock, (size_t)L.N * sizeof(double), st>>>(
      L.d_series, L.d_series_of_t, L.totalK, L.N, (R*)L.leafX, (R*)L.leafW, L.leafL, L.sigma);
  tm->end(0, st);
}

template <typename R>
static int launch_leaves_r(const LeafLaunch& L, hipStream_t st, Timer* tm) {
  switch (L.DX) {
    case 1: launch_leaves_t<R, 1>(L, st, tm); return 0;
    case 2: launch_leaves_t<R, 2>(L, st, tm); return 0;
    case 4: launch_leaves_t<R, 4>(L, st, tm); return 0;
    case 8: launch_leaves_t<R, 8>(L, st, tm); return 0;
    case 16: launch_leaves_t<R, 16>(L, st, tm); return 0;
    case 32: launch_leaves_t<R, 32>(L, st, tm); return 0;
  }
  return -1;
}

int launch_leaves(const LeafLaunch& L, hipStream_t st, Timer* tm) {
  return L.fp64 ? launch_leaves_r<double>(L, st, tm) : launch_leaves_r<float>(L, st, tm);
}

void launch_clear_status(const SeriesDesc* d_series, int B, hipStream_t st) {
  k_clear_status<<<(B + kBlock - 1) / kBlock, kBlock, 0, st>>>(d_series, B);
}

template <typename R>
static void launch_output_t(const LeafLaunch& L, int B, int dx, hipStream_t st, Timer* tm) {
  tm->begin(5, st);
  k_output_rows<R><<<L.totalK, kBlock, 0, st>>>(L.d_series, L.d_series_of_t, L.totalK, L.N, dx,
                                                (const R*)L.leafX, (const R*)L.leafW, L.leafL,
                                                L.sigma);
  k_output_series<R><<<B, kBlock, 0, st>>>(L.d_series, L.N, (const R*)L.leafW, L.leafL);
  tm->end(5, st);
}

void launch_output(const LeafLaunch& L, int B, int dx, hipStream_t st, Timer* tm) {
  if (L.fp64) launch_output_t<double>(L, B, dx, st, tm);
  else launch_output_t<float>(L, B, dx, st, tm);
}

}  // namespace dsmc
