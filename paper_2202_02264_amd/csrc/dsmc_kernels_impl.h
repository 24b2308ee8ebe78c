// Kernel templates of the dSMC combine tree for gfx950 (wave64, fp32/fp64
// VALU, bf16 matrix cores), instantiated once per padded state dimension DX in
// dsmc_kernels_dx*.hip so that the instantiations compile in parallel.
//
//   k_leaves   once per call, one workgroup per time point: Algorithm 2 (draw,
//              weight, normalise), plus the data the time point's consumer
//              combine needs (whitened coordinates and log-weights).
//   k_rows     per level: the N x N pair-weight matrix of every combine, never
//              stored.  Each lane owns RPL rows; all lanes walk the same
//              columns, whose (u, beta) are wave-uniform and come through
//              scalar registers.  Per pair: DX x (sub, fma) + exp2 + add.
//              Output: 32-column chunk sums and fp64 row sums.
//   k_sample   per level: per combine, the fp64 row-marginal CDF, N two-stage
//              multinomial draws (Algorithm 1), the ancestry of the merged
//              block's first and last times, and the data its consumer combine
//              needs.  Several workgroups may share one combine's draws.
//   k_output   once per call: each output entry follows the ancestry from the
//              root combine down to its leaf (the gather of Algorithm 1, done
//              once instead of per level).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "dsmc.h"
#include "dsmc_device.h"
#include "dsmc_launch.h"

namespace dsmc {

// Row sums of combines with DX >= 8 are formed relative to a per-row shift
// (see k_rows); below that the column bound alone keeps them in range.
template <int DX>
inline constexpr bool kRowShift = DX >= 8;

// Four consecutive values, one 16-byte (fp32) or two (fp64) vector loads.
template <typename R>
__device__ __forceinline__ void load4(const R* p, R (&q)[4]);
template <>
__device__ __forceinline__ void load4<float>(const float* p, float (&q)[4]) {
  const float4 v = *(const float4*)p;
  q[0] = v.x; q[1] = v.y; q[2] = v.z; q[3] = v.w;
}
template <>
__device__ __forceinline__ void load4<double>(const double* p, double (&q)[4]) {
  const double2 a = ((const double2*)p)[0], b = ((const double2*)p)[1];
  q[0] = a.x; q[1] = a.y; q[2] = b.x; q[3] = b.y;
}

// Four consecutive values, one 16-byte (fp32) or two (fp64) vector stores.
template <typename R>
__device__ __forceinline__ void store4(R* p, R a, R b, R c, R d);
template <>
__device__ __forceinline__ void store4<float>(float* p, float a, float b, float c, float d) {
  *(float4*)p = make_float4(a, b, c, d);
}
template <>
__device__ __forceinline__ void store4<double>(double* p, double a, double b, double c, double d) {
  ((double2*)p)[0] = make_double2(a, b);
  ((double2*)p)[1] = make_double2(c, d);
}

// Whitened column coordinates of a right-block particle x at boundary c:
// u = Wcol (x - q_mean[c]).
template <int DX>
__device__ __forceinline__ void col_coords(const DevModel& M, int c, const double (&x)[DX],
                                           double (&u)[DX]) {
  const int dx = uniform(M.dx);
  const double* qm = M.q_mean + (size_t)c * dx;
#pragma unroll
  for (int i = 0; i < DX; ++i) {
    double s = 0.0;
    if (i < dx)
      for (int j = 0; j < dx; ++j) s += M.Wcol[i * dx + j] * (x[j] - qm[j]);
    u[i] = s;
  }
}

// Whitened row coordinates of a left-block particle x at boundary c:
// v = Wrow x + wcol_off - Wcol q_mean[c], so that
// ||u - v||^2 = (log2 e / 2) ||Q^{-1/2} (x_R - F x_L - f)||^2.
template <int DX>
__device__ __forceinline__ void row_coords(const DevModel& M, int c, const double (&x)[DX],
                                           double (&v)[DX]) {
  const int dx = uniform(M.dx);
  const double* qm = M.q_mean + (size_t)c * dx;
#pragma unroll
  for (int i = 0; i < DX; ++i) {
    double s = 0.0;
    if (i < dx) {
      s = M.wcol_off[i];
      for (int j = 0; j < dx; ++j) s += M.Wrow[i * dx + j] * x[j] - M.Wcol[i * dx + j] * qm[j];
    }
    v[i] = s;
  }
}

template <typename R, int DX>
__device__ __forceinline__ void load_particle(const R* __restrict__ leafX, int totalK, int N, int g,
                                              int src, int dx, double (&x)[DX]) {
#pragma unroll
  for (int i = 0; i < DX; ++i)
    x[i] = (i < dx) ? (double)leafX[((size_t)i * totalK + g) * N + src] : 0.0;
}

// bf16 bits of x, rounded to nearest even (the hardware conversion).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ float bf16_float(uint32_t b) { return __uint_as_float(b << 16); }

// Table entry of particle n of time row g for the combine at boundary t: u.
template <typename R, int DX>
__device__ __forceinline__ void put_tcol(const NodeBufs& nb, size_t g, int N, int n,
                                         const double (&u)[DX]) {
  R* tp = (R*)nb.tcol + (g * N + n) * DX;
#pragma unroll
  for (int i = 0; i < DX; ++i) tp[i] = (R)u[i];
}

// Table entry of particle n of time row g for the combine at boundary t + 1: v.
template <typename R, int DX>
__device__ __forceinline__ void put_trow(const NodeBufs& nb, size_t g, int N, int n,
                                         const double (&v)[DX]) {
  R* tp = (R*)nb.trow + (g * N + n) * DX;
#pragma unroll
  for (int i = 0; i < DX; ++i) tp[i] = (R)v[i];
}

// bf16 plans keep each matrix-core operand as a pair of bf16 numbers, hi and
// lo = the bf16 rounding of the remainder, so that hi + lo carries 16
// significant bits; a particle's entry is 2 DX bf16 values: DX hi, then DX lo.
__device__ __forceinline__ void bf16_split(float a, uint32_t& hi, uint32_t& lo) {
  hi = bf16_bits(a);
  lo = bf16_bits(a - bf16_float(hi));
}

// Column n of combine `node` := table entry (g, src) with log2 weight beta.
template <typename R, int DX>
__device__ __forceinline__ void copy_col(const NodeBufs& nb, size_t node, int Npad, int n, size_t g,
                                         int N, int src, double beta) {
  const R* tp = (const R*)nb.tcol + (g * N + src) * DX;
  R* cp = (R*)nb.col + (node * Npad + n) * (DX + 1);
#pragma unroll
  for (int i = 0; i < DX; ++i) cp[i] = tp[i];
  cp[DX] = (R)beta;
  if constexpr (sizeof(R) == 4 && DX >= 16) {
    if (nb.colh) {
      const uint4* s4 = (const uint4*)(nb.tcolh + (g * N + src) * 2 * DX);
      uint4* d4 = (uint4*)(nb.colh + (node * Npad + n) * 2 * DX);
#pragma unroll
      for (int q = 0; q < DX / 4; ++q) d4[q] = s4[q];
      nb.colb[node * Npad + n] = (float)beta - nb.tcoln[g * N + src];
    }
  }
}

// Row m of combine `node` := table entry (g, src).
template <typename R, int DX>
__device__ __forceinline__ void copy_row(const NodeBufs& nb, size_t node, int Npad, int m, size_t g,
                                         int N, int src) {
  const R* tp = (const R*)nb.trow + (g * N + src) * DX;
  R* rp = (R*)nb.row + (node * Npad + m) * DX;
#pragma unroll
  for (int i = 0; i < DX; ++i) rp[i] = tp[i];
  if constexpr (sizeof(R) == 4 && DX >= 16) {
    if (nb.rowh) {
      const uint4* s4 = (const uint4*)(nb.trowh + (g * N + src) * 2 * DX);
      uint4* d4 = (uint4*)(nb.rowh + (node * Npad + m) * 2 * DX);
#pragma unroll
      for (int q = 0; q < DX / 4; ++q) d4[q] = s4[q];
      nb.rown[node * Npad + m] = nb.trown[g * N + src];
    }
  }
}

// Matrix operands of the leaf kernel for DX >= 8: the model's per-time leaf
// records (zero-padded to DX x DX, laid out by leafrec_stride) read through the
// constant address space, so that every entry, being wave-uniform, reaches the
// FMAs through scalar registers instead of LDS or vector loads.
typedef const __attribute__((address_space(4))) double cdouble;

// p, opaque to the optimiser: loads through it stay where they are written
// instead of being hoisted out of the particle loop (which would hold every
// matrix entry in registers at once).
__device__ __forceinline__ cdouble* opaque(cdouble* p) {
  asm volatile("" : "+s"(p));
  return p;
}

// A wave-uniform pointer, held in scalar registers.
__device__ __forceinline__ cdouble* uniform_ptr(const double* p) {
  const uint64_t v = (uint64_t)p;
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return (cdouble*)((hi << 32) | lo);
}

// Whitened coordinates of one particle for one boundary, from d = x - q_mean[t]
// (zero past d_x): columns u = Wcol d (Wcol lower triangular), rows
// v = Wrow d + off.  Stores the R-rounded coordinates at dst (16-byte vector
// stores where `aligned`), and in bf16 plans (kSplit) the split operands (2u
// for columns, v for rows; DX/2 words of hi pairs, then DX/2 of lo pairs) at
// dsth and the fp32 squared norm of the rounded entry at *dstn.
template <typename R, int DX, bool kRow, bool kSplit>
__device__ __forceinline__ void emit_coords(cdouble* Wm, cdouble* off, const double (&d)[DX],
                                            R* dst, bool aligned, uint32_t* dsth, float* dstn) {
  double nrm = 0.0;
#pragma unroll
  for (int i0 = 0; i0 < DX; i0 += 4) {
    R r4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = i0 + k;
      double acc = kRow ? off[i] : 0.0;
#pragma unroll
      for (int j = 0; j < (kRow ? DX : i + 1); ++j) acc = fma(Wm[i * DX + j], d[j], acc);
      r4[k] = (R)acc;
    }
    if (aligned) {
      store4<R>(dst + i0, r4[0], r4[1], r4[2], r4[3]);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) dst[i0 + k] = r4[k];
    }
    if constexpr (kSplit) {
      uint32_t h[4], l[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        nrm += (double)r4[k] * (double)r4[k];
        bf16_split(kRow ? (float)r4[k] : 2.0f * (float)r4[k], h[k], l[k]);
      }
      *(uint2*)(dsth + (i0 >> 1)) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
      *(uint2*)(dsth + DX / 2 + (i0 >> 1)) = make_uint2(l[0] | (l[1] << 16), l[2] | (l[3] << 16));
    }
  }
  if constexpr (kSplit) *dstn = (float)nrm;
}

// Padding column n (N <= n < Npad): weight zero.
template <typename R, int DX>
__device__ __forceinline__ void put_col_pad(const NodeBufs& nb, size_t node, int Npad, int n) {
  R* cp = (R*)nb.col + (node * Npad + n) * (DX + 1);
#pragma unroll
  for (int i = 0; i < DX; ++i) cp[i] = (R)0;
  cp[DX] = (R)(-INFINITY);
  if constexpr (sizeof(R) == 4 && DX >= 16) {
    if (nb.colh) {
      uint4* dst = (uint4*)(nb.colh + (node * Npad + n) * 2 * DX);
#pragma unroll
      for (int q = 0; q < DX / 4; ++q) dst[q] = make_uint4(0u, 0u, 0u, 0u);
      nb.colb[node * Npad + n] = -INFINITY;
    }
  }
}

// ================================================================ leaves
// The four standard normals of one leaf Philox block.  fp32 plans use the
// Box-Muller transform with its transcendentals written out (box_muller_poly,
// a few fp64 ulps from the library's); their particles are rounded to fp32,
// which hides the difference in all but rare last-ulp cases.  fp64 plans use
// the library's log, sqrt, cos and sin.
template <typename R>
__device__ __forceinline__ void leaf_normals(const Words4& w, double& z0, double& z1, double& z2,
                                             double& z3) {
  if constexpr (sizeof(R) == 4) {
    box_muller_poly(w.w0, w.w1, z0, z1);
    box_muller_poly(w.w2, w.w3, z2, z3);
  } else {
    box_muller(w.w0, w.w1, z0, z1);
    box_muller(w.w2, w.w3, z2, z3);
  }
}

// Leaf weights of one time row once every particle's unnormalised log weight
// ell[n] and -log q (+ log h) gq[n] are known: normalise (rounded to R, the
// value every consumer sees), write leafW, leafL and the block's shift, and
// return max_n (lbar_n + gq_n) (every thread of the block).
template <typename R>
__device__ __forceinline__ double leaf_normalise(double* ell, const double* gq, int g, int N,
                                                 int bad, const SeriesDesc& sd,
                                                 R* __restrict__ leafW, double* __restrict__ leafL,
                                                 double* __restrict__ bmerged) {
  __shared__ double red[2 * kMaxWaves];
  __shared__ int redi[2 * kMaxWaves];
  const double logN = log((double)N);
  __syncthreads();
  double mx = -INFINITY, gmx = -INFINITY;
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    mx = fmax(mx, ell[n]);
    gmx = fmax(gmx, gq[n]);
  }
  block_max2(mx, gmx, red);
  double s = 0.0;
  if (mx > -INFINITY)
    for (int n = threadIdx.x; n < N; n += blockDim.x) s += exp(ell[n] - mx);
  s = block_sum(s, red);
  const bool degenerate = !(mx > -INFINITY);
  const double lse = mx + log(s);
  double bmax = -INFINITY;  // max_n (lbar_n + gq_n): shift of a leaf right block
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    const double lbar = degenerate ? -logN : ell[n] - lse;
    const R lr = (R)lbar;
    leafW[(size_t)g * N + n] = lr;
    ell[n] = (double)lr;  // the stored (rounded) weight is what every consumer sees
    bmax = fmax(bmax, (double)lr + gq[n]);
  }
  block_max_or(bmax, bad, red, redi);
  if (threadIdx.x == 0) {
    leafL[g] = degenerate ? -INFINITY : lse - logN;
    bmerged[g] = -logN + gmx;
    const int flags = bad | (degenerate ? kFlagDegenerate : 0);
    if (flags) atomicOr(sd.status, flags);
  }
  return bmax;
}

// Unnormalised leaf log weight l and gq = -log q_t(x) (+ log h_t(x) under
// boundary weighting) from log q, log h and (t = 0) the prior.
__device__ __forceinline__ void leaf_logw(int t, int weighting, double lq, double lh,
                                          double lprior, double& l, double& gg) {
  gg = -lq;
  if (t == 0) {
    l = lh + lprior - lq;
    if (weighting == 1) gg += lh;
  } else if (weighting == 0) {
    l = lh;
  } else {
    l = 0.0;
    gg += lh;
  }
}

// DX < 8.  One workgroup per time row g of the packed time axis.
template <typename R, int DX>
__global__ __launch_bounds__(kBlock, 3) void k_leaves(
    const SeriesDesc* __restrict__ series, const int32_t* __restrict__ series_of_t,
    const int32_t* __restrict__ leaf_cons, int row0, int totalK, int N, int Npad,
    R* __restrict__ leafX, R* __restrict__ leafW, double* __restrict__ leafL,
    double* __restrict__ bmerged, NodeBufs nb) {
  static_assert(DX < 8, "DX >= 8 uses k_leaves_mat");
  extern __shared__ double sh[];
  const int g = row0 + blockIdx.x;
  const SeriesDesc& sd = series[series_of_t[g]];
  const DevModel& M = *sd.model;
  const int t = uniform(g - sd.base);
  const int dx = uniform(M.dx);
  const int K = uniform(sd.K);
  const int weighting = uniform(M.weighting);
  double* ell = sh;     // [N] unnormalised leaf log-weights
  double* gq = sh + N;  // [N] -log q_t (+ log h_t, boundary weighting)
  int bad = 0;
  const double* qm = M.q_mean + (size_t)t * dx;
  const double* qc = M.q_chol + (size_t)t * dx * dx;
  const bool unif = uniform(M.prop_kind) == 1;  // uniform proposal: uniforms, not normals
  // particle n from its standard variates v (normals, or uniforms): x =
  // q_mean + L v in place from the last coordinate down (x_i needs v_0 .. v_i),
  // stored, then its weights
  auto particle = [&](int n, double (&x)[DX]) __attribute__((always_inline)) {
#pragma unroll
    for (int i = DX - 1; i >= 0; --i) {
      double xi = 0.0;
      if (i < dx) {
        if (unif) {  // q_mean + half-width (2 u - 1)
          xi = qm[i] + qc[i * dx + i] * (2.0 * x[i] - 1.0);
        } else {
          xi = qm[i];
#pragma unroll
          for (int j = 0; j <= i; ++j) xi += qc[i * dx + j] * x[j];
        }
        const R xr = (R)xi;
        leafX[((size_t)i * totalK + g) * N + n] = xr;
        xi = (double)xr;  // weights are those of the stored particle
      }
      x[i] = xi;
    }
    if (n == 0 && sd.star != nullptr) {
      // conditional run: slot 0 holds the star trajectory (its proposal draw
      // above is discarded), weighted like every other particle
      const R* st = (const R*)sd.star;
#pragma unroll
      for (int i = 0; i < DX; ++i) {
        double xi = 0.0;
        if (i < dx) {
          const R xr = st[(size_t)i * K + t];
          leafX[((size_t)i * totalK + g) * N + n] = xr;
          xi = (double)xr;
        }
        x[i] = xi;
      }
    }
    const double lq = log_proposal<DX>(M, t, x);
    const double lh = log_potential<DX>(M, t, x);
    double l, gg;
    leaf_logw(t, weighting, lq, lh, t == 0 ? log_prior<DX>(M, x) : 0.0, l, gg);
    if (isnan(l) || isnan(gg)) bad = kFlagNumeric;
    ell[n] = l;
    gq[n] = gg;
  };
  auto variates = [&](const Words4& w, double& z0, double& z1, double& z2, double& z3)
      __attribute__((always_inline)) {
    if (unif) {
      z0 = unif53(w.w0);
      z1 = unif53(w.w1);
      z2 = unif53(w.w2);
      z3 = unif53(w.w3);
    } else {
      leaf_normals<R>(w, z0, z1, z2, z3);
    }
  };
  if constexpr (DX <= 2) {
    // d_x dividing 4: one flat stream of variates per time, block q giving
    // variates 4q .. 4q+3, coordinate i of particle n being variate n d_x + i
    constexpr int PPB = 4 / DX;  // particles per block
    for (int q = threadIdx.x; q * PPB < N; q += blockDim.x) {
      const Words4 w = philox4x64_10((uint64_t)q, (uint64_t)t, kPurposeLeaf, 0ull, sd.seed, kKey1);
      double z[4];
      variates(w, z[0], z[1], z[2], z[3]);
#pragma unroll
      for (int k = 0; k < PPB; ++k) {
        const int n = q * PPB + k;
        if (n < N) {
          double x[DX];
#pragma unroll
          for (int i = 0; i < DX; ++i) x[i] = z[k * DX + i];
          particle(n, x);
        }
      }
    }
  } else {
    // otherwise ceil(d_x / 4) blocks (n, t, 2, j) per particle, variates 4j .. 4j+3
    for (int n = threadIdx.x; n < N; n += blockDim.x) {
      double x[DX];
#pragma unroll
      for (int j = 0; j < (DX + 3) / 4; ++j) {
        const Words4 w = philox4x64_10((uint64_t)n, (uint64_t)t, kPurposeLeaf, (uint64_t)j,
                                       sd.seed, kKey1);
        double z0, z1, z2, z3;
        variates(w, z0, z1, z2, z3);
        if (4 * j < DX) x[4 * j] = z0;
        if (4 * j + 1 < DX) x[4 * j + 1] = z1;
        if (4 * j + 2 < DX) x[4 * j + 2] = z2;
        if (4 * j + 3 < DX) x[4 * j + 3] = z3;
      }
      particle(n, x);
    }
  }
  const double bmax = leaf_normalise<R>(ell, gq, g, N, bad, sd, leafW, leafL, bmerged);
  // Every particle's data for the combines at both boundaries of t (the
  // tables merged blocks gather from), and the data of the combine that
  // consumes this single-point block: its right block (c == t) or its left
  // block (c == t + 1).
  const int cons = leaf_cons[g];
  const int P = cons >> 1, role = cons & 1;
  for (int n = threadIdx.x; n < N; n += blockDim.x) {
    double x[DX];
    load_particle<R, DX>(leafX, totalK, N, g, n, dx, x);
    nb.tgq[(size_t)g * N + n] = gq[n];
    if (t >= 1) {
      double u[DX];
      col_coords<DX>(M, t, x, u);
      put_tcol<R, DX>(nb, (size_t)g, N, n, u);
      if (cons >= 0 && role == 1) {
        const double beta = (bmax > -INFINITY) ? (ell[n] + gq[n] - bmax) * kLog2e : -INFINITY;
        copy_col<R, DX>(nb, (size_t)P, Npad, n, (size_t)g, N, n, beta);
      }
    }
    if (t + 1 < K) {
      double v[DX];
      row_coords<DX>(M, t + 1, x, v);
      put_trow<R, DX>(nb, (size_t)g, N, n, v);
      if (cons >= 0 && role == 0) {
        copy_row<R, DX>(nb, (size_t)P, Npad, n, (size_t)g, N, n);
        ((R*)nb.alpha)[(size_t)P * N + n] = (R)ell[n];
      }
    }
  }
  if (cons >= 0 && role == 1) {
    for (int n = N + threadIdx.x; n < Npad; n += blockDim.x) put_col_pad<R, DX>(nb, (size_t)P, Npad, n);
    if (threadIdx.x == 0) nb.bcol[P] = bmax;
  }
}

// DX >= 8.  One workgroup per time row g; each particle's whole leaf step in
// registers: the normals, x = q_mean + L z, log q from L^{-1} (x - q_mean),
// the linear-Gaussian log h from the whitened residual, and the whitened
// coordinates for both boundaries of t, every matrix entry a scalar operand
// (the model's leaf records).  A boundary consumed by this leaf's level-0
// combine is written straight into that combine's buffers (no table entry:
// no other combine reads it); the other boundary goes to its table.
// Launched with kBlock threads (the loops stride by the constant: with
// blockDim.x the compiler spilled several times more scalar registers).
template <typename R, int DX, bool kSplit>
__global__ __launch_bounds__(kBlock, 3) void k_leaves_mat(
    const SeriesDesc* __restrict__ series, const int32_t* __restrict__ series_of_t,
    const int32_t* __restrict__ leaf_cons, int row0, int totalK, int N, int Npad,
    R* __restrict__ leafX, R* __restrict__ leafW, double* __restrict__ leafL,
    double* __restrict__ bmerged, NodeBufs nb) {
  static_assert(DX >= 8 && DX % 4 == 0, "k_leaves_mat: DX >= 8, a multiple of 4");
  extern __shared__ double sh[];
  double* ell = sh;  // [N] leaf log-weights, unnormalised then normalised
  const int g = row0 + blockIdx.x;
  const SeriesDesc& sd = series[series_of_t[g]];
  const DevModel& M = *sd.model;
  const int t = uniform(g - sd.base);
  const int dx = uniform(M.dx);
  const int dy = uniform(M.dy);
  const int K = uniform(sd.K);
  const int weighting = uniform(M.weighting);
  constexpr int S = leafrec_stride(DX);
  cdouble* const rec0 = uniform_ptr(M.leafrec + (size_t)t * S);
  cdouble* const inv0 = uniform_ptr(M.leafrec + (size_t)uniform(M.K) * S);
  const bool lg_obs = uniform(M.obs_kind) == 0 && dy <= DX;
  const double qln = M.q_lognorm[t];
  const int cons = leaf_cons[g];
  const int P = cons >> 1, role = cons & 1;
  const bool col_direct = cons >= 0 && role == 1;  // boundary t belongs to combine P
  const bool row_direct = cons >= 0 && role == 0;  // boundary t + 1 belongs to combine P
  int bad = 0;
  auto reload = [&](int n, double (&x)[DX]) { load_particle<R, DX>(leafX, totalK, N, g, n, dx, x); };
  for (int n = threadIdx.x; n < N; n += kBlock) {
    cdouble* rec = opaque(rec0);
    cdouble* Lc = rec;                // q_chol[t]
    cdouble* Li = rec + DX * DX;      // q_chol[t]^{-1}
    cdouble* qm = rec + 2 * DX * DX;  // q_mean[t]
    cdouble* ro = qm + DX;            // row offset for boundary t + 1
    cdouble* yo = ro + DX;            // whitened y_t - H q_mean[t]
    cdouble* inv = opaque(inv0);
    cdouble* Wc = inv;                // Wcol (lower triangular)
    cdouble* Wr = inv + DX * DX;      // Wrow
    cdouble* Hw = inv + 2 * DX * DX;  // whitened H, dy rows
    double d[DX];  // x - q_mean[t] of the stored particle (zero past d_x)
    {
      double x[DX];
#pragma unroll
      for (int i = 0; i < DX; ++i) x[i] = qm[i];
      // one Philox block (four normals) at a time, each added into every x_i
      // it enters (x_i needs z_0 .. z_i)
#pragma unroll
      for (int j = 0; j < DX / 4; ++j) {
        const Words4 w = philox4x64_10((uint64_t)n, (uint64_t)t, kPurposeLeaf, (uint64_t)j,
                                       sd.seed, kKey1);
        double z[4];
        leaf_normals<R>(w, z[0], z[1], z[2], z[3]);
#pragma unroll
        for (int i = 4 * j; i < DX; ++i) {
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (4 * j + k <= i) x[i] = fma(Lc[i * DX + 4 * j + k], z[k], x[i]);
        }
      }
      if (n == 0 && sd.star != nullptr) {
        // conditional run: slot 0 holds the star trajectory (its proposal
        // draw above is discarded), weighted like every other particle
        const R* st = (const R*)sd.star;
#pragma unroll
        for (int i = 0; i < DX; ++i) x[i] = (i < dx) ? (double)st[(size_t)i * K + t] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < DX; ++i) {
        double xi = 0.0;
        if (i < dx) {
          const R xr = (R)x[i];
          leafX[((size_t)i * totalK + g) * N + n] = xr;
          xi = (double)xr;  // weights are those of the stored particle
        }
        d[i] = xi - qm[i];
      }
    }
    // log q_t(x) = -||L^{-1} (x - q_mean)||^2 / 2 + log normaliser
    double qq = 0.0;
#pragma unroll
    for (int i = 0; i < DX; ++i) {
      double zi = 0.0;
#pragma unroll
      for (int j = 0; j <= i; ++j) zi = fma(Li[i * DX + j], d[j], zi);
      qq = fma(zi, zi, qq);
    }
    const double lq = -0.5 * qq + qln;
    double lh = 0.0;  // other potentials: in the pass below
    if (lg_obs) {  // whitened residual y_t - H x = yo - H d
      double qh = 0.0;
#pragma unroll 1
      for (int i = 0; i < dy; ++i) {
        double r = yo[i];
#pragma unroll
        for (int k = 0; k < DX; ++k) r = fma(-Hw[i * DX + k], d[k], r);
        qh = fma(r, r, qh);
      }
      lh = -0.5 * qh + M.obs_lognorm;
    }
    ell[n] = lh;
    nb.tgq[(size_t)g * N + n] = -lq;
    if (t >= 1) {  // u for boundary t
      const size_t e = col_direct ? (size_t)P * Npad + n : (size_t)g * N + n;
      R* dst = col_direct ? (R*)nb.col + e * (DX + 1) : (R*)nb.tcol + e * DX;
      uint32_t* dh = kSplit ? (uint32_t*)(col_direct ? nb.colh : nb.tcolh) + e * DX : nullptr;
      float* dn = kSplit ? nb.tcoln + (size_t)g * N + n : nullptr;  // read back for the weight
      emit_coords<R, DX, false, kSplit>(Wc, nullptr, d, dst, !col_direct, dh, dn);
    }
    if (t + 1 < K) {  // v for boundary t + 1
      const size_t e = row_direct ? (size_t)P * Npad + n : (size_t)g * N + n;
      R* dst = (R*)(row_direct ? nb.row : nb.trow) + e * DX;
      uint32_t* dh = kSplit ? (uint32_t*)(row_direct ? nb.rowh : nb.trowh) + e * DX : nullptr;
      float* dn = kSplit ? (row_direct ? nb.rown : nb.trown) + e : nullptr;
      emit_coords<R, DX, true, kSplit>(Wr, ro, d, dst, true, dh, dn);
    }
  }
  // The weights, from log q and (linear-Gaussian) log h kept above; other
  // potentials and the prior at t = 0 re-read the stored particle.  Kept out
  // of the loop above, whose registers these rare paths would crowd.
  double* gq = nb.tgq + (size_t)g * N;  // this thread's own entries, read back
  for (int n = threadIdx.x; n < N; n += kBlock) {
    double lh = ell[n], lprior = 0.0;
    if (!lg_obs || t == 0) {
      double x[DX];
      reload(n, x);
      if (!lg_obs) lh = log_potential<DX>(M, t, x);
      if (t == 0) lprior = log_prior<DX>(M, x);
    }
    double l, gg;
    leaf_logw(t, weighting, -gq[n], lh, lprior, l, gg);
    if (isnan(l) || isnan(gg)) bad = kFlagNumeric;
    ell[n] = l;
    gq[n] = gg;
  }
  const double bmax = leaf_normalise<R>(ell, gq, g, N, bad, sd, leafW, leafL, bmerged);
  if (col_direct) {
    for (int n = threadIdx.x; n < N; n += kBlock) {
      const double beta = (bmax > -INFINITY) ? (ell[n] + gq[n] - bmax) * kLog2e : -INFINITY;
      const size_t e = (size_t)P * Npad + n;
      ((R*)nb.col)[e * (DX + 1) + DX] = (R)beta;
      if constexpr (kSplit) nb.colb[e] = (float)beta - nb.tcoln[(size_t)g * N + n];
    }
    for (int n = N + threadIdx.x; n < Npad; n += kBlock) put_col_pad<R, DX>(nb, (size_t)P, Npad, n);
    if (threadIdx.x == 0) nb.bcol[P] = bmax;
  }
  if (row_direct)
    for (int n = threadIdx.x; n < N; n += kBlock) ((R*)nb.alpha)[(size_t)P * N + n] = (R)ell[n];
}

// ================================================================= rows
// Tile = (combine, row block of RPL*64*W rows, column split of KC chunks, KC a
// multiple of 8).  Lane owns rows base + lane + 64 r, r < RPL; lanes past N
// recompute row N-1 and store the same values (no per-row branches).  Chunk
// sums go to P[node][m][k] (row stride NcP = Nc rounded up to 8), eight chunks
// (one aligned 32-byte sector) per pair of vector stores, so that no sector is
// written in part, and the sampler reads a row's sums as one contiguous run.
// The fp64 row sum is the sum, in group order, of the fp64 sums of its groups
// of kGroup chunks (each in chunk order), whatever the tile: with one column
// split the tile stores it; with more, every split stores its groups' sums
// (Gs) and the sampling kernel adds them.

template <typename R, int DX, int RPL>
__global__ __launch_bounds__(kBlock) void k_rows(const R* __restrict__ col,
                                                 const R* __restrict__ row,
                                                 R* __restrict__ P, double* __restrict__ Rsum,
                                                 float* __restrict__ Rshift,
                                                 double* __restrict__ Gs,
                                                 const int32_t* __restrict__ node_list,
                                                 int node0, int N, int Npad, int Nc, int NcP,
                                                 int NGS, int RB, int CS, int KC, int force_redo) {
  const int W = blockDim.x >> 6;
  const int tiles = RB * CS;
  const int node_local = blockIdx.x / tiles;
  const int tile = blockIdx.x - node_local * tiles;
  const int rb = tile / CS, cs = tile - rb * CS;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int base = (rb * W + wave) * 64 * RPL;
  if (base >= N) return;  // wave-uniform
  const size_t nodeid = node_list ? (size_t)node_list[node_local] : (size_t)node0 + node_local;
  const R* __restrict__ colp = col + nodeid * Npad * (DX + 1);
  R v[RPL][DX];
  int mrow[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int m = base + lane + 64 * r;
    mrow[r] = m < N ? m : N - 1;
#pragma unroll
    for (int i = 0; i < DX; ++i) v[r][i] = row[(nodeid * Npad + mrow[r]) * DX + i];
  }
  // Row shift (DX >= 8): the row's largest log2 weight over its first chunk,
  // so that row sums stay inside the fp32 range when every pair weight is far
  // below the column bound.
  R sft[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) sft[r] = (R)0;
  if constexpr (kRowShift<DX>) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      R mx = (R)(-INFINITY);
      for (int jj = 0; jj < kChunk; ++jj) {
        R u[DX];
#pragma unroll
        for (int i = 0; i < DX; ++i) u[i] = colp[jj * (DX + 1) + i];
        mx = fmax(mx, pair_log2w<R, DX>(u, colp[jj * (DX + 1) + DX], v[r]));
      }
      // held at fp32 precision: the sampling kernel reads it back as fp32
      sft[r] = (mx > (R)(-INFINITY) && mx < (R)INFINITY) ? (R)(float)mx : (R)0;
    }
  }
  double Rm[RPL];
  R* __restrict__ Pn = P + (size_t)node_local * N * NcP;
  const int k0 = cs * KC, k1 = min(Nc, k0 + KC);
  auto pass = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) Rm[r] = 0.0;
    for (int kg = k0; kg < k1; kg += kGroup) {
      R acc[RPL][kGroup];
      double G[RPL];  // the group's sum
#pragma unroll
      for (int r = 0; r < RPL; ++r) G[r] = 0.0;
#pragma unroll
      for (int q = 0; q < kGroup; ++q) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) acc[r][q] = (R)0;
        if (kg + q < k1) {  // uniform
          const R* __restrict__ cp = colp + (size_t)(kg + q) * kChunk * (DX + 1);
#pragma unroll
          for (int jj = 0; jj < kChunk; ++jj) {
            R u[DX];
#pragma unroll
            for (int i = 0; i < DX; ++i) u[i] = cp[jj * (DX + 1) + i];
            const R beta = cp[jj * (DX + 1) + DX];
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
              if constexpr (kRowShift<DX>)
                acc[r][q] += Real<R>::exp2(pair_log2w<R, DX>(u, beta, v[r]) - sft[r]);
              else
                acc[r][q] += Real<R>::exp2(pair_log2w<R, DX>(u, beta, v[r]));
            }
          }
#pragma unroll
          for (int r = 0; r < RPL; ++r) G[r] += (double)acc[r][q];
        }
      }
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        Rm[r] += G[r];
        R* pm = Pn + (size_t)mrow[r] * NcP + kg;
        store4<R>(pm, acc[r][0], acc[r][1], acc[r][2], acc[r][3]);
        store4<R>(pm + 4, acc[r][4], acc[r][5], acc[r][6], acc[r][7]);
        if (CS > 1) Gs[((size_t)node_local * N + mrow[r]) * NGS + kg / kGroup] = G[r];
      }
    }
  };
  pass();
  if constexpr (kRowShift<DX>) {
    // A row whose sum left the fp32 range (its largest weight far above the
    // chunk-0 estimate, or every weight far below it) takes its exact maximum
    // as shift and the wave redoes its rows; the other rows recompute the same
    // values.  Rows are whole here (one column split for DX >= 8).
    bool bad[RPL];
    int any = 0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      bad[r] = ((!(Rm[r] >= Real<R>::kTiny) || isinf(Rm[r])) && !isnan(Rm[r])) || force_redo;
      any |= bad[r] ? 1 : 0;
    }
    if (__any(any)) {
      R mx[RPL];
#pragma unroll
      for (int r = 0; r < RPL; ++r) mx[r] = (R)(-INFINITY);
      for (int k = k0; k < k1; ++k) {
        const R* __restrict__ cp = colp + (size_t)k * kChunk * (DX + 1);
        for (int jj = 0; jj < kChunk; ++jj) {
          R u[DX];
#pragma unroll
          for (int i = 0; i < DX; ++i) u[i] = cp[jj * (DX + 1) + i];
          const R beta = cp[jj * (DX + 1) + DX];
#pragma unroll
          for (int r = 0; r < RPL; ++r) mx[r] = fmax(mx[r], pair_log2w<R, DX>(u, beta, v[r]));
        }
      }
#pragma unroll
      for (int r = 0; r < RPL; ++r)
        if (bad[r]) sft[r] = (mx[r] > (R)(-INFINITY) && mx[r] < (R)INFINITY) ? (R)(float)mx[r] : (R)0;
      pass();
    }
    if (cs == 0) {
#pragma unroll
      for (int r = 0; r < RPL; ++r) Rshift[(size_t)node_local * N + mrow[r]] = (float)sft[r];
    }
  }
  if (CS == 1) {
#pragma unroll
    for (int r = 0; r < RPL; ++r) Rsum[(size_t)node_local * N + mrow[r]] = Rm[r];
  }
}

// ============================================================ rows (bf16)
// Matrix-core form of k_rows for bf16 plans (DX = 16 or 32).  The pair's log2
// weight beta_n - ||u_n - v_m||^2 equals (beta_n - ||u_n||^2) - ||v_m||^2 +
// (2 u_n) . v_m, with the norms in fp32 and the dot product from split bf16
// operands: with 2u = Uh + Ul and v = Vh + Vl (hi and remainder, each bf16),
// (2u) . v = Uh.Vh + Uh.Vl + Ul.Vh up to the dropped Ul.Vl (about 2^-16 of
// it).  A wave owns 32 MB rows; for each 32-column chunk and each block of 32
// rows, 3 DX / 16 v_mfma_f32_32x32x16_bf16 add the 32 x 32 dot products (u on
// the instruction's row side, v on its column side) onto accumulators that
// start at the two fp32 norm terms, so each accumulator ends as the pair's
// log2 weight.  Lane (j, h) holds column j of the block (row m = block + j) for the
// 16 chunk columns 8 (r / 4) + 4 h + r % 4, r < 16; the lanes j and j + 32
// together hold the whole chunk.  Outputs as k_rows (chunk sums, and fp64 row
// sums in chunk order with one column split).
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

template <int DX, int MB>
__global__ __launch_bounds__(kBlock) void k_rows_mfma(
    const uint16_t* __restrict__ colh, const float* __restrict__ colb,
    const uint16_t* __restrict__ rowh, const float* __restrict__ rown, float* __restrict__ P,
    double* __restrict__ Rsum, float* __restrict__ Rshift, const int32_t* __restrict__ node_list,
    int node0, int N, int Npad, int Nc, int NcP, int RB, int CS, int KC, int force_redo) {
  static_assert(DX == 16 || DX == 32, "bf16 rows need DX 16 or 32");
  constexpr int KS = DX / 16;  // instructions per 32 x 32 block
  const int W = blockDim.x >> 6;
  const int tiles = RB * CS;
  const int node_local = blockIdx.x / tiles;
  const int tile = blockIdx.x - node_local * tiles;
  const int rb = tile / CS, cs = tile - rb * CS;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j32 = lane & 31, h = lane >> 5;
  const int base = (rb * W + wave) * 32 * MB;
  if (base >= N) return;  // wave-uniform
  const size_t nodeid = node_list ? (size_t)node_list[node_local] : (size_t)node0 + node_local;
  bf16x8_t vf[MB][KS], vl[MB][KS];
  float vv[MB];
  int mrow[MB];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    const int m = base + 32 * b + j32;
    mrow[b] = m < N ? m : N - 1;
    const uint16_t* rp = rowh + ((size_t)nodeid * Npad + mrow[b]) * 2 * DX + 8 * h;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      vf[b][s] = *(const bf16x8_t*)(rp + 16 * s);
      vl[b][s] = *(const bf16x8_t*)(rp + DX + 16 * s);
    }
    vv[b] = rown[(size_t)nodeid * Npad + mrow[b]];
  }
  const uint16_t* __restrict__ ch = colh + (size_t)nodeid * Npad * 2 * DX;
  const float* __restrict__ cb = colb + (size_t)nodeid * Npad;
  // Row shift: the row's largest log2 weight over chunk 0 (as k_rows), folded
  // into the row norm term so the main loop pays nothing for it.
  float vv0[MB], sft[MB];
#pragma unroll
  for (int b = 0; b < MB; ++b) vv0[b] = vv[b];
  // log2 weights of chunk k for block b, into acc (row-norm term vv[b])
  auto block = [&](int k, int b, f32x16_t& acc) __attribute__((always_inline)) {
    const int n0 = k * kChunk;
    bf16x8_t uf[KS], ul[KS];
    const uint16_t* up = ch + (size_t)(n0 + j32) * 2 * DX + 8 * h;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      uf[s] = *(const bf16x8_t*)(up + 16 * s);
      ul[s] = *(const bf16x8_t*)(up + DX + 16 * s);
    }
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4) {
      const float4 t4 = *(const float4*)(cb + n0 + 8 * g4 + 4 * h);
      acc[4 * g4] = t4.x - vv[b];
      acc[4 * g4 + 1] = t4.y - vv[b];
      acc[4 * g4 + 2] = t4.z - vv[b];
      acc[4 * g4 + 3] = t4.w - vv[b];
    }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ul[s], vf[b][s], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(uf[s], vl[b][s], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(uf[s], vf[b][s], acc, 0, 0, 0);
    }
  };
  // largest log2 weight of each row block over chunks [ka, kb)
  auto row_max = [&](int ka, int kb, float (&mx)[MB]) {
#pragma unroll
    for (int b = 0; b < MB; ++b) mx[b] = -INFINITY;
    for (int k = ka; k < kb; ++k) {
#pragma unroll
      for (int b = 0; b < MB; ++b) {
        f32x16_t acc;
        block(k, b, acc);
#pragma unroll
        for (int r = 0; r < 16; ++r) mx[b] = fmaxf(mx[b], acc[r]);
      }
    }
#pragma unroll
    for (int b = 0; b < MB; ++b) mx[b] = fmaxf(mx[b], __shfl_xor(mx[b], 32, 64));
  };
  {
    float mx[MB];
    row_max(0, 1, mx);
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      sft[b] = (mx[b] > -INFINITY && mx[b] < INFINITY) ? mx[b] : 0.0f;
      vv[b] = vv0[b] + sft[b];
    }
  }
  double Rm[MB];
  float* __restrict__ Pn = P + (size_t)node_local * N * NcP;
  const int k0 = cs * KC, k1 = min(Nc, k0 + KC);
  auto pass = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int b = 0; b < MB; ++b) Rm[b] = 0.0;
    for (int kg = k0; kg < k1; kg += kGroup) {
      float c4[MB][kGroup];
      double G[MB];  // the group's sum
#pragma unroll
      for (int b = 0; b < MB; ++b) G[b] = 0.0;
#pragma unroll
      for (int q = 0; q < kGroup; ++q) {
#pragma unroll
        for (int b = 0; b < MB; ++b) c4[b][q] = 0.0f;
        if (kg + q < k1) {  // uniform
#pragma unroll
          for (int b = 0; b < MB; ++b) {
            f32x16_t acc;
            block(kg + q, b, acc);
            float e = 0.0f;
#pragma unroll
            for (int r = 0; r < 16; ++r) e += Real<float>::exp2(acc[r]);
            e += __shfl_xor(e, 32, 64);
            c4[b][q] = e;
            G[b] += (double)e;
          }
        }
      }
#pragma unroll
      for (int b = 0; b < MB; ++b) Rm[b] += G[b];
      if (h == 0) {
#pragma unroll
        for (int b = 0; b < MB; ++b) {
          float* pm = Pn + (size_t)mrow[b] * NcP + kg;
          store4<float>(pm, c4[b][0], c4[b][1], c4[b][2], c4[b][3]);
          store4<float>(pm + 4, c4[b][4], c4[b][5], c4[b][6], c4[b][7]);
        }
      }
    }
  };
  pass();
  // As k_rows: a row whose sum left the fp32 range takes its exact maximum as
  // shift and the wave redoes its rows (whole rows: one column split).
  int any = 0;
  bool bad[MB];
#pragma unroll
  for (int b = 0; b < MB; ++b) {
    bad[b] = ((!(Rm[b] >= Real<float>::kTiny) || isinf(Rm[b])) && !isnan(Rm[b])) || force_redo;
    any |= bad[b] ? 1 : 0;
  }
  if (__any(any)) {
#pragma unroll
    for (int b = 0; b < MB; ++b) vv[b] = vv0[b];
    float mx[MB];
    row_max(k0, k1, mx);
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      if (bad[b]) sft[b] = (mx[b] > -INFINITY && mx[b] < INFINITY) ? mx[b] : 0.0f;
      vv[b] = vv0[b] + sft[b];
    }
    pass();
  }
  if (cs == 0 && h == 0) {
#pragma unroll
    for (int b = 0; b < MB; ++b) Rshift[(size_t)node_local * N + mrow[b]] = sft[b];
  }
  if (CS == 1 && h == 0) {
#pragma unroll
    for (int b = 0; b < MB; ++b) Rsum[(size_t)node_local * N + mrow[b]] = Rm[b];
  }
}

// =============================================================== sample
// Workgroup (combine, ds) of DS workgroups per combine; each builds the row
// CDF of its combine and takes the draws n in [ds per, (ds+1) per).
//   w_m = exp(a_m - A*) R_m  (fp64),  C_m = sum_{i<=m} w_i,
//   Z_c = A* + B + trans_lognorm + ln C_{N-1}
//   l_n = first m with C_m > u1 C_{N-1}
//   r_n = first j with (chunk prefix + within-chunk prefix) > u2 R_l
// Rows whose R_m leaves the fp32 range (underflow, or overflow when a row
// shift estimated from one chunk is too low) are recomputed with their exact
// maximum as shift: their chunk sums go to Pr, R_m carries a factor
// 2^shift_m and the weights are formed in log space.
// The combine's column data is staged in LDS when it fits (col_in_lds).

// Draw n of combine `nodeid` is (l, r): its ancestry, the merged block's
// first/last-time leaf indices, and the data the consuming combine reads.
// The leaf indices of draw (l, r) at the merged block's first and last times.
__device__ __forceinline__ void draw_sources(const NodeBufs& nb, const NodeDesc& nd, int N, int l,
                                             int r, int& sf, int& sl) {
  sf = (nd.lchild < 0) ? l : nb.sfirst[(size_t)nd.lchild * N + l];
  sl = (nd.rchild < 0) ? r : nb.slast[(size_t)nd.rchild * N + r];
}

template <typename R, int DX>
__device__ __forceinline__ void record_draw(const NodeBufs& nb, const NodeDesc& nd, int nodeid,
                                            int N, int Npad, int n, int l, int r, int sf, int sl,
                                            int32_t* ancL, int32_t* ancR, int gA, int gB,
                                            double logN, const double* __restrict__ bmerged) {
  ancL[n] = l;
  ancR[n] = r;
  nb.sfirst[(size_t)nodeid * N + n] = sf;
  nb.slast[(size_t)nodeid * N + n] = sl;
  const int cons = nd.consumer;
  if (cons >= 0) {
    if (nd.role == 1) {  // merged block is the right block of `cons` (boundary a)
      const double b = -logN + nb.tgq[(size_t)gA * N + sf];
      copy_col<R, DX>(nb, (size_t)cons, Npad, n, (size_t)gA, N, sf, (b - bmerged[gA]) * kLog2e);
    } else {  // merged block is the left block of `cons` (boundary b)
      copy_row<R, DX>(nb, (size_t)cons, Npad, n, (size_t)gB, N, sl);
      ((R*)nb.alpha)[(size_t)cons * N + n] = (R)(-logN);
    }
  }
}

// Column data of the combine in LDS: 32-column chunks padded by 8 bytes, so
// that lanes reading the same column of different chunks (the draws' chunk
// recompute) fall into different LDS banks.
template <typename R, int DX>
constexpr int col_chunk_lds_stride() {
  return kChunk * (DX + 1) + (int)(8 / sizeof(R));
}
template <typename R, int DX>
__device__ __forceinline__ int col_chunk_stride(int col_in_lds) {
  return col_in_lds ? col_chunk_lds_stride<R, DX>() : kChunk * (DX + 1);
}

// fp64 sum of a rescued row's chunk sums (in Pr) in chunk order: the sum the
// rescue forms for the row's CDF weight
template <typename R>
__device__ __forceinline__ double row_sum(const R* __restrict__ Pm, int Nc, int NcP) {
  double s = 0.0;
  for (int kb = 0; kb < NcP; kb += 16) {
    R q[16];
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4) {
      R t4[4];
      if (kb + 4 * g4 < NcP) load4<R>(Pm + kb + 4 * g4, t4);
#pragma unroll
      for (int i = 0; i < 4; ++i) q[4 * g4 + i] = (kb + 4 * g4 < NcP) ? t4[i] : (R)0;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (kb + i < Nc) s += (double)q[i];
  }
  return s;
}

template <typename R, int DX>
__global__ __launch_bounds__(kBlock) void k_sample(
    const NodeDesc* __restrict__ nodes, const SeriesDesc* __restrict__ series,
    const int32_t* __restrict__ node_list, int node0, int DS,
    int N, int Npad, int Nc, int NcP, int rows_summed, int NGS, int col_in_lds,
    int force_rescue, int rescale_chunk, const double* __restrict__ bmerged,
    const R* __restrict__ P, R* __restrict__ Pr, double* __restrict__ Rsum,
    const double* __restrict__ Gs, float* __restrict__ Rshift,
    unsigned long long* __restrict__ rescue_count, NodeBufs nb) {
  extern __shared__ double smem[];
  const int nthr = blockDim.x;
  const int cstr = col_chunk_stride<R, DX>(col_in_lds);
  // LDS (sample_lds): cdf [Npad] fp64: row sums R_m, then the row CDF; csum
  // [Nc] fp64: chunk sums of the row being rescued; shift [Npad] (DX >= 8
  // only: the rows' fp32 shifts; below, only rescued rows have one, kept in
  // Rshift); aw [Npad]: row weights alpha_m (left leaf); need, resc
  // [Npad / 32]: rows still to rescue, rescued rows (their chunk sums are in
  // Pr); rescue_list [nthr]; lcol [Nc][cstr] when col_in_lds.
  double* cdf = smem;
  double* csum = cdf + Npad;
  float* shift = (float*)(csum + Nc);
  R* aw = (R*)(shift + (kRowShift<DX> ? Npad : 0));
  unsigned* need = (unsigned*)(aw + Npad);
  unsigned* resc = need + Npad / 32;
  int* rescue_list = (int*)(resc + Npad / 32);
  R* lcol = (R*)(rescue_list + nthr);
  __shared__ double red[2 * kMaxWaves];
  __shared__ int redi[2 * kMaxWaves];
  const int node_local = blockIdx.x / DS;
  const int ds = blockIdx.x - node_local * DS;
  const int nodeid = node_list ? node_list[node_local] : node0 + node_local;
  const NodeDesc nd = nodes[nodeid];
  const SeriesDesc& sd = series[nd.series];
  const DevModel& M = *sd.model;
  const int c = nd.c;
  const bool left_leaf = nd.lchild < 0;
  const double logN = log((double)N);
  const R* __restrict__ gcol = (const R*)nb.col + (size_t)nodeid * Npad * (DX + 1);
  const R* __restrict__ rowp = (const R*)nb.row + (size_t)nodeid * Npad * DX;
  const R* __restrict__ Pn = P + (size_t)node_local * N * NcP;
  R* __restrict__ Prn = Pr + (size_t)node_local * N * NcP;
  double* __restrict__ Rn = Rsum + (size_t)node_local * N;
  const R* __restrict__ alp = (const R*)nb.alpha + (size_t)nodeid * N;
  // the shift of row m (fp32): DX >= 8 every row's; below, rescued rows only
  float* rsh = Rshift + (size_t)node_local * N;
  auto row_shift = [&](int m) __attribute__((always_inline)) -> float {
    if constexpr (kRowShift<DX>) return shift[m];
    return ((resc[m >> 5] >> (m & 31)) & 1u) ? rsh[m] : 0.0f;
  };
  if (col_in_lds) {  // four loads in flight per thread
    constexpr int CW = kChunk * (DX + 1);
    const int tot = Npad * (DX + 1);
    for (int i0 = threadIdx.x; i0 < tot; i0 += 4 * nthr) {
      R cv[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) cv[b] = gcol[min(i0 + b * nthr, tot - 1)];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int i = i0 + b * nthr;
        if (i < tot) {
          const int k = i / CW;
          lcol[k * cstr + (i - k * CW)] = cv[b];
        }
      }
    }
  }
  const R* colp = col_in_lds ? lcol : gcol;
  // column j, coordinate d of the combine (padded layout in LDS)
  auto colv = [&](int j, int d) __attribute__((always_inline)) -> R { return colp[(j >> 5) * cstr + (j & 31) * (DX + 1) + d]; };
  __syncthreads();

  // ---- row sums (thread owns a contiguous segment of rows)
  __shared__ int n_rescue;
  for (int i = threadIdx.x; i < Npad / 32; i += nthr) {
    need[i] = 0u;
    resc[i] = 0u;
  }
  __syncthreads();
  const int per = (N + nthr - 1) / nthr;
  const int m0 = threadIdx.x * per, m1 = min(N, m0 + per);
  double amax = -INFINITY;
  int rescued = 0, row_nan = 0;
  for (int mb = m0; mb < m1; mb += 4) {
    double Rv[4];
    R av[4];
    float sv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // the loads of four rows issued together
      const int m = min(mb + i, m1 - 1);
      if (rows_summed) {
        Rv[i] = Rn[m];
      } else {
        // column splits: the rows kernel left the sums of the row's groups of
        // kGroup chunks; their sum in group order is the row sum of one split
        const double* gp = Gs + ((size_t)node_local * N + m) * NGS;
        const int NG = NcP / kGroup;
        double t;
        if (NGS == 4) {
          const double2 g01 = ((const double2*)gp)[0], g23 = ((const double2*)gp)[1];
          t = g01.x;
          if (NG > 1) t += g01.y;
          if (NG > 2) t += g23.x;
          if (NG > 3) t += g23.y;
        } else {
          t = gp[0];
          for (int g = 1; g < NG; ++g) t += gp[g];
        }
        Rv[i] = t;
      }
      av[i] = left_leaf ? alp[m] : (R)0;
      sv[i] = kRowShift<DX> ? Rshift[(size_t)node_local * N + m] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = mb + i;
      if (m < m1) {
        amax = fmax(amax, left_leaf ? (double)av[i] : -logN);
        const double Rm = Rv[i];
        if ((!(Rm >= Real<R>::kTiny) || isinf(Rm) || force_rescue) && !isnan(Rm)) {
          atomicOr(&need[m >> 5], 1u << (m & 31));
          atomicOr(&resc[m >> 5], 1u << (m & 31));
          rescued = 1;
        } else if (!rows_summed) {
          // stored for the draws: every workgroup of the combine writes the
          // same values, and none reads them before its own write
          Rn[m] = Rm;
        }
        if (isnan(Rm)) row_nan = 1;
        cdf[m] = Rm;
        if constexpr (kRowShift<DX>) shift[m] = sv[i];
        aw[m] = av[i];
      }
    }
  }
  double Astar = amax;
  block_max_or(Astar, rescued, red, redi);  // also orders the writes above
  // Underflow rescue, one row at a time by the whole workgroup: exact row
  // maximum as shift, then the fp64 sum of exp2(s - shift) over a fixed
  // partition of the columns in a fixed reduction order.  Rows are taken in
  // passes of at most one per thread.
  bool first_pass = true;
  while (rescued) {
    if (threadIdx.x == 0) n_rescue = 0;
    __syncthreads();
    for (int wd = threadIdx.x; wd < Npad / 32; wd += nthr) {
      unsigned bits = need[wd];
      while (bits) {
        const int b = __ffs(bits) - 1;
        bits &= bits - 1;
        const int slot = atomicAdd(&n_rescue, 1);
        if (slot < nthr) {
          rescue_list[slot] = wd * 32 + b;
          atomicAnd(&need[wd], ~(1u << b));
        }
      }
    }
    __syncthreads();
    const int total = n_rescue;
    const int cnt = min(total, nthr);
    if (first_pass && rescue_count && ds == 0 && threadIdx.x == 0)
      atomicAdd(rescue_count, (unsigned long long)total);
    first_pass = false;
    for (int i = 0; i < cnt; ++i) {
      const int m = rescue_list[i];
      R v[DX];
#pragma unroll
      for (int d = 0; d < DX; ++d) v[d] = rowp[(size_t)m * DX + d];
      double smax = -INFINITY;
      for (int j = threadIdx.x; j < N; j += nthr) {
        R u[DX];
#pragma unroll
        for (int d = 0; d < DX; ++d) u[d] = colv(j, d);
        smax = fmax(smax, (double)pair_log2w<R, DX>(u, colv(j, DX), v));
      }
      smax = block_max(smax, red);
      const R sh = (R)(float)smax;  // the shift is kept as fp32
      // the row's chunk sums relative to sh, into Pr (thread k owns chunk k;
      // the same terms in the same order as the draw's chunk recompute; every
      // workgroup of the combine writes the same values), and their fp64 sum
      // in chunk order
      R* Pm = Prn + (size_t)m * NcP;
      for (int k = threadIdx.x; k < Nc; k += nthr) {
        R acc = (R)0;
        if (smax > -INFINITY) {
          const R* cp = colp + (size_t)k * cstr;
#pragma unroll 4
          for (int jj = 0; jj < kChunk; ++jj) {
            R u[DX];
#pragma unroll
            for (int d = 0; d < DX; ++d) u[d] = cp[jj * (DX + 1) + d];
            acc += Real<R>::exp2(pair_log2w<R, DX>(u, cp[jj * (DX + 1) + DX], v) - sh);
          }
        }
        Pm[k] = acc;
        csum[k] = (double)acc;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int k = 0; k < Nc; ++k) tot += csum[k];
        cdf[m] = (smax > -INFINITY) ? tot : 0.0;
        const float fs = (smax > -INFINITY) ? (float)sh : 0.0f;
        if constexpr (kRowShift<DX>) shift[m] = fs;
        else rsh[m] = fs;  // every workgroup of the combine writes the same value
      }
      __syncthreads();
    }
    if (total <= nthr) break;
  }
  const double Bc = nb.bcol[nodeid];
  if (ds == 0 && sd.row_lse) {  // r_m = log of row m's sum of pair weights
    double* rl = sd.row_lse + (size_t)(c - 1) * N;
    for (int m = m0; m < m1; ++m) {
      const double a = left_leaf ? (double)aw[m] : -logN;
      rl[m] = a + Bc + M.trans_lognorm + log(cdf[m]) + (double)row_shift(m) * kLn2;
    }
  }

  // ---- row weights (each thread its own rows): direct, or in log space when
  // a row carries a shift
  double G = 0.0;
  if (rescued || kRowShift<DX>) {
    double gmax = -INFINITY;
    for (int m = m0; m < m1; ++m) {
      const double a = left_leaf ? (double)aw[m] : -logN;
      double rho = -INFINITY;
      if (Astar > -INFINITY && cdf[m] > 0.0) rho = a - Astar + (double)row_shift(m) * kLn2 + log(cdf[m]);
      cdf[m] = rho;
      gmax = fmax(gmax, rho);
    }
    G = block_max(gmax, red);
    for (int m = m0; m < m1; ++m) cdf[m] = (G > -INFINITY) ? exp(cdf[m] - G) : 0.0;
  } else {
    for (int m = m0; m < m1; ++m) {
      double w = 0.0;
      if (Astar > -INFINITY) w = (left_leaf ? exp((double)aw[m] - Astar) : 1.0) * cdf[m];
      cdf[m] = w;
    }
  }
  double seg = 0.0;
  int lastpos = -1;
  for (int m = m0; m < m1; ++m) {
    const double w = cdf[m];
    if (w > 0.0) lastpos = m;
    seg += w;
    cdf[m] = seg;  // segment-local inclusive prefix for now
  }
  {  // workgroup scan of the segment totals
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
  int any_nan = row_nan;
  block_max_i_or(lastpos, any_nan, redi);
  __syncthreads();
  const double T = cdf[N - 1];
  const bool degenerate = !(T > 0.0);
  if (ds == 0 && threadIdx.x == 0) {
    sd.zinc[c - 1] = degenerate ? -INFINITY : Astar + Bc + M.trans_lognorm + G + log(T);
    const int flags = (degenerate ? kFlagDegenerate : 0) | ((isnan(T) || any_nan) ? kFlagNumeric : 0);
    if (flags) atomicOr(sd.status, flags);
  }
  // consumer of the merged block [a, b)
  const int cons = nd.consumer;
  const int crole = nd.role;
  const int ca = nd.a, cb = nd.b;
  const int gA = sd.base + ca, gB = sd.base + cb - 1;
  if (cons >= 0 && crole == 1 && ds == 0) {
    for (int n = N + threadIdx.x; n < Npad; n += nthr) put_col_pad<R, DX>(nb, (size_t)cons, Npad, n);
    if (threadIdx.x == 0) nb.bcol[cons] = bmerged[gA];
  }
  // ---- draws, one per thread at a time (consecutive draws in consecutive
  // lanes, so that their records are coalesced).  Per draw: the left index by
  // the CDF search in LDS, then row l's coordinates and row sum R_l (rescued
  // rows: the sum of their chunk sums in Pr), its chunk sums 16 at a time, the
  // recomputed chunk, the sources.  (Two draws in lockstep took about 190
  // registers and measured slower.)
  const int dper = (N + DS - 1) / DS;
  const int n0 = ds * dper, n1 = min(N, n0 + dper);
  int32_t* ancL = sd.anc + (size_t)(c - 1) * 2 * N;
  int32_t* ancR = ancL + N;
  const bool star = sd.star != nullptr;
  auto draw = [&](int n, double u1, double u2) __attribute__((always_inline)) {
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
      const bool lres = (resc[l >> 5] >> (l & 31)) & 1u;
      const double Rl = Rn[l];
      const R* Pl = (lres ? Prn : Pn) + (size_t)l * NcP;
      const float sh = row_shift(l);
      const double target2 = u2 * (lres ? row_sum<R>(Pl, Nc, NcP) : Rl);
      // chunk: first k whose prefix of chunk sums exceeds u2 R_l (16 at a time)
      double pref = 0.0, pref_last = 0.0, pk = 0.0, plast = 0.0;
      int k = -1, klast = 0;
      for (int kb = 0; kb < Nc && k < 0; kb += 16) {
        R qq[16];
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
          R t4[4];
          if (kb + 4 * g4 < NcP) load4<R>(Pl + kb + 4 * g4, t4);
#pragma unroll
          for (int i = 0; i < 4; ++i) qq[4 * g4 + i] = (kb + 4 * g4 < NcP) ? t4[i] : (R)0;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int kk = kb + i;
          if (k < 0 && kk < Nc) {
            const double pp = (double)qq[i];
            if (pp > 0.0) { klast = kk; pref_last = pref; plast = pp; }
            if (target2 < pref + pp) { k = kk; pk = pp; } else pref += pp;
          }
        }
      }
      if (k < 0) { k = klast; pref = pref_last; pk = plast; }
      double rem = target2 - pref;
      // recompute chunk k of row l in the rows kernel's order
      const R* cp = colp + (size_t)k * cstr;
      auto col_w = [&](int jj) __attribute__((always_inline)) -> R {
        R u[DX];
#pragma unroll
        for (int i = 0; i < DX; ++i) u[i] = cp[jj * (DX + 1) + i];
        return Real<R>::exp2(pair_log2w<R, DX>(u, cp[jj * (DX + 1) + DX], v) - (R)sh);
      };
      R acc = (R)0;
      int lastj = 0, rr = -1;
      bool done = false;
      if constexpr (sizeof(R) == 4 && DX >= 16) {
        if (rescale_chunk) {
          // bf16 plans: the stored chunk sums come from the matrix cores'
          // expanded form; the recompute here is the direct form, so the
          // search is rescaled to the recomputed chunk total
          R ev[kChunk];
          R tot = (R)0;
#pragma unroll
          for (int jj = 0; jj < kChunk; ++jj) {
            ev[jj] = col_w(jj);
            tot += ev[jj];
          }
          if (pk > 0.0 && tot > (R)0) rem *= (double)tot / pk;
#pragma unroll
          for (int jj = 0; jj < kChunk; ++jj) {
            acc += ev[jj];
            if (ev[jj] > (R)0) lastj = jj;
            if (rr < 0 && rem < (double)acc) rr = jj;
          }
          done = true;
        }
      }
      if (!done) {
#pragma unroll
        for (int jj = 0; jj < kChunk; ++jj) {
          acc += col_w(jj);
          if (rr < 0 && rem < (double)acc) rr = jj;
        }
        // rounding left u2 R_l at or past the chunk's total: the last column
        // of positive weight, found again only in this rare case
        if (rr < 0)
          for (int jj = kChunk - 1; jj > 0 && lastj == 0; --jj)
            if (col_w(jj) > (R)0) lastj = jj;
      }
      if (rr < 0) rr = lastj;
      rr += k * kChunk;
      r = rr < N ? rr : N - 1;  // N - 1 only reachable through NaN weights
    }
    if (n == 0 && star) {  // conditional combine: slot 0 keeps the star, (0, 0)
      l = 0;
      r = 0;
    }
    int sf, sl;
    draw_sources(nb, nd, N, l, r, sf, sl);
    record_draw<R, DX>(nb, nd, nodeid, N, Npad, n, l, r, sf, sl, ancL, ancR, gA, gB, logN,
                       bmerged);
  };
  for (int n = n0 + threadIdx.x; n < n1; n += nthr) {
    const Words4 w = philox4x64_10((uint64_t)n, (uint64_t)c, kPurposeCombine, 0ull, sd.seed, kKey1);
    draw(n, unif53(w.w0), unif53(w.w1));
  }
}


// ========================================================= lazy sampling
// Lazy resampling of one combine (Section 4.2): the N index pairs are drawn
// without the pair-row pass, by N independent chains that evaluate only the
// pairs they propose.  lazy == 1: Algorithm 7, `param` Metropolis-Hastings
// steps from (n, n) with proposals uniform over the N^2 pairs; lazy == 2:
// Algorithm 8, rejection from uniform proposals against the bound
// max_m a_m + max_n b_n + max log p_c (at most `param` proposals per chain).
// The target is the pair weight exp(a_m) 2^(beta_n - ||u_n - v_m||^2) relative
// to that bound.  No increment is estimated (Z_c = NaN).
template <typename R, int DX>
__global__ __launch_bounds__(kBlock) void k_sample_lazy(
    const NodeDesc* __restrict__ nodes, const SeriesDesc* __restrict__ series,
    const int32_t* __restrict__ node_list, int node0, int DS, int N, int Npad, int lazy,
    int param, const double* __restrict__ bmerged, NodeBufs nb) {
  __shared__ double red[2 * kMaxWaves];
  const int node_local = blockIdx.x / DS;
  const int ds = blockIdx.x - node_local * DS;
  const int nodeid = node_list ? node_list[node_local] : node0 + node_local;
  const NodeDesc nd = nodes[nodeid];
  const SeriesDesc& sd = series[nd.series];
  const int c = nd.c;
  const bool left_leaf = nd.lchild < 0;
  const double logN = log((double)N);
  const R* __restrict__ colp = (const R*)nb.col + (size_t)nodeid * Npad * (DX + 1);
  const R* __restrict__ rowp = (const R*)nb.row + (size_t)nodeid * Npad * DX;
  const R* __restrict__ alp = (const R*)nb.alpha + (size_t)nodeid * N;
  // the bound: max_m a_m, and max_n beta_n (the column shift B can exceed the
  // block's own maximum for a merged right block)
  double Astar = left_leaf ? -INFINITY : -logN, bmax = -INFINITY;
  for (int m = threadIdx.x; m < N; m += kBlock) {
    if (left_leaf) Astar = fmax(Astar, (double)alp[m]);
    bmax = fmax(bmax, (double)colp[(size_t)m * (DX + 1) + DX]);
  }
  block_max2(Astar, bmax, red);
  const int cons = nd.consumer;
  const int gA = sd.base + nd.a, gB = sd.base + nd.b - 1;
  if (ds == 0) {
    if (threadIdx.x == 0) sd.zinc[c - 1] = __builtin_nan("");
    if (sd.row_lse) {
      double* rl = sd.row_lse + (size_t)(c - 1) * N;
      for (int m = threadIdx.x; m < N; m += kBlock) rl[m] = __builtin_nan("");
    }
    if (cons >= 0 && nd.role == 1) {
      for (int n = N + threadIdx.x; n < Npad; n += kBlock) put_col_pad<R, DX>(nb, (size_t)cons, Npad, n);
      if (threadIdx.x == 0) nb.bcol[cons] = bmerged[gA];
    }
  }
  // natural log of pair (i, j)'s weight relative to the rejection bound
  auto logw = [&](int i, int j) __attribute__((always_inline)) -> double {
    R v[DX], u[DX];
#pragma unroll
    for (int d = 0; d < DX; ++d) {
      v[d] = rowp[(size_t)i * DX + d];
      u[d] = colp[(size_t)j * (DX + 1) + d];
    }
    const double a = left_leaf ? (double)alp[i] : -logN;
    return (a - Astar) +
           kLn2 * ((double)pair_log2w<R, DX>(u, colp[(size_t)j * (DX + 1) + DX], v) - bmax);
  };
  const uint64_t purpose = (lazy == 1) ? kPurposeLazyMH : kPurposeLazyRS;
  const int dper = (N + DS - 1) / DS;
  const int n0 = ds * dper, n1 = min(N, n0 + dper);
  int32_t* ancL = sd.anc + (size_t)(c - 1) * 2 * N;
  int32_t* ancR = ancL + N;
  // proposal indices from the two 32-bit halves of one Philox word
  auto index_lo = [N](uint64_t w) { return (int)(((w & 0xffffffffull) * (uint64_t)N) >> 32); };
  auto index_hi = [N](uint64_t w) { return (int)(((w >> 32) * (uint64_t)N) >> 32); };
  int capped = 0, bad = 0;
  for (int n = n0 + threadIdx.x; n < n1; n += kBlock) {
    int l = n, r = n;
    if (lazy == 1) {
      double cur = logw(l, r);
      auto step = [&](uint64_t wi, uint64_t wu) __attribute__((always_inline)) {
        const int ip = index_lo(wi), jp = index_hi(wi);
        const double prop = logw(ip, jp);
        if (unif53(wu) < exp(prop - cur)) {
          l = ip;
          r = jp;
          cur = prop;
        }
      };
      // block j serves proposals 2j (words 0, 1) and 2j + 1 (words 2, 3)
      for (int b = 0; b < param; b += 2) {
        const Words4 w = philox4x64_10((uint64_t)n, (uint64_t)c, purpose, (uint64_t)(b >> 1),
                                       sd.seed, kKey1);
        step(w.w0, w.w1);
        if (b + 1 < param) step(w.w2, w.w3);
      }
      if (isnan(cur)) bad = 1;
    } else {
      bool done = false;
      auto trial = [&](uint64_t wi, uint64_t wu) __attribute__((always_inline)) {
        l = index_lo(wi);
        r = index_hi(wi);
        const double lw = logw(l, r);
        if (isnan(lw)) bad = 1;
        done = unif53(wu) < exp(lw);
      };
      for (int k = 0; k < param && !done; k += 2) {
        const Words4 w = philox4x64_10((uint64_t)n, (uint64_t)c, purpose, (uint64_t)(k >> 1),
                                       sd.seed, kKey1);
        trial(w.w0, w.w1);
        if (!done && k + 1 < param) trial(w.w2, w.w3);
      }
      if (!done) capped = 1;
    }
    if (n == 0 && sd.star != nullptr) {  // conditional combine: slot 0 keeps the star
      l = 0;
      r = 0;
    }
    int sf, sl;
    draw_sources(nb, nd, N, l, r, sf, sl);
    record_draw<R, DX>(nb, nd, nodeid, N, Npad, n, l, r, sf, sl, ancL, ancR, gA, gB, logN, bmerged);
  }
  if (capped || bad) atomicOr(sd.status, (capped ? kFlagLazyCap : 0) | (bad ? kFlagNumeric : 0));
}

// ============================================================ launchers
template <int DX, int MB>
static void launch_rows_mfma(const LevelLaunch& L, hipStream_t st, unsigned grid, unsigned block) {
  k_rows_mfma<DX, MB><<<grid, block, 0, st>>>(L.nb.colh, L.nb.colb, L.nb.rowh, L.nb.rown,
                                              (float*)L.P, L.Rsum, L.Rshift, L.node_list, L.node0,
                                              L.N, L.Npad, L.Nc, L.NcP, L.RB, L.CS, L.KC,
                                              L.force_rescue ? 1 : 0);
}

template <typename R, int DX, int RPL>
static void launch_rows_valu(const LevelLaunch& L, hipStream_t st, unsigned grid, unsigned block) {
  k_rows<R, DX, RPL><<<grid, block, 0, st>>>((const R*)L.nb.col, (const R*)L.nb.row, (R*)L.P,
                                             L.Rsum, L.Rshift, L.Gs, L.node_list,
                                             L.node0, L.N, L.Npad, L.Nc, L.NcP, group_stride(L.NcP),
                                             L.RB, L.CS, L.KC,
                                             L.force_rescue ? 1 : 0);
}

template <typename R, int DX>
static int launch_rows_t(const LevelLaunch& L, hipStream_t st) {
  const unsigned grid = (unsigned)L.nodes * L.RB * L.CS;
  const unsigned block = 64u * L.W;
  if constexpr (sizeof(R) == 4 && DX >= 16) {
    if (L.bf16) {  // 64 RPL rows per wave, as the fp32 kernel
      switch (L.RPL) {
        case 1: launch_rows_mfma<DX, 2>(L, st, grid, block); return 0;
        case 2: launch_rows_mfma<DX, 4>(L, st, grid, block); return 0;
        case 4: launch_rows_mfma<DX, 8>(L, st, grid, block); return 0;
      }
      return -1;
    }
  }
  if (L.bf16) return -1;
  switch (L.RPL) {
    case 1: launch_rows_valu<R, DX, 1>(L, st, grid, block); return 0;
    case 2: launch_rows_valu<R, DX, 2>(L, st, grid, block); return 0;
    case 4: launch_rows_valu<R, DX, 4>(L, st, grid, block); return 0;
  }
  return -1;
}

template <typename R, int DX>
static int launch_level_t(const LevelLaunch& L, hipStream_t st, Timer* tm) {
  if (L.lazy) {  // no pair-row pass
    tm->begin(2, st);
    k_sample_lazy<R, DX><<<(unsigned)L.nodes * L.DS, kBlock, 0, st>>>(
        L.d_nodes, L.d_series, L.node_list, L.node0, L.DS, L.N, L.Npad, L.lazy, L.lazy_param,
        L.bmerged, L.nb);
    tm->end(2, st);
    return 0;
  }
  tm->begin(1, st);
  if (launch_rows_t<R, DX>(L, st)) return -1;
  tm->end(1, st);
  size_t lds_samp = sample_lds(L.Npad, L.Nc, (size_t)L.SB, kRowShift<DX>, sizeof(R));
  const size_t lds_col = (size_t)(L.Npad / kChunk) * col_chunk_lds_stride<R, DX>() * sizeof(R);
  const int col_in_lds = (lds_samp + lds_col <= 96 * 1024) ? 1 : 0;
  if (col_in_lds) lds_samp += lds_col;
  tm->begin(2, st);
  k_sample<R, DX><<<(unsigned)L.nodes * L.DS, (unsigned)L.SB, lds_samp, st>>>(
      L.d_nodes, L.d_series, L.node_list, L.node0, L.DS, L.N, L.Npad, L.Nc, L.NcP,
      L.CS == 1 ? 1 : 0, group_stride(L.NcP), col_in_lds, L.force_rescue ? 1 : 0, L.bf16 ? 1 : 0, L.bmerged,
      (const R*)L.P, (R*)L.Pr, L.Rsum, L.Gs, L.Rshift, L.rescue_count, L.nb);
  tm->end(2, st);
  return 0;
}

template <typename R, int DX>
static void launch_leaves_t(const LeafLaunch& L, hipStream_t st, Timer* tm) {
  tm->begin(0, st);
  if constexpr (DX >= 8) {
    const size_t lds = (size_t)L.N * sizeof(double);
    if constexpr (sizeof(R) == 4 && DX >= 16) {
      if (L.nb.colh) {  // bf16 plan: split operands too
        k_leaves_mat<R, DX, true><<<L.rows, kBlock, lds, st>>>(
            L.d_series, L.d_series_of_t, L.d_leaf_cons, L.row0, L.totalK, L.N, L.Npad,
            (R*)L.leafX, (R*)L.leafW, L.leafL, L.bmerged, L.nb);
        tm->end(0, st);
        return;
      }
    }
    k_leaves_mat<R, DX, false><<<L.rows, kBlock, lds, st>>>(
        L.d_series, L.d_series_of_t, L.d_leaf_cons, L.row0, L.totalK, L.N, L.Npad, (R*)L.leafX,
        (R*)L.leafW, L.leafL, L.bmerged, L.nb);
  } else {
    k_leaves<R, DX><<<L.rows, leaf_block(L.N), 2 * (size_t)L.N * sizeof(double), st>>>(
        L.d_series, L.d_series_of_t, L.d_leaf_cons, L.row0, L.totalK, L.N, L.Npad, (R*)L.leafX,
        (R*)L.leafW, L.leafL, L.bmerged, L.nb);
  }
  tm->end(0, st);
}


// Entry points of one (DX, real type) instantiation (dsmc_kernels_dx*.hip).
#define DSMC_INSTANTIATE(DX, R, SUF)                                                    \
  int launch_level_dx##DX##SUF(const LevelLaunch& L, hipStream_t st, Timer* tm) {       \
    return launch_level_t<R, DX>(L, st, tm);                                            \
  }                                                                                     \
  void launch_leaves_dx##DX##SUF(const LeafLaunch& L, hipStream_t st, Timer* tm) {      \
    launch_leaves_t<R, DX>(L, st, tm);                                                  \
  }

}  // namespace dsmc
