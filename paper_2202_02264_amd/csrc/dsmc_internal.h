// Internal data structures shared by the host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsmc {

constexpr int kBlock = 256;     // threads per workgroup of the leaf / lazy-sampling / output kernels
constexpr int kMaxWaves = 16;  // largest workgroup (1024 threads) of any kernel, in waves
constexpr int kChunk = 32;   // columns per chunk of the pair matrix
constexpr int kGroup = 8;    // chunk sums per store group (a 32-byte sector in fp32); row
                             // stride of the chunk sums and column splits are multiples

// Device-resident model (one allocation: this header, then the arrays).
// Inverse Cholesky factors and log normalisers are derived on the host in fp64.
struct DevModel {
  int K, dx, dy, obs_kind, weighting;
  int prop_kind;          // 0 Gaussian, 1 uniform on q_mean +- diag(q_chol)
  const double* m0;       // [dx]
  const double* P0_inv;   // [dx][dx] inverse of the prior Cholesky factor
  double prior_lognorm;   // -sum log diag(P0_chol) - dx/2 log(2 pi)
  const double* F;        // [dx][dx]
  const double* f;        // [dx]
  const double* Q_inv;    // [dx][dx] inverse of the transition Cholesky factor
  double trans_lognorm;   // -sum log diag(Q_chol) - dx/2 log(2 pi)
  const double* H;        // [dy][dx] R^{-1/2} H (linear-Gaussian potential)
  const double* y;        // [K][dy]  R^{-1/2} (y_t - h), or raw y_t (stochastic volatility)
  double obs_lognorm;
  const double* q_mean;   // [K][dx]
  const double* q_chol;   // [K][dx][dx]
  const double* q_inv;    // [K][dx][dx]
  const double* q_lognorm;  // [K]  Gaussian: log normaliser; uniform: -sum log(2 half-width)
  const double* Wcol;     // [dx][dx] = kappa Q_inv          (column whitening)
  const double* Wrow;     // [dx][dx] = kappa Q_inv F        (row whitening)
  const double* wcol_off; // [dx]     = kappa Q_inv f
  const double* P0_chol;  // [dx][dx] prior Cholesky factor
  const double* Q_chol;   // [dx][dx] transition Cholesky factor
  const double* leafrec;  // leaf records (padded d_x >= 8; leafrec_stride), else null
};

// Leaf records of a model whose padded state dimension DX is at least 8: at
// t * leafrec_stride(DX), q_chol[t] and its inverse (DX x DX, zero padded,
// lower triangular), then q_mean[t], the row offset of boundary t + 1
// (kappa Q^{-1/2} f - Wcol q_mean[t + 1] + Wrow q_mean[t]) and the whitened
// y_t - H q_mean[t] (DX each, zero padded); after the K records, Wcol, Wrow and
// the whitened H (DX x DX each, zero padded).  Built on the device from the
// model's arrays whenever those change.
__host__ __device__ constexpr int leafrec_stride(int DX) {
  return (2 * DX * DX + 3 * DX + 31) / 32 * 32;
}
inline size_t leafrec_size(int K, int DX) {
  return (size_t)K * leafrec_stride(DX) + 3 * (size_t)DX * DX;
}

// One series of a (batched) run.
struct SeriesDesc {
  const DevModel* model;  // device pointer
  uint64_t seed;
  int K;
  int base;               // offset of its time 0 on the packed time axis
  int root;               // node id of its last combine (-1 if K == 1)
  int pad_;
  int32_t* anc;           // [K-1][2][N]
  double* zinc;           // [K-1]
  double* row_lse;        // [K-1][N] or null
  int32_t* status;        // [1]
  void* traj;             // [dx][K][N]
  void* logw;             // [N] or null
  double* log_Z;          // [1]
  void* leaf_x;           // [dx][K][N] or null
  void* leaf_logw;        // [K][N] or null
  double* leaf_logL;      // [K] or null
  int32_t* index;         // [K][N] or null
  const void* star;       // [dx][K] star trajectory of a conditional run (slot 0), or null
};

// One combine at boundary c of series `series`: left block [a, c), right
// block [c, b).  lchild / rchild: node that formed the left / right block
// (-1: the block is a single leaf).  consumer: the node that will combine the
// block formed here (-1: root); role 0 = it is that node's left block, 1 = right.
struct NodeDesc {
  int32_t series;
  int32_t c;
  int32_t a;
  int32_t b;
  int32_t lchild;
  int32_t rchild;
  int32_t consumer;
  int32_t role;
};

// Per-node buffers, indexed by node id (position in the schedule).
struct NodeBufs {
  void* col;        // [nodes][Npad][DX+1]  (u_n, beta_n) of the node's right block
  void* row;        // [nodes][Npad][DX]    v_m of the node's left block
  void* alpha;      // [nodes][N]           left block log-weights a_m (real type)
  double* bcol;     // [nodes]              B: shift of the node's beta (log2 units: beta = log2e (b - B))
  int32_t* sfirst;  // [nodes][N]           leaf index, at the block's first time, of trajectory n
  int32_t* slast;   // [nodes][N]           same at the block's last time
  // bf16 matrix-core operands (null unless the plan is DSMC_BF16).  col and row
  // then hold the bf16-rounded u and v as fp32.
  uint16_t* colh;   // [nodes][Npad][DX]    bf16 bits of 2 u_n (zero in padding columns)
  float* colb;      // [nodes][Npad]        beta_n - ||u_n||^2 (-inf in padding columns)
  uint16_t* rowh;   // [nodes][Npad][DX]    bf16 bits of v_m
  float* rown;      // [nodes][Npad]        ||v_m||^2
  // Per time row g of the packed time axis (written by the leaf kernel): the
  // data of every leaf particle for the combines at the two boundaries of its
  // time t, which merged blocks gather when they reach their consumer.
  void* tcol;       // [rows][N][DX]  u of particle n for boundary t (t >= 1)
  double* tgq;      // [rows][N]      -log q_t(x) (+ log h_t(x) under boundary weighting)
  void* trow;       // [rows][N][DX]  v of particle n for boundary t + 1 (t + 1 < K)
  uint16_t* tcolh;  // [rows][N][DX]  bf16 plans: bits of 2u
  float* tcoln;     // [rows][N]      bf16 plans: ||u||^2
  uint16_t* trowh;  // [rows][N][DX]  bf16 plans: bits of v
  float* trown;     // [rows][N]      bf16 plans: ||v||^2
};

enum : int32_t { kFlagDegenerate = 1, kFlagNumeric = 2, kFlagLazyCap = 4 };

}  // namespace dsmc
