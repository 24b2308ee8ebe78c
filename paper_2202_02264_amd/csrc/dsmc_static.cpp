// dsmc_smooth_static: one smoother run with no device allocation.  Every
// workspace buffer of the run (particles, weights, per-time tables, per-combine
// data, chunk sums, the schedule itself) is carved out of one fixed device
// array, `scratch`, that the library holds on each GPU until the process ends.
// The schedule of Algorithm 6 is written by a kernel from its closed form, so
// the call makes no host-to-device copy either; the launch sequence is that of
// dsmc_smooth (same kernels, heuristic tiles; results do not depend on tiles).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "dsmc.h"
#include "dsmc_host.h"
#include "dsmc_internal.h"
#include "dsmc_launch.h"

using namespace dsmc;

namespace {

constexpr size_t kScratchBytes = DSMC_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
constexpr int kMaxLevels = 32;

// The workspace of every dsmc_smooth_static call on this GPU.  In host code
// the name is a host-side stand-in: only the address returned by
// hipGetSymbolAddress (kept per device below) is used.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's copy of `scratch` (looked up once per device, with
// that device current).
int scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(DSMC_EUNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DSMC_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DSMC_OK;
}

// Levels of Algorithm 6 for K points: level l combines at the boundaries
// c = (2k + 1) 2^l < K, k = 0, 1, ...; ids run level by level.
struct Levels {
  int L = 0;
  int off[kMaxLevels + 1] = {};
  int cnt[kMaxLevels] = {};
};

Levels levels_of(int K) {
  Levels lv;
  int n = 0;
  for (int l = 0; l < kMaxLevels && (1L << l) < K; ++l) {
    const long w = 1L << l;
    lv.off[l] = n;
    lv.cnt[l] = (int)((K - w + 2 * w - 1) / (2 * w));  // #k with (2k + 1) w < K
    n += lv.cnt[l];
    lv.L = l + 1;
  }
  lv.off[lv.L] = n;
  return lv;
}

__device__ int node_id(const Levels& lv, int l, int k) { return lv.off[l] + k; }

// The combine that consumes the block starting at a = w 2^j of level j (the
// block is the window [w 2^j, (w + 1) 2^j) cut at K): at the first level where
// it has a neighbour it is the right block of the combine at a (w odd) or the
// left block of the combine at a + 2^j (w even); a block with no right
// neighbour passes up unchanged.  Returns 2 id + role, or -1 (root).
__device__ int consumer_of(const Levels& lv, int K, int j, long w) {
  for (; j < lv.L; ++j, w >>= 1) {
    if (w & 1) return 2 * node_id(lv, j, (int)((w - 1) >> 1)) + 1;
    if ((w + 1) * (1L << j) < K) return 2 * node_id(lv, j, (int)(w >> 1));
  }
  return -1;
}

__global__ void k_static_schedule(Levels lv, int K, NodeDesc* __restrict__ nodes,
                                  int32_t* __restrict__ series_of_t,
                                  int32_t* __restrict__ leaf_cons, SeriesDesc* __restrict__ series,
                                  SeriesDesc sd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *series = sd;
  if (i >= K) return;
  series_of_t[i] = 0;
  leaf_cons[i] = consumer_of(lv, K, 0, i);
  if (i >= K - 1) return;
  int l = 0;
  while (l + 1 < lv.L && i >= lv.off[l + 1]) ++l;
  const int k = i - lv.off[l];
  const long w = 1L << l;
  NodeDesc nd;
  nd.series = 0;
  nd.c = (int)((2L * k + 1) * w);
  nd.a = (int)(nd.c - w);
  nd.b = (int)((nd.c + w < K) ? nd.c + w : K);
  nd.lchild = (l == 0) ? -1 : node_id(lv, l - 1, 2 * k);
  const int s = nd.b - nd.c;  // right block [c, b): a leaf, or formed at level ceil(log2 s) - 1
  if (s == 1) {
    nd.rchild = -1;
  } else {
    int lr = 0;
    while ((1 << (lr + 1)) < s) ++lr;
    nd.rchild = node_id(lv, lr, nd.c >> (lr + 1));
  }
  const int cons = consumer_of(lv, K, l + 1, k);
  nd.consumer = cons < 0 ? -1 : cons >> 1;
  nd.role = cons < 0 ? 0 : (cons & 1);
  nodes[i] = nd;
}

// Bump allocator over the scratch array (offsets only; 256-byte aligned).
struct Carve {
  size_t used = 0;
  size_t take(size_t bytes) {
    const size_t at = used;
    used += (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
    return at;
  }
};

}  // namespace

extern "C" int dsmc_smooth_static(const dsmc_model_t* model, int N, int precision, uint64_t seed,
                                  const dsmc_output* out, void* stream) {
  if (!model || !model->dev) return fail(DSMC_EINVAL, "null model");
  if (N < 1 || N > DSMC_MAX_N) return fail(DSMC_EUNSUPPORTED, "N must be in 1..%d", DSMC_MAX_N);
  if (precision != DSMC_FP32 && precision != DSMC_FP64)
    return fail(DSMC_EUNSUPPORTED, "dsmc_smooth_static runs DSMC_FP32 or DSMC_FP64 (got %d)", precision);
  int rc = check_output(out);
  if (rc) return rc;
  const int K = model->K, dx = model->dx;
  const int DX = padded_dx(dx);
  const bool fp64 = precision == DSMC_FP64;
  const size_t R = fp64 ? 8 : 4;
  const int Npad = (N + kChunk - 1) / kChunk * kChunk, Nc = Npad / kChunk, NcP = (Nc + kGroup - 1) / kGroup * kGroup;
  const Levels lv = levels_of(K);
  const size_t TK = (size_t)K, Ns = (size_t)N;

  // ---- layout: per-run buffers, then as many combines' chunk sums as fit
  Carve cv;
  const size_t o_series = cv.take(sizeof(SeriesDesc));
  const size_t o_nodes = cv.take(TK * sizeof(NodeDesc));
  const size_t o_sot = cv.take(TK * sizeof(int32_t));
  const size_t o_cons = cv.take(TK * sizeof(int32_t));
  const size_t o_leafX = cv.take((size_t)dx * TK * Ns * R);
  const size_t o_leafW = cv.take(TK * Ns * R);
  const size_t o_leafL = cv.take(TK * sizeof(double));
  const size_t o_bmerged = cv.take(TK * sizeof(double));
  const size_t o_anc = out->ancestry ? 0 : cv.take(TK * 2 * Ns * sizeof(int32_t));
  const size_t o_zinc = out->logZ_inc ? 0 : cv.take(TK * sizeof(double));
  const size_t o_col = cv.take(TK * Npad * (DX + 1) * R);
  const size_t o_row = cv.take(TK * Npad * DX * R);
  const size_t o_alpha = cv.take(TK * Ns * R);
  const size_t o_bcol = cv.take(TK * sizeof(double));
  const size_t o_sfirst = cv.take(TK * Ns * sizeof(int32_t));
  const size_t o_slast = cv.take(TK * Ns * sizeof(int32_t));
  const size_t o_tcol = cv.take(TK * Ns * DX * R);
  const size_t o_tgq = cv.take(TK * Ns * sizeof(double));
  const size_t o_trow = cv.take(TK * Ns * DX * R);
  const size_t fixed = cv.used;
  const size_t NGS = (size_t)group_stride(NcP);
  const size_t per_node = 2 * (((Ns * NcP * R) + 255) & ~size_t(255)) + Ns * sizeof(double) +
                          Ns * sizeof(float) + Ns * NGS * sizeof(double) + 768;
  const int want_nodes = std::max(1, lv.cnt[0]);
  if (fixed + per_node > kScratchBytes)
    return fail(DSMC_EUNSUPPORTED,
                "K=%d, N=%d, d_x=%d needs %zu bytes of workspace; the static workspace holds %zu",
                K, N, dx, fixed + per_node, kScratchBytes);
  const int node_cap = (int)std::min<size_t>(want_nodes, (kScratchBytes - fixed) / per_node);
  const size_t o_P = cv.take((size_t)node_cap * Ns * NcP * R);
  const size_t o_Pr = cv.take((size_t)node_cap * Ns * NcP * R);
  const size_t o_Rsum = cv.take((size_t)node_cap * Ns * sizeof(double));
  const size_t o_Rshift = cv.take((size_t)node_cap * Ns * sizeof(float));
  const size_t o_Gs = cv.take((size_t)node_cap * Ns * NGS * sizeof(double));
  if (cv.used > kScratchBytes) return fail(DSMC_EUNSUPPORTED, "static workspace layout overflow");

  void* base = nullptr;
  rc = scratch_address(&base);
  if (rc) return rc;
  char* b = (char*)base;
  auto at = [b](size_t o) { return (void*)(b + o); };
  hipStream_t st = (hipStream_t)stream;

  SeriesDesc sd{};
  sd.model = model->dev;
  sd.seed = seed;
  sd.K = K;
  sd.base = 0;
  sd.root = K >= 2 ? lv.off[lv.L - 1] : -1;
  sd.anc = out->ancestry ? out->ancestry : (int32_t*)at(o_anc);
  sd.zinc = out->logZ_inc ? out->logZ_inc : (double*)at(o_zinc);
  sd.row_lse = out->row_lse;
  sd.status = out->status;
  sd.traj = out->traj;
  sd.logw = out->logw;
  sd.log_Z = out->log_Z;
  sd.leaf_x = out->leaf_x;
  sd.leaf_logw = out->leaf_logw;
  sd.leaf_logL = out->leaf_logL;
  sd.index = out->index;
  sd.star = nullptr;
  auto* d_series = (SeriesDesc*)at(o_series);
  auto* d_nodes = (NodeDesc*)at(o_nodes);
  auto* d_sot = (int32_t*)at(o_sot);
  auto* d_cons = (int32_t*)at(o_cons);
  k_static_schedule<<<(K + kBlock - 1) / kBlock, kBlock, 0, st>>>(lv, K, d_nodes, d_sot, d_cons,
                                                                  d_series, sd);
  HIP_TRY(hipGetLastError());

  NodeBufs nb{};
  nb.col = at(o_col);
  nb.row = at(o_row);
  nb.alpha = at(o_alpha);
  nb.bcol = (double*)at(o_bcol);
  nb.sfirst = (int32_t*)at(o_sfirst);
  nb.slast = (int32_t*)at(o_slast);
  nb.tcol = at(o_tcol);
  nb.tgq = (double*)at(o_tgq);
  nb.trow = at(o_trow);

  Timer untimed;
  launch_clear_status(d_series, 0, 1, st);
  LeafLaunch LL{};
  LL.fp64 = fp64;
  LL.DX = DX;
  LL.N = N;
  LL.Npad = Npad;
  LL.totalK = K;
  LL.row0 = 0;
  LL.rows = K;
  LL.d_series = d_series;
  LL.d_series_of_t = d_sot;
  LL.d_leaf_cons = d_cons;
  LL.d_nodes = d_nodes;
  LL.leafX = at(o_leafX);
  LL.leafW = at(o_leafW);
  LL.leafL = (double*)at(o_leafL);
  LL.bmerged = (double*)at(o_bmerged);
  LL.nb = nb;
  if (launch_leaves(LL, st, &untimed)) return fail(DSMC_EUNSUPPORTED, "no leaf kernel for d_x");
  HIP_TRY(hipGetLastError());
  for (int l = 0; l < lv.L; ++l) {
    for (int s0 = 0; s0 < lv.cnt[l]; s0 += node_cap) {
      const int nodes = std::min(node_cap, lv.cnt[l] - s0);
      LevelLaunch L{};
      L.fp64 = fp64;
      L.bf16 = false;
      L.DX = DX;
      L.node_list = nullptr;
      L.node0 = lv.off[l] + s0;
      L.nodes = nodes;
      L.N = N;
      L.Npad = Npad;
      L.Nc = Nc;
      L.NcP = NcP;
      L.totalK = K;
      L.d_nodes = d_nodes;
      L.d_series = d_series;
      L.leafX = LL.leafX;
      L.bmerged = LL.bmerged;
      L.P = at(o_P);
      L.Pr = at(o_Pr);
      L.Rsum = (double*)at(o_Rsum);
      L.Rshift = (float*)at(o_Rshift);
      L.Gs = (double*)at(o_Gs);
      L.force_rescue = false;
      L.rescue_count = nullptr;
      L.nb = nb;
      L.lazy = 0;
      L.lazy_param = 0;
      set_sample_shape(L);
      set_tile(L, heuristic_tile(nodes, N, Nc, DX < 8));
      if (launch_level(L, st, &untimed)) return fail(DSMC_EUNSUPPORTED, "no combine kernel for d_x");
      HIP_TRY(hipGetLastError());
    }
  }
  launch_output(LL, 0, 1, dx, st, &untimed);
  HIP_TRY(hipGetLastError());
  return DSMC_OK;
}
