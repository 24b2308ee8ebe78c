// Host side of the C ABI declared in include/dsmc.h: model validation (with the
// callback self-check) and upload, plans and their device workspace, the
// Algorithm 6 schedule, and the launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "dsmc.h"
#include "dsmc_host.h"
#include "dsmc_internal.h"
#include "dsmc_launch.h"

using namespace dsmc;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

int dsmc::fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

extern "C" const char* dsmc_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------- model

// Inverse of a lower-triangular matrix (forward substitution), fp64.
static bool tri_inverse(const double* L, int d, double* out) {
  std::fill(out, out + d * d, 0.0);
  for (int j = 0; j < d; ++j) {
    if (!(L[j * d + j] > 0.0) || !std::isfinite(L[j * d + j])) return false;
    out[j * d + j] = 1.0 / L[j * d + j];
    for (int i = j + 1; i < d; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[i * d + k] * out[k * d + j];
      out[i * d + j] = -s / L[i * d + i];
    }
  }
  return true;
}

static double log_norm(const double* L, int d) {
  double s = 0.0;
  for (int i = 0; i < d; ++i) s += std::log(L[i * d + i]);
  return -s - 0.5 * d * std::log(2.0 * M_PI);
}

static bool all_finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Sizes, kinds and parameters of a description (no callbacks, no device).
static int validate_desc(const dsmc_model_desc* d) {
  if (!d) return fail(DSMC_EINVAL, "null argument");
  const int K = d->K, dx = d->d_x, dy = d->d_y;
  if (K < 1) return fail(DSMC_EINVAL, "K must be >= 1 (got %d)", K);
  if (dx < 1 || dx > DSMC_MAX_DX) return fail(DSMC_EINVAL, "d_x must be in 1..%d", DSMC_MAX_DX);
  if (dy < 1) return fail(DSMC_EINVAL, "d_y must be >= 1");
  const bool complete = d->m0 && d->P0_chol && d->F && d->f && d->Q_chol && d->y && d->q_mean &&
                        d->q_chol && d->obs_kind != DSMC_OBS_NONE;
  if (!complete && d->callbacks)
    return fail(DSMC_EUNSUPPORTED,
                "the model is given by callbacks without a complete parametric (device) form; "
                "the GPU cannot run host callbacks");
  if (!d->m0 || !d->P0_chol || !d->F || !d->f || !d->Q_chol || !d->y || !d->q_mean || !d->q_chol)
    return fail(DSMC_EINVAL, "missing model array");
  if (d->obs_kind == DSMC_OBS_STOCH_VOL) {
    if (dx != 1 || dy != 1) return fail(DSMC_EINVAL, "stochastic volatility needs d_x = d_y = 1");
  } else if (d->obs_kind == DSMC_OBS_LINEAR_GAUSSIAN) {
    if (!d->H || !d->h || !d->R_chol) return fail(DSMC_EINVAL, "missing observation array");
  } else if (d->obs_kind == DSMC_OBS_BOX) {
    if (dy != 2 * dx) return fail(DSMC_EINVAL, "box potential needs d_y = 2 d_x");
  } else {
    return fail(DSMC_EINVAL, "unknown obs_kind %d", d->obs_kind);
  }
  if (d->weighting != DSMC_WEIGHT_LEAF_OBS && d->weighting != DSMC_WEIGHT_BOUNDARY_OBS)
    return fail(DSMC_EINVAL, "unknown weighting %d", d->weighting);
  if (d->proposal_kind != DSMC_PROPOSAL_GAUSSIAN && d->proposal_kind != DSMC_PROPOSAL_UNIFORM)
    return fail(DSMC_EINVAL, "unknown proposal_kind %d", d->proposal_kind);
  if (d->proposal_kind == DSMC_PROPOSAL_UNIFORM && dx > 4)
    return fail(DSMC_EINVAL, "uniform proposals need d_x <= 4");
  const size_t dd = (size_t)dx * dx;
  if (!all_finite(d->m0, dx) || !all_finite(d->P0_chol, dd) || !all_finite(d->F, dd) ||
      !all_finite(d->f, dx) || !all_finite(d->Q_chol, dd) ||
      !all_finite(d->q_mean, (size_t)K * dx) || !all_finite(d->q_chol, (size_t)K * dd))
    return fail(DSMC_EINVAL, "non-finite model parameter");
  return DSMC_OK;
}

// ---- host evaluation of the parametric form, for the callback self-check

// -1/2 || Linv (v) ||^2 for lower-triangular Linv [d][d].
static double neg_half_quad(const double* Linv, const double* v, int d) {
  double q = 0.0;
  for (int i = 0; i < d; ++i) {
    double z = 0.0;
    for (int j = 0; j <= i; ++j) z += Linv[i * d + j] * v[j];
    q += z * z;
  }
  return -0.5 * q;
}

namespace {
struct HostForm {
  const dsmc_model_desc* d;
  std::vector<double> P0i, Qi, Ri;
  double prior_ln = 0, trans_ln = 0, obs_ln = 0;

  bool init() {
    const int dx = d->d_x, dy = d->d_y;
    P0i.resize((size_t)dx * dx);
    Qi.resize((size_t)dx * dx);
    if (!tri_inverse(d->P0_chol, dx, P0i.data()) || !tri_inverse(d->Q_chol, dx, Qi.data()))
      return false;
    prior_ln = log_norm(d->P0_chol, dx);
    trans_ln = log_norm(d->Q_chol, dx);
    if (d->obs_kind == DSMC_OBS_LINEAR_GAUSSIAN) {
      Ri.resize((size_t)dy * dy);
      if (!tri_inverse(d->R_chol, dy, Ri.data())) return false;
      obs_ln = log_norm(d->R_chol, dy);
    }
    return true;
  }
  double log_prior(const double* x) const {
    const int dx = d->d_x;
    std::vector<double> v(dx);
    for (int i = 0; i < dx; ++i) v[i] = x[i] - d->m0[i];
    return neg_half_quad(P0i.data(), v.data(), dx) + prior_ln;
  }
  double log_transition(const double* xp, const double* x) const {
    const int dx = d->d_x;
    std::vector<double> v(dx);
    for (int i = 0; i < dx; ++i) {
      double m = d->f[i];
      for (int j = 0; j < dx; ++j) m += d->F[i * dx + j] * xp[j];
      v[i] = x[i] - m;
    }
    return neg_half_quad(Qi.data(), v.data(), dx) + trans_ln;
  }
  double log_observation(int t, const double* x) const {
    const int dx = d->d_x, dy = d->d_y;
    const double* y = d->y + (size_t)t * dy;
    if (d->obs_kind == DSMC_OBS_STOCH_VOL)
      return -0.5 * std::log(2.0 * M_PI) - 0.5 * x[0] - 0.5 * y[0] * y[0] * std::exp(-x[0]);
    if (d->obs_kind == DSMC_OBS_BOX) {
      for (int i = 0; i < dx; ++i)
        if (!(x[i] >= y[i] && x[i] <= y[dx + i])) return -INFINITY;
      return 0.0;
    }
    std::vector<double> v(dy);
    for (int i = 0; i < dy; ++i) {
      double m = d->h[i];
      for (int k = 0; k < dx; ++k) m += d->H[i * dx + k] * x[k];
      v[i] = y[i] - m;
    }
    return neg_half_quad(Ri.data(), v.data(), dy) + obs_ln;
  }
  // x = the draw of q_t made from variates z; returns log q_t(x)
  double proposal(int t, const double* z, double* x) const {
    const int dx = d->d_x;
    const double* qm = d->q_mean + (size_t)t * dx;
    const double* qc = d->q_chol + (size_t)t * dx * dx;
    if (d->proposal_kind == DSMC_PROPOSAL_UNIFORM) {
      double ln = 0.0;
      for (int i = 0; i < dx; ++i) {
        const double hw = qc[i * dx + i];
        x[i] = qm[i] + hw * (2.0 * z[i] - 1.0);
        ln -= std::log(2.0 * hw);
      }
      return ln;
    }
    std::vector<double> qi((size_t)dx * dx), v(dx);
    tri_inverse(qc, dx, qi.data());
    for (int i = 0; i < dx; ++i) {
      double s = qm[i];
      for (int j = 0; j <= i; ++j) s += qc[i * dx + j] * z[j];
      x[i] = s;
      v[i] = s - qm[i];
    }
    return neg_half_quad(qi.data(), v.data(), dx) + log_norm(qc, dx);
  }
};

// Fixed generator of the check points (splitmix64; any deterministic points do).
struct CheckRng {
  uint64_t s = 0x9E3779B97F4A7C15ull;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double unif() { return (double)(next() >> 11) * 0x1p-53; }
  double normal() {
    const double u1 = ((double)(next() >> 11) + 1.0) * 0x1p-53, u2 = unif();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
  }
};

bool close_enough(double got, double want) {
  if (std::isinf(want) || std::isinf(got)) return got == want;
  if (std::isnan(got) || std::isnan(want)) return false;
  return std::fabs(got - want) <= 1e-9 * std::max(1.0, std::fabs(want));
}
}  // namespace

// Evaluate the callbacks at 256 check points and compare with the parametric form.
static int self_check(const dsmc_model_desc* d) {
  const dsmc_model_callbacks* cb = d->callbacks;
  HostForm hf{d};
  if (!hf.init()) return fail(DSMC_EINVAL, "bad Cholesky factor");
  const int K = d->K, dx = d->d_x;
  constexpr int kTimes = 16, kPer = 16;
  CheckRng rng;
  const bool unif = d->proposal_kind == DSMC_PROPOSAL_UNIFORM;
  std::vector<double> z(kPer * dx), zp(kPer * dx), x(kPer * dx), xp(kPer * dx), want(kPer),
      got(kPer), gx(kPer * dx), lq(kPer);
  for (int j = 0; j < kTimes; ++j) {
    const int t = (int)(((long)j * (K - 1)) / (kTimes - 1));
    for (auto& v : z) v = unif ? rng.unif() : rng.normal();
    for (auto& v : zp) v = unif ? rng.unif() : rng.normal();
    std::vector<double> lqw(kPer);
    for (int i = 0; i < kPer; ++i) lqw[i] = hf.proposal(t, &z[i * dx], &x[i * dx]);
    const int tp = t >= 1 ? t - 1 : 0;
    for (int i = 0; i < kPer; ++i) hf.proposal(tp, &zp[i * dx], &xp[i * dx]);
    auto mismatch = [&](const char* what, int i) {
      return fail(DSMC_EINVAL,
                  "device form disagrees with the %s callback at t=%d, point %d: %.17g (callback) "
                  "vs %.17g (device form)",
                  what, t, i, got[i], want[i]);
    };
    if (cb->proposal) {
      if (cb->proposal(cb->ctx, t, kPer, z.data(), gx.data(), lq.data()))
        return fail(DSMC_ECALLBACK, "proposal callback failed at t=%d", t);
      for (int i = 0; i < kPer; ++i) {
        for (int k = 0; k < dx; ++k)
          if (!close_enough(gx[i * dx + k], x[i * dx + k]))
            return fail(DSMC_EINVAL,
                        "device form disagrees with the proposal callback at t=%d, point %d, "
                        "coordinate %d: %.17g (callback) vs %.17g (device form)",
                        t, i, k, gx[i * dx + k], x[i * dx + k]);
        got[i] = lq[i];
        want[i] = lqw[i];
        if (!close_enough(got[i], want[i])) return mismatch("proposal density", i);
      }
    }
    if (cb->log_prior && j == 0) {
      if (cb->log_prior(cb->ctx, kPer, x.data(), got.data()))
        return fail(DSMC_ECALLBACK, "log_prior callback failed");
      for (int i = 0; i < kPer; ++i) {
        want[i] = hf.log_prior(&x[i * dx]);
        if (!close_enough(got[i], want[i])) return mismatch("log_prior", i);
      }
    }
    if (cb->log_observation) {
      if (cb->log_observation(cb->ctx, t, kPer, x.data(), got.data()))
        return fail(DSMC_ECALLBACK, "log_observation callback failed at t=%d", t);
      for (int i = 0; i < kPer; ++i) {
        want[i] = hf.log_observation(t, &x[i * dx]);
        if (!close_enough(got[i], want[i])) return mismatch("log_observation", i);
      }
    }
    if (cb->log_transition && K >= 2 && t >= 1) {
      if (cb->log_transition(cb->ctx, t, kPer, xp.data(), x.data(), got.data()))
        return fail(DSMC_ECALLBACK, "log_transition callback failed at t=%d", t);
      for (int i = 0; i < kPer; ++i) {
        want[i] = hf.log_transition(&xp[i * dx], &x[i * dx]);
        if (!close_enough(got[i], want[i])) return mismatch("log_transition", i);
      }
    }
  }
  return DSMC_OK;
}

extern "C" int dsmc_model_check(const dsmc_model_desc* d) {
  int rc = validate_desc(d);
  if (rc) return rc;
  if (!d->callbacks) return DSMC_OK;
  return self_check(d);
}

extern "C" int dsmc_model_create(const dsmc_model_desc* d, dsmc_model_t** out) {
  if (!d || !out) return fail(DSMC_EINVAL, "null argument");
  *out = nullptr;
  int rc = dsmc_model_check(d);
  if (rc) return rc;
  const int K = d->K, dx = d->d_x, dy = d->d_y;
  const size_t dd = (size_t)dx * dx;

  // host copies of every array the device needs
  std::vector<double> m0(d->m0, d->m0 + dx), P0i(dd), F(d->F, d->F + dd), f(d->f, d->f + dx),
      Qi(dd), H, y, qm(d->q_mean, d->q_mean + (size_t)K * dx),
      qc(d->q_chol, d->q_chol + (size_t)K * dd), qi((size_t)K * dd), qln(K), Wcol(dd), Wrow(dd),
      woff(dx);
  if (!tri_inverse(d->P0_chol, dx, P0i.data())) return fail(DSMC_EINVAL, "bad P0_chol");
  if (!tri_inverse(d->Q_chol, dx, Qi.data())) return fail(DSMC_EINVAL, "bad Q_chol");
  for (int t = 0; t < K; ++t) {
    if (!tri_inverse(d->q_chol + (size_t)t * dd, dx, qi.data() + (size_t)t * dd))
      return fail(DSMC_EINVAL, "bad q_chol at t=%d", t);
    qln[t] = log_norm(d->q_chol + (size_t)t * dd, dx);
    if (d->proposal_kind == DSMC_PROPOSAL_UNIFORM) {  // box q_mean +- diag(q_chol)
      double s = 0.0;
      for (int i = 0; i < dx; ++i) s -= std::log(2.0 * d->q_chol[(size_t)t * dd + i * dx + i]);
      qln[t] = s;
    }
  }
  double obs_ln = 0.0;
  if (d->obs_kind == DSMC_OBS_LINEAR_GAUSSIAN) {
    std::vector<double> Ri((size_t)dy * dy);
    if (!tri_inverse(d->R_chol, dy, Ri.data())) return fail(DSMC_EINVAL, "bad R_chol");
    obs_ln = log_norm(d->R_chol, dy);
    H.assign((size_t)dy * dx, 0.0);  // R^{-1/2} H
    for (int i = 0; i < dy; ++i)
      for (int k = 0; k < dx; ++k) {
        double s = 0.0;
        for (int j = 0; j <= i; ++j) s += Ri[i * dy + j] * d->H[j * dx + k];
        H[i * dx + k] = s;
      }
    y.assign((size_t)K * dy, 0.0);  // R^{-1/2} (y_t - h)
    for (int t = 0; t < K; ++t)
      for (int i = 0; i < dy; ++i) {
        double s = 0.0;
        for (int j = 0; j <= i; ++j) s += Ri[i * dy + j] * (d->y[(size_t)t * dy + j] - d->h[j]);
        y[(size_t)t * dy + i] = s;
      }
  } else {
    H.assign(1, 0.0);
    y.assign(d->y, d->y + (size_t)K * dy);
  }
  // whitening: ||kappa Q^{-1/2} (x_R - F x_L - f)||^2 = (log2 e / 2) * quadratic form
  const double kappa = std::sqrt(0.5 / std::log(2.0));
  for (int i = 0; i < dx; ++i) {
    double so = 0.0;
    for (int j = 0; j < dx; ++j) {
      Wcol[i * dx + j] = kappa * Qi[i * dx + j];
      double s = 0.0;
      for (int k = 0; k < dx; ++k) s += Qi[i * dx + k] * F[k * dx + j];
      Wrow[i * dx + j] = kappa * s;
      so += Qi[i * dx + j] * f[j];
    }
    woff[i] = kappa * so;
  }

  // pack: header, then arrays (each 256-byte aligned)
  std::vector<double> P0c(d->P0_chol, d->P0_chol + dd), Qc(d->Q_chol, d->Q_chol + dd);
  const int DXp = padded_dx(dx);
  std::vector<double> lrec(DXp >= 8 ? leafrec_size(K, DXp) : 0, 0.0);  // filled on the device
  std::vector<const std::vector<double>*> arrs = {&m0, &P0i, &F,  &f,  &Qi,  &H,    &y,
                                                  &qm, &qc,  &qi, &qln, &Wcol, &Wrow, &woff,
                                                  &P0c, &Qc, &lrec};
  size_t off = (sizeof(DevModel) + 255) & ~size_t(255);
  std::vector<size_t> offs;
  for (auto* a : arrs) {
    offs.push_back(off);
    off += (a->size() * sizeof(double) + 255) & ~size_t(255);
  }
  std::vector<char> blob(off, 0);
  auto* m = new dsmc_model;
  m->K = K;
  m->dx = dx;
  hipError_t e = hipMalloc(&m->dmem, off);
  if (e != hipSuccess) {
    delete m;
    return fail(DSMC_ENOMEM, "hipMalloc(model): %s", hipGetErrorString(e));
  }
  char* base = (char*)m->dmem;
  for (size_t i = 0; i < arrs.size(); ++i)
    std::memcpy(blob.data() + offs[i], arrs[i]->data(), arrs[i]->size() * sizeof(double));
  DevModel hdr{};
  hdr.K = K;
  hdr.dx = dx;
  hdr.dy = dy;
  hdr.obs_kind = d->obs_kind;
  hdr.prop_kind = d->proposal_kind;
  hdr.weighting = d->weighting;
  auto P = [&](int i) { return (const double*)(base + offs[i]); };
  hdr.m0 = P(0);
  hdr.P0_inv = P(1);
  hdr.prior_lognorm = log_norm(d->P0_chol, dx);
  hdr.F = P(2);
  hdr.f = P(3);
  hdr.Q_inv = P(4);
  hdr.trans_lognorm = log_norm(d->Q_chol, dx);
  hdr.H = P(5);
  hdr.y = P(6);
  hdr.obs_lognorm = obs_ln;
  hdr.q_mean = P(7);
  hdr.q_chol = P(8);
  hdr.q_inv = P(9);
  hdr.q_lognorm = P(10);
  hdr.Wcol = P(11);
  hdr.Wrow = P(12);
  hdr.wcol_off = P(13);
  hdr.P0_chol = P(14);
  hdr.Q_chol = P(15);
  hdr.leafrec = lrec.empty() ? nullptr : P(16);
  std::memcpy(blob.data(), &hdr, sizeof hdr);
  e = hipMemcpy(m->dmem, blob.data(), off, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    hipFree(m->dmem);
    delete m;
    return fail(DSMC_EDEVICE, "hipMemcpy(model): %s", hipGetErrorString(e));
  }
  m->dev = (DevModel*)m->dmem;
  m->hdr = hdr;
  if (hdr.leafrec) {
    launch_leaf_records(m->dev, (double*)hdr.leafrec, K, DXp, nullptr);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
      hipFree(m->dmem);
      delete m;
      return fail(DSMC_EDEVICE, "leaf records: %s", hipGetErrorString(e));
    }
  }
  m->dy = dy;
  m->obs_kind = d->obs_kind;
  m->prop_kind = d->proposal_kind;
  *out = m;
  return DSMC_OK;
}

extern "C" void dsmc_model_destroy(dsmc_model_t* m) {
  if (!m) return;
  (void)hipFree(m->dmem);
  if (m->pit_ws) (void)hipFree(m->pit_ws);
  delete m;
}

extern "C" int dsmc_model_K(const dsmc_model_t* m) { return m ? m->K : -1; }

// -------------------------------------------------------------------- plan

struct dsmc_plan_impl {
  dsmc_plan_desc d{};
  int DX = 1;
  bool fp64 = false;
  bool bf16 = false;
  size_t rsz = 4;
  hipStream_t stream = nullptr;
  int Npad = 0, Nc = 0, NcP = 0;
  int node_cap = 0;  // combines per launch slice
  bool autotune = false;
  int lazy_param = 0;  // MH steps or rejection cap actually used (defaults resolved)
  // device workspace: per time row
  void* leafX = nullptr;
  void* leafW = nullptr;
  double* leafL = nullptr;
  double* bmerged = nullptr;
  int32_t* anc = nullptr;
  double* zinc = nullptr;
  // per combine
  NodeBufs nb{};
  // per launch slice
  void* P = nullptr;
  void* Pr = nullptr;
  double* Rsum = nullptr;
  float* Rshift = nullptr;
  double* Gs = nullptr;                      // chunk-group sums of rows under column splits
  unsigned long long* d_rescued = nullptr;  // profiling: rescued-row counter
  // schedule
  NodeDesc* d_nodes = nullptr;
  int32_t* d_series_of_t = nullptr;
  int32_t* d_leaf_cons = nullptr;
  SeriesDesc* d_series = nullptr;
  int series_cap = 0;
  // pinned staging
  NodeDesc* h_nodes = nullptr;
  int32_t* h_series_of_t = nullptr;
  int32_t* h_leaf_cons = nullptr;
  SeriesDesc* h_series = nullptr;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  // schedule of the last call and the K list it was built for
  std::vector<int> sched_K;
  std::vector<int> roots;
  // hipGraph of one batch shape (DSMC_PLAN_GRAPH)
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int> graph_K;
  const SeriesDesc* graph_series = nullptr;
  std::vector<int> level_off, level_cnt;
  int total_nodes = 0;
  // rows-kernel tile per launch size (autotuned or heuristic)
  std::map<int, TileChoice> tiles;
  // profiling
  Timer timer;
  double last_pairs = 0.0;
};

static void plan_free(dsmc_plan_t* p) {
  void* dev[] = {p->leafX, p->leafW, p->leafL, p->bmerged, p->anc, p->zinc, p->nb.col, p->nb.row,
                 p->nb.alpha, p->nb.bcol, p->nb.sfirst, p->nb.slast, p->nb.colh, p->nb.colb,
                 p->nb.rowh, p->nb.rown, p->nb.tcol, p->nb.tgq, p->nb.trow, p->nb.tcolh,
                 p->nb.tcoln, p->nb.trowh, p->nb.trown, p->P, p->Pr, p->Rsum, p->Rshift,
                 p->Gs, p->d_rescued, p->d_nodes, p->d_series_of_t, p->d_leaf_cons,
                 p->d_series};
  for (void* q : dev) (void)hipFree(q);
  void* host[] = {p->h_nodes, p->h_series_of_t, p->h_leaf_cons, p->h_series};
  for (void* q : host) (void)hipHostFree(q);
  if (p->staged) (void)hipEventDestroy(p->staged);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
}

int dsmc::padded_dx(int dx) {
  int q = 1;
  while (q < dx) q <<= 1;
  return q;
}

// Failure injection (dsmc_debug_fail_allocation): workspace allocations left
// before the one that fails; -1 when off.
static std::atomic<int> g_fail_alloc{-1};

static bool take_injected_failure() {
  int k = g_fail_alloc.load();
  while (k >= 0) {
    if (g_fail_alloc.compare_exchange_weak(k, k - 1)) return k == 0;
  }
  return false;
}

extern "C" int dsmc_debug_fail_allocation(int k) {
  g_fail_alloc.store(k < 0 ? -1 : k);
  return DSMC_OK;
}

extern "C" int dsmc_plan(const dsmc_plan_desc* d, dsmc_plan_t** out) {
  if (!d || !out) return fail(DSMC_EINVAL, "null argument");
  *out = nullptr;
  if (d->N < 1 || d->N > DSMC_MAX_N) return fail(DSMC_EUNSUPPORTED, "N must be in 1..%d", DSMC_MAX_N);
  if (d->d_x < 1 || d->d_x > DSMC_MAX_DX) return fail(DSMC_EUNSUPPORTED, "d_x must be in 1..%d", DSMC_MAX_DX);
  if (d->max_K < 1) return fail(DSMC_EINVAL, "max_K must be >= 1");
  if (d->precision != DSMC_FP32 && d->precision != DSMC_FP64 && d->precision != DSMC_BF16)
    return fail(DSMC_EUNSUPPORTED, "precision %d not supported", d->precision);
  if (d->precision == DSMC_BF16 && padded_dx(d->d_x) < 16)
    return fail(DSMC_EUNSUPPORTED, "DSMC_BF16 needs d_x >= 9 (got %d)", d->d_x);
  if (d->resampling != DSMC_RESAMPLE_EXACT && d->resampling != DSMC_RESAMPLE_MH &&
      d->resampling != DSMC_RESAMPLE_RS)
    return fail(DSMC_EINVAL, "resampling %d not supported", d->resampling);
  if (d->lazy_param < 0) return fail(DSMC_EINVAL, "lazy_param must be >= 0");
  if (d->precision == DSMC_BF16 && d->resampling != DSMC_RESAMPLE_EXACT)
    return fail(DSMC_EUNSUPPORTED, "DSMC_BF16 selects the matrix-core pair rows, which lazy plans do not run");
  auto* p = new dsmc_plan_t;
  p->d = *d;
  if (p->d.max_total_K < p->d.max_K) p->d.max_total_K = p->d.max_K;
  p->DX = padded_dx(d->d_x);
  p->fp64 = d->precision == DSMC_FP64;
  p->lazy_param = d->lazy_param ? d->lazy_param
                                : (d->resampling == DSMC_RESAMPLE_MH ? DSMC_MH_STEPS_DEFAULT
                                                                     : DSMC_RS_CAP_DEFAULT);
  p->bf16 = d->precision == DSMC_BF16;
  p->rsz = p->fp64 ? 8 : 4;
  p->stream = (hipStream_t)d->stream;
  p->timer.on = (d->flags & DSMC_PLAN_PROFILE) != 0;
  p->autotune = (d->flags & DSMC_PLAN_AUTOTUNE) != 0;
  p->use_graph = (d->flags & DSMC_PLAN_GRAPH) != 0;
  const int N = d->N;
  p->Npad = (N + kChunk - 1) / kChunk * kChunk;
  p->Nc = p->Npad / kChunk;
  p->NcP = (p->Nc + kGroup - 1) / kGroup * kGroup;
  const size_t TK = (size_t)p->d.max_total_K;
  const size_t max_nodes = std::max<size_t>(1, TK / 2);
  const size_t per_node_P = 2 * (size_t)N * p->NcP * p->rsz + (size_t)N * (sizeof(double) + sizeof(float));
  const size_t cap_by_mem = std::max<size_t>(1, ((size_t)2 << 30) / per_node_P);
  p->node_cap = (int)std::min(max_nodes, cap_by_mem);
  const size_t nc = (size_t)p->node_cap;
  const size_t R = p->rsz, DXp = (size_t)p->DX;
  int rc = DSMC_OK;
  struct A {
    void** ptr;
    size_t bytes;
    const char* what;
  } allocs[] = {
      {&p->leafX, (size_t)d->d_x * TK * N * R, "leaf particles"},
      {&p->leafW, TK * N * R, "leaf weights"},
      {(void**)&p->leafL, TK * sizeof(double), "leaf log L"},
      {(void**)&p->bmerged, TK * sizeof(double), "column bounds"},
      {(void**)&p->anc, TK * 2 * N * sizeof(int32_t), "ancestry"},
      {(void**)&p->zinc, TK * sizeof(double), "increments"},
      {&p->nb.col, TK * p->Npad * (DXp + 1) * R, "column data"},
      {&p->nb.row, TK * p->Npad * DXp * R, "row data"},
      {&p->nb.alpha, TK * N * R, "row weights"},
      {(void**)&p->nb.bcol, TK * sizeof(double), "column shifts"},
      {(void**)&p->nb.sfirst, TK * N * sizeof(int32_t), "first-time ancestry"},
      {(void**)&p->nb.slast, TK * N * sizeof(int32_t), "last-time ancestry"},
      {&p->nb.tcol, TK * N * DXp * R, "column table"},
      {(void**)&p->nb.tgq, TK * N * sizeof(double), "proposal table"},
      {&p->nb.trow, TK * N * DXp * R, "row table"},
      {&p->P, nc * N * p->NcP * R, "chunk sums"},
      {&p->Pr, nc * N * p->NcP * R, "rescued chunk sums"},
      {(void**)&p->Rsum, nc * N * sizeof(double), "row sums"},
      {(void**)&p->Rshift, nc * N * sizeof(float), "row shifts"},
      {(void**)&p->Gs, nc * N * group_stride(p->NcP) * sizeof(double), "chunk-group sums"},
      {(void**)&p->d_nodes, TK * sizeof(NodeDesc), "schedule"},
      {(void**)&p->d_series_of_t, TK * sizeof(int32_t), "series map"},
      {(void**)&p->d_leaf_cons, TK * sizeof(int32_t), "leaf consumers"},
  };
  std::vector<A> all(std::begin(allocs), std::end(allocs));
  if (p->timer.on) all.push_back({(void**)&p->d_rescued, sizeof(unsigned long long), "rescue counter"});
  if (p->bf16) {
    // split operands: 2 DX bf16 values (hi, then lo) per particle
    all.push_back({(void**)&p->nb.colh, TK * p->Npad * DXp * 4, "bf16 column operands"});
    all.push_back({(void**)&p->nb.colb, TK * p->Npad * sizeof(float), "column norms"});
    all.push_back({(void**)&p->nb.rowh, TK * p->Npad * DXp * 4, "bf16 row operands"});
    all.push_back({(void**)&p->nb.rown, TK * p->Npad * sizeof(float), "row norms"});
    all.push_back({(void**)&p->nb.tcolh, TK * N * DXp * 4, "bf16 column table"});
    all.push_back({(void**)&p->nb.tcoln, TK * N * sizeof(float), "column table norms"});
    all.push_back({(void**)&p->nb.trowh, TK * N * DXp * 4, "bf16 row table"});
    all.push_back({(void**)&p->nb.trown, TK * N * sizeof(float), "row table norms"});
  }
  for (auto& a : all) {
    hipError_t e = take_injected_failure() ? hipErrorOutOfMemory
                                           : hipMalloc(a.ptr, std::max<size_t>(a.bytes, 256));
    if (e != hipSuccess) {
      rc = fail(DSMC_ENOMEM, "hipMalloc(%s, %zu B): %s", a.what, a.bytes, hipGetErrorString(e));
      plan_free(p);
      delete p;
      return rc;
    }
  }
  if (hipHostMalloc((void**)&p->h_nodes, TK * sizeof(NodeDesc), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p->h_series_of_t, TK * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p->h_leaf_cons, TK * sizeof(int32_t), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&p->staged, hipEventDisableTiming) != hipSuccess ||
      (p->use_graph && hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)) {
    plan_free(p);
    delete p;
    return fail(DSMC_ENOMEM, "host staging allocation failed");
  }
  if (p->d_rescued) {
    const unsigned long long zero = 0;
    if (hipMemcpy(p->d_rescued, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) {
      plan_free(p);
      delete p;
      return fail(DSMC_EDEVICE, "rescue counter initialisation failed");
    }
  }
  *out = p;
  return DSMC_OK;
}

extern "C" void dsmc_plan_destroy(dsmc_plan_t* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->stream);
  plan_free(p);
  delete p;
}

static int ensure_series_cap(dsmc_plan_t* p, int B) {
  if (B <= p->series_cap) return DSMC_OK;
  if (p->staged_pending) HIP_TRY(hipEventSynchronize(p->staged));
  HIP_TRY(hipStreamSynchronize(p->stream));
  (void)hipFree(p->d_series);
  (void)hipHostFree(p->h_series);
  p->d_series = nullptr;
  p->h_series = nullptr;
  int cap = std::max(B, 2 * p->series_cap);
  HIP_TRY(hipMalloc((void**)&p->d_series, (size_t)cap * sizeof(SeriesDesc)));
  HIP_TRY(hipHostMalloc((void**)&p->h_series, (size_t)cap * sizeof(SeriesDesc), hipHostMallocDefault));
  p->series_cap = cap;
  return DSMC_OK;
}

// Algorithm 6 for every series.  Blocks start as single time points; at each
// level adjacent blocks (2k, 2k+1) are merged by one combine and a trailing
// block without a right neighbour is kept as it is.  Combines get ids level
// by level (all series of a level contiguous), and each records the combine
// that formed its left and right blocks and the combine that consumes the
// block it forms.
static void build_schedule(dsmc_plan_t* p, const std::vector<int>& Ks, const std::vector<int>& bases) {
  struct Blk {
    int a, b, former;
  };
  const int B = (int)Ks.size();
  std::vector<std::vector<Blk>> blocks(B);
  for (int s = 0; s < B; ++s) {
    blocks[s].reserve(Ks[s]);
    for (int t = 0; t < Ks[s]; ++t) {
      blocks[s].push_back({t, t + 1, -1});
      p->h_series_of_t[bases[s] + t] = s;
      p->h_leaf_cons[bases[s] + t] = -1;
    }
  }
  p->level_off.clear();
  p->level_cnt.clear();
  int n = 0;
  for (;;) {
    bool any = false;
    for (int s = 0; s < B; ++s) any |= blocks[s].size() > 1;
    if (!any) break;
    p->level_off.push_back(n);
    for (int s = 0; s < B; ++s) {
      auto& bl = blocks[s];
      if (bl.size() <= 1) continue;
      std::vector<Blk> nxt;
      nxt.reserve((bl.size() + 1) / 2);
      for (size_t k = 0; k < bl.size(); k += 2) {
        if (k + 1 == bl.size()) {
          nxt.push_back(bl[k]);
          continue;
        }
        const Blk& L = bl[k];
        const Blk& R = bl[k + 1];
        const int id = n++;
        NodeDesc nd;
        nd.series = s;
        nd.a = L.a;
        nd.c = R.a;
        nd.b = R.b;
        nd.lchild = L.former;
        nd.rchild = R.former;
        nd.consumer = -1;
        nd.role = 0;
        p->h_nodes[id] = nd;
        if (L.former >= 0) {
          p->h_nodes[L.former].consumer = id;
          p->h_nodes[L.former].role = 0;
        } else {
          p->h_leaf_cons[bases[s] + L.a] = 2 * id;
        }
        if (R.former >= 0) {
          p->h_nodes[R.former].consumer = id;
          p->h_nodes[R.former].role = 1;
        } else {
          p->h_leaf_cons[bases[s] + R.a] = 2 * id + 1;
        }
        nxt.push_back({L.a, R.b, id});
      }
      bl.swap(nxt);
    }
    p->level_cnt.push_back(n - p->level_off.back());
  }
  p->total_nodes = n;
  p->roots.assign(B, -1);
  for (int s = 0; s < B; ++s) p->roots[s] = blocks[s][0].former;
}

int dsmc::check_output(const dsmc_output* o) {
  if (!o) return fail(DSMC_EINVAL, "null output");
  if (!o->traj || !o->log_Z || !o->status)
    return fail(DSMC_EINVAL, "output traj, log_Z and status are required");
  return DSMC_OK;
}

// Column splits that bring a launch to about `want` waves (8 waves per SIMD).
// With one split the rows kernel also forms the row sums; with more, the
// sampler re-reads the chunk sums to form them.
int dsmc::pick_cs(int nodes, int N, int Nc, int rpl, int W) {
  const long rb = (N + 64L * rpl * W - 1) / (64L * rpl * W);
  const long waves = (long)nodes * rb * W;
  const long want = 8192;
  const long cs = (want + waves - 1) / waves;
  return (int)std::max<long>(1, std::min<long>(cs, Nc));
}

// Heuristic rows-kernel tile (times of every level of the headline workload on
// MI355X under each tile picked these thresholds): four rows per lane when the
// level has at least 2 M rows, two down to 128 K rows, else one row per lane;
// four waves per workgroup; and when the level's waves cannot fill the chip,
// column splits up to about 8192 waves (split_ok: d_x < 8; wider rows stay
// whole so that a wave can redo its rows with exact shifts).
TileChoice dsmc::heuristic_tile(int nodes, int N, int Nc, bool split_ok) {
  const long rows = (long)nodes * N;
  const int rpl = rows >= (2L << 20) ? 4 : (rows >= (128L << 10) ? 2 : 1);
  int W = 4;
  while (W > 1 && 64 * rpl * W > N) W >>= 1;
  const long waves = (long)nodes * ((N + 64L * rpl * W - 1) / (64L * rpl * W)) * W;
  return {rpl, W, (split_ok && waves < 4096) ? pick_cs(nodes, N, Nc, rpl, W) : 1};
}

void dsmc::set_tile(LevelLaunch& L, TileChoice tc) {
  L.RPL = tc.RPL;
  L.W = tc.W;
  L.RB = (L.N + 64 * tc.RPL * tc.W - 1) / (64 * tc.RPL * tc.W);
  L.KC = ((L.Nc + tc.CS - 1) / tc.CS + kGroup - 1) / kGroup * kGroup;  // whole chunk groups
  L.CS = (L.Nc + L.KC - 1) / L.KC;
}

// Time every (rows per lane, waves per workgroup) candidate, each with the
// column splits that fill the chip, on this launch's real inputs, and keep
// the fastest.  A trial runs the whole level (pair rows and sampling): the
// sampler's cost also depends on the tile (with column splits it adds the
// group sums of every row).  Re-running a level
// rewrites the same values (its kernels never modify their own inputs), and
// the tile does not change any result.
static TileChoice autotune_tile(dsmc_plan_t* p, LevelLaunch L) {
  const bool split_ok = L.DX < 8;
  const TileChoice heur = heuristic_tile(L.nodes, L.N, L.Nc, split_ok);
  TileChoice best = heur;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return best;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return best;
  }
  auto waves = [&](const TileChoice& tc) {
    const long rb = (L.N + 64L * tc.RPL * tc.W - 1) / (64L * tc.RPL * tc.W);
    return (long)L.nodes * rb * tc.CS * tc.W;
  };
  // a level time: the first run loads the kernels' code, the best of the next four counts
  auto time_level = [&](const TileChoice& tc, float* ms) {
    set_tile(L, tc);
    *ms = 1e30f;
    Timer untimed;
    for (int rep = 0; rep < 5; ++rep) {
      float t = 0.0f;
      if (hipEventRecord(e0, p->stream) != hipSuccess || launch_level(L, p->stream, &untimed) != 0 ||
          hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        return false;
      if (rep > 0) *ms = std::min(*ms, t);
    }
    return true;
  };
  float heur_ms = 1e30f;
  if (!time_level(heur, &heur_ms)) heur_ms = 1e30f;
  float best_ms = heur_ms;
  const long min_waves = std::min<long>(1024, waves(heur));
  const int rpls[3] = {1, 2, 4};
  const int ws[3] = {1, 2, 4};
  for (int rpl : rpls)
    for (int w : ws)
      for (int split = 0; split < 2; ++split) {
        if (64 * rpl * w > 2 * L.N && !(rpl == 1 && w == 1)) continue;
        if (split && !split_ok) continue;
        const TileChoice tc{rpl, w, split ? pick_cs(L.nodes, L.N, L.Nc, rpl, w) : 1};
        if (split && tc.CS == 1) continue;
        if (tc.RPL == heur.RPL && tc.W == heur.W && tc.CS == heur.CS) continue;
        // tiles with fewer waves than the heuristic's (at most 1024) leave
        // most SIMDs idle or with one long wave each; they are not tried
        if (waves(tc) < min_waves) continue;
        float ms = 0.0f;
        // a candidate replaces the heuristic tile only when clearly faster
        if (time_level(tc, &ms) && ms < 0.9f * heur_ms && ms < best_ms) {
          best_ms = ms;
          best = tc;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

void dsmc::build_series_schedule(int K, int series, int node_base, std::vector<NodeDesc>& nodes,
                                 std::vector<int>& lvl_off, std::vector<int>& lvl_cnt,
                                 std::vector<int32_t>& leaf_cons, int* root) {
  struct Blk {
    int a, b, former;
  };
  std::vector<Blk> bl;
  bl.reserve(K);
  for (int t = 0; t < K; ++t) bl.push_back({t, t + 1, -1});
  leaf_cons.assign(K, -1);
  lvl_off.clear();
  lvl_cnt.clear();
  const size_t first = nodes.size();
  int n = 0;
  while (bl.size() > 1) {
    lvl_off.push_back(n);
    std::vector<Blk> nxt;
    nxt.reserve((bl.size() + 1) / 2);
    for (size_t k = 0; k < bl.size(); k += 2) {
      if (k + 1 == bl.size()) {
        nxt.push_back(bl[k]);
        continue;
      }
      const Blk L = bl[k], R = bl[k + 1];
      const int id = node_base + n++;
      NodeDesc nd;
      nd.series = series;
      nd.a = L.a;
      nd.c = R.a;
      nd.b = R.b;
      nd.lchild = L.former;
      nd.rchild = R.former;
      nd.consumer = -1;
      nd.role = 0;
      nodes.push_back(nd);
      if (L.former >= 0) {
        nodes[first + (L.former - node_base)].consumer = id;
        nodes[first + (L.former - node_base)].role = 0;
      } else {
        leaf_cons[L.a] = 2 * id;
      }
      if (R.former >= 0) {
        nodes[first + (R.former - node_base)].consumer = id;
        nodes[first + (R.former - node_base)].role = 1;
      } else {
        leaf_cons[R.a] = 2 * id + 1;
      }
      nxt.push_back({L.a, R.b, id});
    }
    bl.swap(nxt);
    lvl_cnt.push_back(n - lvl_off.back());
  }
  *root = bl.empty() ? -1 : bl[0].former;
}

PoolSizes dsmc::pool_sizes(int N, int DX, int dx_alloc, size_t rsz) {
  const size_t Npad = (size_t)(N + kChunk - 1) / kChunk * kChunk;
  const size_t Nc = Npad / kChunk, NcP = (Nc + kGroup - 1) / kGroup * kGroup;
  PoolSizes ps;
  ps.per_row = (size_t)dx_alloc * N * rsz + N * rsz + 2 * sizeof(double)  // particles, weights, log L, bound
               + 2 * N * sizeof(int32_t) + sizeof(double)                // ancestry, increment
               + Npad * (DX + 1) * rsz + Npad * DX * rsz + N * rsz      // column / row data, row weights
               + sizeof(double) + 2 * N * sizeof(int32_t)                // shift, first/last ancestry
               + 2 * (size_t)N * DX * rsz + N * sizeof(double)          // column / row tables
               + sizeof(NodeDesc) + 2 * sizeof(int32_t);                 // schedule
  ps.per_node = 2 * (size_t)N * NcP * rsz + (size_t)N * (sizeof(double) + sizeof(float));
  return ps;
}

static bool tiles_known(const dsmc_plan_t* p);
static int enqueue_batch(dsmc_plan_t* p, int B, int totalK, hipStream_t st);

static int smooth_batch(dsmc_plan_t* p, int B, const dsmc_model_t* const* models,
                        const uint64_t* seeds, const void* const* stars, const dsmc_output* outs) {
  if (!p || B < 1 || !models || !seeds || !outs) return fail(DSMC_EINVAL, "bad argument");
  const int N = p->d.N;
  std::vector<int> Ks(B), bases(B);
  long total = 0;
  for (int s = 0; s < B; ++s) {
    const dsmc_model_t* m = models[s];
    if (!m) return fail(DSMC_EINVAL, "null model %d", s);
    if (m->dx != p->d.d_x) return fail(DSMC_EINVAL, "model %d has d_x %d, plan %d", s, m->dx, p->d.d_x);
    if (m->K > p->d.max_K) return fail(DSMC_EINVAL, "model %d has K %d > max_K %d", s, m->K, p->d.max_K);
    int rc = check_output(&outs[s]);
    if (rc) return rc;
    Ks[s] = m->K;
    bases[s] = (int)total;
    total += m->K;
  }
  if (total > p->d.max_total_K)
    return fail(DSMC_EINVAL, "sum of K %ld > max_total_K %d", total, p->d.max_total_K);
  const int totalK = (int)total;
  int rc = ensure_series_cap(p, B);
  if (rc) return rc;
  // the staging buffers of the previous call must have been consumed
  if (p->staged_pending) HIP_TRY(hipEventSynchronize(p->staged));
  const bool new_sched = (Ks != p->sched_K);
  if (new_sched) {
    build_schedule(p, Ks, bases);
    p->sched_K = Ks;
  }
  double pairs = 0.0;
  for (int s = 0; s < B; ++s) {
    const dsmc_output& o = outs[s];
    SeriesDesc sd{};
    sd.model = models[s]->dev;
    sd.seed = seeds[s];
    sd.K = Ks[s];
    sd.base = bases[s];
    sd.root = p->roots[s];
    sd.anc = o.ancestry ? o.ancestry : p->anc + (size_t)bases[s] * 2 * N;
    sd.zinc = o.logZ_inc ? o.logZ_inc : p->zinc + bases[s];
    sd.row_lse = o.row_lse;
    sd.status = o.status;
    sd.traj = o.traj;
    sd.logw = o.logw;
    sd.log_Z = o.log_Z;
    sd.leaf_x = o.leaf_x;
    sd.leaf_logw = o.leaf_logw;
    sd.leaf_logL = o.leaf_logL;
    sd.index = o.index;
    sd.star = stars ? stars[s] : nullptr;
    p->h_series[s] = sd;
    pairs += (double)(Ks[s] - 1) * N * (double)N;
  }
  p->last_pairs += pairs;
  hipStream_t st = p->stream;
  HIP_TRY(hipMemcpyAsync(p->d_series, p->h_series, (size_t)B * sizeof(SeriesDesc),
                         hipMemcpyHostToDevice, st));
  if (new_sched) {
    if (p->total_nodes)
      HIP_TRY(hipMemcpyAsync(p->d_nodes, p->h_nodes, (size_t)p->total_nodes * sizeof(NodeDesc),
                             hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->d_series_of_t, p->h_series_of_t, (size_t)totalK * sizeof(int32_t),
                           hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(p->d_leaf_cons, p->h_leaf_cons, (size_t)totalK * sizeof(int32_t),
                           hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipEventRecord(p->staged, st));
  p->staged_pending = true;

  if (p->use_graph && !p->timer.on) {
    if (p->gexec && Ks == p->graph_K && p->graph_series == p->d_series) {
      HIP_TRY(hipGraphLaunch(p->gexec, st));
      return DSMC_OK;
    }
    if (tiles_known(p)) {  // capture; the first call of a shape ran eagerly and tuned the tiles
      if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
      if (p->graph) (void)hipGraphDestroy(p->graph);
      p->gexec = nullptr;
      p->graph = nullptr;
      p->graph_K.clear();
      HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
      const int erc = enqueue_batch(p, B, totalK, p->cap_stream);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
      if (erc) {
        if (g) (void)hipGraphDestroy(g);
        return erc;
      }
      if (e != hipSuccess) return fail(DSMC_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
      p->graph = g;
      HIP_TRY(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
      p->graph_K = Ks;
      p->graph_series = p->d_series;
      HIP_TRY(hipGraphLaunch(p->gexec, st));
      return DSMC_OK;
    }
  }
  return enqueue_batch(p, B, totalK, st);
}

// True when every launch slice size of the current schedule has a tile.
static bool tiles_known(const dsmc_plan_t* p) {
  for (size_t l = 0; l < p->level_cnt.size(); ++l)
    for (int s0 = 0; s0 < p->level_cnt[l]; s0 += p->node_cap)
      if (!p->tiles.count(std::min(p->node_cap, p->level_cnt[l] - s0))) return false;
  return true;
}

// Every kernel of one dsmc_smooth_batch call, on stream st (capturable: no
// synchronisation, no memset; tiles must be known when st is capturing).
static int enqueue_batch(dsmc_plan_t* p, int B, int totalK, hipStream_t st) {
  const int N = p->d.N;
  launch_clear_status(p->d_series, 0, B, st);
  LeafLaunch LL{};
  LL.fp64 = p->fp64;
  LL.DX = p->DX;
  LL.N = N;
  LL.Npad = p->Npad;
  LL.totalK = totalK;
  LL.row0 = 0;
  LL.rows = totalK;
  LL.d_series = p->d_series;
  LL.d_series_of_t = p->d_series_of_t;
  LL.d_leaf_cons = p->d_leaf_cons;
  LL.d_nodes = p->d_nodes;
  LL.leafX = p->leafX;
  LL.leafW = p->leafW;
  LL.leafL = p->leafL;
  LL.bmerged = p->bmerged;
  LL.nb = p->nb;
  if (launch_leaves(LL, st, &p->timer)) return fail(DSMC_EUNSUPPORTED, "no leaf kernel for d_x");
  HIP_TRY(hipGetLastError());

  for (size_t l = 0; l < p->level_cnt.size(); ++l) {
    const int cnt = p->level_cnt[l];
    for (int s0 = 0; s0 < cnt; s0 += p->node_cap) {
      const int nodes = std::min(p->node_cap, cnt - s0);
      LevelLaunch L{};
      L.fp64 = p->fp64;
      L.bf16 = p->bf16;
      L.DX = p->DX;
      L.node_list = nullptr;
      L.node0 = p->level_off[l] + s0;
      L.nodes = nodes;
      L.N = N;
      L.Npad = p->Npad;
      L.Nc = p->Nc;
      L.NcP = p->NcP;
      L.totalK = totalK;
      L.d_nodes = p->d_nodes;
      L.d_series = p->d_series;
      L.leafX = p->leafX;
      L.bmerged = p->bmerged;
      L.P = p->P;
      L.Pr = p->Pr;
      L.Rsum = p->Rsum;
      L.Rshift = p->Rshift;
      L.Gs = p->Gs;
      L.force_rescue = (p->d.flags & DSMC_PLAN_RESCUE_ALL) != 0;
      L.rescue_count = p->d_rescued;
      L.nb = p->nb;
      L.lazy = p->d.resampling;
      L.lazy_param = p->lazy_param;
      set_sample_shape(L);
      auto it = p->tiles.find(nodes);
      TileChoice tc;
      if (it != p->tiles.end()) {
        tc = it->second;
      } else {  // lazy plans run no pair-row kernel: nothing to tune
        tc = (p->autotune && !L.lazy) ? autotune_tile(p, L)
                                      : heuristic_tile(nodes, N, p->Nc, p->DX < 8);
        p->tiles[nodes] = tc;
      }
      set_tile(L, tc);
      if (launch_level(L, st, &p->timer)) return fail(DSMC_EUNSUPPORTED, "no combine kernel for d_x");
      HIP_TRY(hipGetLastError());
    }
  }
  launch_output_levels(LL, p->level_off.data(), p->level_cnt.data(), (int)p->level_cnt.size(),
                       p->nb.sfirst, B, p->d.d_x, st, &p->timer);
  HIP_TRY(hipGetLastError());
  return DSMC_OK;
}

extern "C" int dsmc_schedule(int K, int cap, int32_t* a, int32_t* c, int32_t* b, int32_t* level) {
  if (K < 1) return fail(DSMC_EINVAL, "K must be >= 1");
  if (K - 1 > cap) return fail(DSMC_EINVAL, "cap %d < K - 1 = %d", cap, K - 1);
  if (K > 1 && (!a || !c || !b || !level)) return fail(DSMC_EINVAL, "null output");
  std::vector<NodeDesc> nodes;
  std::vector<int> lvl_off, lvl_cnt;
  std::vector<int32_t> leaf_cons;
  int root = -1;
  build_series_schedule(K, 0, 0, nodes, lvl_off, lvl_cnt, leaf_cons, &root);
  for (size_t l = 0; l < lvl_cnt.size(); ++l)
    for (int i = 0; i < lvl_cnt[l]; ++i) {
      const NodeDesc& nd = nodes[lvl_off[l] + i];
      const int id = lvl_off[l] + i;
      a[id] = nd.a;
      c[id] = nd.c;
      b[id] = nd.b;
      level[id] = (int32_t)l;
    }
  return (int)nodes.size();
}

extern "C" int dsmc_device_count(int* count) {
  if (!count) return fail(DSMC_EINVAL, "null count");
  *count = 0;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) return fail(DSMC_EDEVICE, "no GPU visible");
  *count = n;
  return DSMC_OK;
}

extern "C" int dsmc_smooth_batch(dsmc_plan_t* p, int B, const dsmc_model_t* const* models,
                                 const uint64_t* seeds, const dsmc_output* outs) {
  return smooth_batch(p, B, models, seeds, nullptr, outs);
}

extern "C" int dsmc_smooth(dsmc_plan_t* p, const dsmc_model_t* model, uint64_t seed,
                           const dsmc_output* out) {
  const dsmc_model_t* ms[1] = {model};
  return smooth_batch(p, 1, ms, &seed, nullptr, out);
}

extern "C" int dsmc_smooth_batch_conditional(dsmc_plan_t* p, int B,
                                             const dsmc_model_t* const* models,
                                             const uint64_t* seeds, const void* const* stars,
                                             const dsmc_output* outs) {
  if (!stars) return fail(DSMC_EINVAL, "null star list");
  return smooth_batch(p, B, models, seeds, stars, outs);
}

extern "C" int dsmc_smooth_conditional(dsmc_plan_t* p, const dsmc_model_t* model, uint64_t seed,
                                       const void* star, const dsmc_output* out) {
  if (!star) return fail(DSMC_EINVAL, "null star trajectory");
  const dsmc_model_t* ms[1] = {model};
  const void* stars[1] = {star};
  return smooth_batch(p, 1, ms, &seed, stars, out);
}

extern "C" int dsmc_plan_profile(dsmc_plan_t* p, dsmc_profile* out) {
  if (!p || !out) return fail(DSMC_EINVAL, "null argument");
  std::memset(out, 0, sizeof *out);
  if (!p->timer.on) return fail(DSMC_EINVAL, "plan was created without DSMC_PLAN_PROFILE");
  HIP_TRY(hipStreamSynchronize(p->stream));
  for (size_t i = 0; i < p->timer.cls.size(); ++i) {
    float ms = 0.0f;
    if (p->timer.beg[i] && p->timer.fin[i])
      HIP_TRY(hipEventElapsedTime(&ms, p->timer.beg[i], p->timer.fin[i]));
    const int c = p->timer.cls[i];
    out->launches[c] += 1;
    out->ms[c] += ms;
  }
  out->pairs = p->last_pairs;
  unsigned long long resc = 0;
  const unsigned long long zero = 0;
  HIP_TRY(hipMemcpy(&resc, p->d_rescued, sizeof resc, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(p->d_rescued, &zero, sizeof zero, hipMemcpyHostToDevice));
  out->rescued_rows = (double)resc;
  p->timer.reset();
  p->last_pairs = 0.0;
  return DSMC_OK;
}
