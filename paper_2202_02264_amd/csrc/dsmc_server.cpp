// Serving engine of include/dsmc.h: continuous batching of smoothing jobs.
//
// Jobs are grouped into classes by (N, padded d_x, precision).  Each class owns
// device pools sized at creation (time rows, combine ids, job slots) with
// first-fit range allocators, and a stream of its own.  One scheduler thread
//   - admits queued jobs whose rows, combines and slot fit (first fit in
//     arrival order), uploads their schedule and runs their leaves;
//   - at each step packs the next tree level of every resident job of a class
//     into one pair-rows and one sampling launch (a list of combine ids), with
//     at most two steps in flight per class so that new jobs join quickly;
//   - enqueues the output of jobs whose last level is done and, once the
//     job's completion event has fired, marks it DONE and frees its space.
// Kernels and per-combine arithmetic are those of dsmc_smooth, so a job's
// results do not depend on what it was batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "dsmc.h"
#include "dsmc_host.h"
#include "dsmc_internal.h"
#include "dsmc_launch.h"
#include "dsmc_range_alloc.h"

using namespace dsmc;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Job {
  uint64_t id = 0;
  dsmc_job job{};
  int K = 0, dx = 0;
  int state = DSMC_JOB_QUEUED;
  int code = DSMC_EAGAIN;
  bool cancel = false;  // set by dsmc_cancel (under the server mutex)
  double t_submit = 0, t_start = 0, t_done = 0;
  int row0 = -1, node0 = -1, slot = -1;
  std::vector<int> lvl_off, lvl_cnt;
  size_t next_level = 0;
  hipEvent_t done_ev = nullptr;
  // host sources of the job's uploads, kept until the job is done
  std::vector<NodeDesc> h_nodes;
  std::vector<int32_t> h_sot, h_leaf_cons;
  SeriesDesc h_sd{};
};

struct Class {
  int N = 0, DX = 1;
  bool fp64 = false;
  size_t rsz = 4;
  int Npad = 0, Nc = 0, NcP = 0;
  int rows_cap = 0, slots_cap = 0, node_cap = 0;
  hipStream_t stream = nullptr;
  void* leafX = nullptr;
  void* leafW = nullptr;
  double* leafL = nullptr;
  double* bmerged = nullptr;
  int32_t* anc = nullptr;
  double* zinc = nullptr;
  NodeBufs nb{};
  void* P = nullptr;
  void* Pr = nullptr;
  double* Rsum = nullptr;
  float* Rshift = nullptr;
  double* Gs = nullptr;  // chunk-group sums of rows under column splits
  NodeDesc* d_nodes = nullptr;
  int32_t* d_series_of_t = nullptr;
  int32_t* d_leaf_cons = nullptr;
  SeriesDesc* d_series = nullptr;
  int32_t* d_list = nullptr;
  int32_t* h_list[2] = {nullptr, nullptr};  // pinned, one per step in flight
  int list_turn = 0;
  RangeAlloc rows, nodes;
  std::vector<int> free_slots;
  std::deque<Job*> queue;
  std::vector<Job*> running;
  std::vector<Job*> finishing;
  std::deque<hipEvent_t> ticks;
  std::vector<void*> allocs;

  ~Class() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* q : allocs) (void)hipFree(q);
    for (auto& h : h_list)
      if (h) (void)hipHostFree(h);
    for (auto e : ticks) (void)hipEventDestroy(e);
    if (stream) (void)hipStreamDestroy(stream);
  }
};

}  // namespace

struct dsmc_server_impl {
  dsmc_server_desc d{};
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Job*> incoming;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  std::map<std::pair<int, int>, std::unique_ptr<Class>> classes;  // scheduler thread only
  uint64_t next_id = 1;
  bool stop = false;
  std::thread th;
  Timer no_timer;
};

namespace {

template <typename T>
int dalloc(Class* c, T** p, size_t bytes) {
  hipError_t e = hipMalloc((void**)p, std::max<size_t>(bytes, 256));
  if (e != hipSuccess) return fail(DSMC_ENOMEM, "server pool hipMalloc(%zu B): %s", bytes, hipGetErrorString(e));
  c->allocs.push_back((void*)*p);
  return DSMC_OK;
}

int make_class(dsmc_server_impl* s, int N, int DX, std::unique_ptr<Class>* out) {
  auto c = std::make_unique<Class>();
  c->N = N;
  c->DX = DX;
  c->fp64 = s->d.precision == DSMC_FP64;
  c->rsz = c->fp64 ? 8 : 4;
  c->Npad = (N + kChunk - 1) / kChunk * kChunk;
  c->Nc = c->Npad / kChunk;
  c->NcP = (c->Nc + kGroup - 1) / kGroup * kGroup;
  const size_t budget = s->d.mem_budget / (size_t)s->d.max_classes;
  const PoolSizes ps = pool_sizes(N, DX, DX, c->rsz);
  const size_t p_budget = std::min<size_t>(budget / 4, (size_t)2 << 30);  // chunk sums + rescued copies
  c->node_cap = (int)std::max<size_t>(1, p_budget / ps.per_node);
  const size_t rest = budget > c->node_cap * ps.per_node ? budget - c->node_cap * ps.per_node : 0;
  c->rows_cap = (int)std::min<size_t>(rest / ps.per_row, (size_t)1 << 30);
  if (c->rows_cap < 2) return fail(DSMC_ENOMEM, "server class budget too small for N=%d", N);
  c->slots_cap = s->d.max_jobs;
  const size_t TK = (size_t)c->rows_cap, R = c->rsz, nc = (size_t)c->node_cap;
  int rc = DSMC_OK;
  if ((rc = dalloc(c.get(), &c->leafX, (size_t)DX * TK * N * R)) ||
      (rc = dalloc(c.get(), &c->leafW, TK * N * R)) ||
      (rc = dalloc(c.get(), &c->leafL, TK * sizeof(double))) ||
      (rc = dalloc(c.get(), &c->bmerged, TK * sizeof(double))) ||
      (rc = dalloc(c.get(), &c->anc, TK * 2 * N * sizeof(int32_t))) ||
      (rc = dalloc(c.get(), &c->zinc, TK * sizeof(double))) ||
      (rc = dalloc(c.get(), &c->nb.col, TK * c->Npad * (DX + 1) * R)) ||
      (rc = dalloc(c.get(), &c->nb.row, TK * c->Npad * DX * R)) ||
      (rc = dalloc(c.get(), &c->nb.alpha, TK * N * R)) ||
      (rc = dalloc(c.get(), &c->nb.bcol, TK * sizeof(double))) ||
      (rc = dalloc(c.get(), &c->nb.sfirst, TK * N * sizeof(int32_t))) ||
      (rc = dalloc(c.get(), &c->nb.slast, TK * N * sizeof(int32_t))) ||
      (rc = dalloc(c.get(), &c->nb.tcol, TK * N * DX * R)) ||
      (rc = dalloc(c.get(), &c->nb.tgq, TK * N * sizeof(double))) ||
      (rc = dalloc(c.get(), &c->nb.trow, TK * N * DX * R)) ||
      (rc = dalloc(c.get(), &c->P, nc * N * c->NcP * R)) ||
      (rc = dalloc(c.get(), &c->Pr, nc * N * c->NcP * R)) ||
      (rc = dalloc(c.get(), &c->Rsum, nc * N * sizeof(double))) ||
      (rc = dalloc(c.get(), &c->Rshift, nc * N * sizeof(float))) ||
      (rc = dalloc(c.get(), &c->Gs, nc * N * group_stride(c->NcP) * sizeof(double))) ||
      (rc = dalloc(c.get(), &c->d_nodes, TK * sizeof(NodeDesc))) ||
      (rc = dalloc(c.get(), &c->d_series_of_t, TK * sizeof(int32_t))) ||
      (rc = dalloc(c.get(), &c->d_leaf_cons, TK * sizeof(int32_t))) ||
      (rc = dalloc(c.get(), &c->d_series, (size_t)c->slots_cap * sizeof(SeriesDesc))) ||
      (rc = dalloc(c.get(), &c->d_list, TK * sizeof(int32_t))))
    return rc;
  for (auto& h : c->h_list)
    if (hipHostMalloc((void**)&h, TK * sizeof(int32_t), hipHostMallocDefault) != hipSuccess)
      return fail(DSMC_ENOMEM, "server pinned list allocation failed");
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
    return fail(DSMC_EDEVICE, "hipStreamCreate failed");
  c->rows.reset(c->rows_cap);
  c->nodes.reset(c->rows_cap);
  for (int i = c->slots_cap - 1; i >= 0; --i) c->free_slots.push_back(i);
  *out = std::move(c);
  return DSMC_OK;
}

LeafLaunch leaf_launch(Class* c, int row0, int rows) {
  LeafLaunch LL{};
  LL.fp64 = c->fp64;
  LL.DX = c->DX;
  LL.N = c->N;
  LL.Npad = c->Npad;
  LL.totalK = c->rows_cap;
  LL.row0 = row0;
  LL.rows = rows;
  LL.d_series = c->d_series;
  LL.d_series_of_t = c->d_series_of_t;
  LL.d_leaf_cons = c->d_leaf_cons;
  LL.d_nodes = c->d_nodes;
  LL.leafX = c->leafX;
  LL.leafW = c->leafW;
  LL.leafL = c->leafL;
  LL.bmerged = c->bmerged;
  LL.nb = c->nb;
  return LL;
}

void set_state(dsmc_server_impl* s, Job* j, int state, int code) {
  std::lock_guard<std::mutex> lk(s->mu);
  j->state = state;
  j->code = code;
  if (state == DSMC_JOB_RUNNING) j->t_start = now_s();
  if (state == DSMC_JOB_DONE || state == DSMC_JOB_FAILED) j->t_done = now_s();
}

void release(Class* c, Job* j) {
  if (j->row0 >= 0) c->rows.release(j->row0, j->K);
  if (j->node0 >= 0) c->nodes.release(j->node0, j->K - 1);
  if (j->slot >= 0) c->free_slots.push_back(j->slot);
  j->row0 = j->node0 = j->slot = -1;
}

int enqueue_output(dsmc_server_impl* s, Class* c, Job* j) {
  launch_output(leaf_launch(c, j->row0, j->K), j->slot, 1, j->dx, c->stream, &s->no_timer);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventCreateWithFlags(&j->done_ev, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(j->done_ev, c->stream));
  c->finishing.push_back(j);
  return DSMC_OK;
}

// Place a job in its class pools, upload its schedule and series
// descriptor, and enqueue its leaves.  Returns DSMC_EAGAIN if it does not fit now.
int admit(dsmc_server_impl* s, Class* c, Job* j) {
  const int K = j->K, N = c->N;
  if (K > c->rows_cap || K - 1 > c->rows_cap) return fail(DSMC_ENOMEM, "job with K=%d exceeds the class pool", K);
  if (c->free_slots.empty()) return DSMC_EAGAIN;
  const int row0 = c->rows.alloc(K);
  if (row0 < 0) return DSMC_EAGAIN;
  int node0 = 0;
  if (K > 1) {
    node0 = c->nodes.alloc(K - 1);
    if (node0 < 0) {
      c->rows.release(row0, K);
      return DSMC_EAGAIN;
    }
  }
  const int slot = c->free_slots.back();
  c->free_slots.pop_back();
  j->row0 = row0;
  j->node0 = K > 1 ? node0 : -1;
  j->slot = slot;
  std::vector<NodeDesc>& nodes = j->h_nodes;
  nodes.clear();
  nodes.reserve(K > 1 ? K - 1 : 0);
  int root = -1;
  build_series_schedule(K, slot, node0, nodes, j->lvl_off, j->lvl_cnt, j->h_leaf_cons, &root);
  j->h_sot.assign(K, slot);
  const dsmc_output& o = j->job.out;
  SeriesDesc& sd = j->h_sd;
  sd = SeriesDesc{};
  sd.model = j->job.model->dev;
  sd.seed = j->job.seed;
  sd.K = K;
  sd.base = row0;
  sd.root = root;
  sd.anc = o.ancestry ? o.ancestry : c->anc + (size_t)row0 * 2 * N;
  sd.zinc = o.logZ_inc ? o.logZ_inc : c->zinc + row0;
  sd.row_lse = o.row_lse;
  sd.status = o.status;
  sd.traj = o.traj;
  sd.logw = o.logw;
  sd.log_Z = o.log_Z;
  sd.leaf_x = o.leaf_x;
  sd.leaf_logw = o.leaf_logw;
  sd.leaf_logL = o.leaf_logL;
  sd.index = o.index;
  if (!nodes.empty())
    HIP_TRY(hipMemcpyAsync(c->d_nodes + node0, nodes.data(), nodes.size() * sizeof(NodeDesc),
                           hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d_series_of_t + row0, j->h_sot.data(), K * sizeof(int32_t),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d_leaf_cons + row0, j->h_leaf_cons.data(), K * sizeof(int32_t),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d_series + slot, &sd, sizeof sd, hipMemcpyHostToDevice, c->stream));
  launch_clear_status(c->d_series, slot, 1, c->stream);
  if (launch_leaves(leaf_launch(c, row0, K), c->stream, &s->no_timer))
    return fail(DSMC_EUNSUPPORTED, "no leaf kernel for d_x");
  HIP_TRY(hipGetLastError());
  set_state(s, j, DSMC_JOB_RUNNING, DSMC_EAGAIN);
  j->next_level = 0;
  if (j->lvl_cnt.empty()) return enqueue_output(s, c, j);
  c->running.push_back(j);
  return DSMC_OK;
}

// One step: the next level of every running job of the class, packed.
int tick(dsmc_server_impl* s, Class* c) {
  int32_t* h = c->h_list[c->list_turn];
  int cnt = 0;
  for (Job* j : c->running) {
    const int off = j->node0 + j->lvl_off[j->next_level];
    for (int i = 0; i < j->lvl_cnt[j->next_level]; ++i) h[cnt++] = off + i;
  }
  if (cnt == 0) return DSMC_OK;
  HIP_TRY(hipMemcpyAsync(c->d_list, h, (size_t)cnt * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
  const int N = c->N;
  for (int s0 = 0; s0 < cnt; s0 += c->node_cap) {
    const int nodes = std::min(c->node_cap, cnt - s0);
    LevelLaunch L{};
    L.fp64 = c->fp64;
    L.DX = c->DX;
    L.node_list = c->d_list + s0;
    L.node0 = 0;
    L.nodes = nodes;
    L.N = N;
    L.Npad = c->Npad;
    L.Nc = c->Nc;
    L.NcP = c->NcP;
    L.totalK = c->rows_cap;
    L.d_nodes = c->d_nodes;
    L.d_series = c->d_series;
    L.leafX = c->leafX;
    L.bmerged = c->bmerged;
    L.P = c->P;
    L.Pr = c->Pr;
    L.Rsum = c->Rsum;
    L.Rshift = c->Rshift;
    L.Gs = c->Gs;
    L.nb = c->nb;
    set_sample_shape(L);
    set_tile(L, heuristic_tile(nodes, N, c->Nc, c->DX < 8));
    if (launch_level(L, c->stream, &s->no_timer)) return fail(DSMC_EUNSUPPORTED, "no combine kernel");
    HIP_TRY(hipGetLastError());
  }
  hipEvent_t ev;
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(ev, c->stream));
  c->ticks.push_back(ev);
  c->list_turn ^= 1;
  std::vector<Job*> still;
  for (Job* j : c->running) {
    ++j->next_level;
    if (j->next_level == j->lvl_cnt.size()) {
      int rc = enqueue_output(s, c, j);
      if (rc) return rc;
    } else {
      still.push_back(j);
    }
  }
  c->running.swap(still);
  return DSMC_OK;
}

// Returns true if anything changed.
bool service_class(dsmc_server_impl* s, Class* c, bool admitting) {
  bool did = false;
  // completed steps
  while (!c->ticks.empty() && hipEventQuery(c->ticks.front()) == hipSuccess) {
    (void)hipEventDestroy(c->ticks.front());
    c->ticks.pop_front();
  }
  // completed jobs
  for (size_t i = 0; i < c->finishing.size();) {
    Job* j = c->finishing[i];
    if (hipEventQuery(j->done_ev) == hipSuccess) {
      (void)hipEventDestroy(j->done_ev);
      j->done_ev = nullptr;
      release(c, j);
      j->h_nodes = {};
      j->h_sot = {};
      j->h_leaf_cons = {};
      set_state(s, j, DSMC_JOB_DONE, DSMC_OK);
      c->finishing[i] = c->finishing.back();
      c->finishing.pop_back();
      did = true;
    } else {
      ++i;
    }
  }
  // cancelled jobs and missed admission deadlines leave the queue
  {
    const double now = now_s();
    for (size_t i = 0; i < c->queue.size();) {
      Job* j = c->queue[i];
      bool cancelled;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        cancelled = j->cancel;
      }
      const bool late = j->job.admit_deadline > 0 && now > j->t_submit + j->job.admit_deadline;
      if (cancelled || late) {
        c->queue.erase(c->queue.begin() + i);
        set_state(s, j, DSMC_JOB_FAILED, cancelled ? DSMC_ECANCELLED : DSMC_EDEADLINE);
        did = true;
      } else {
        ++i;
      }
    }
  }
  // admissions (arrival order, first fit)
  if (admitting) {
    for (size_t i = 0; i < c->queue.size();) {
      Job* j = c->queue[i];
      int rc = admit(s, c, j);
      if (rc == DSMC_EAGAIN) {
        ++i;
        continue;
      }
      c->queue.erase(c->queue.begin() + i);
      did = true;
      if (rc != DSMC_OK) {
        release(c, j);
        set_state(s, j, DSMC_JOB_FAILED, rc);
      }
    }
  }
  // one packed step if fewer than two are in flight
  if (!c->running.empty() && c->ticks.size() < 2) {
    std::vector<Job*> in_step = c->running;
    int rc = tick(s, c);
    if (rc) {
      for (Job* j : in_step) {
        release(c, j);
        set_state(s, j, DSMC_JOB_FAILED, rc);
      }
      c->running.clear();
    }
    did = true;
  }
  return did;
}

void scheduler(dsmc_server_impl* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    bool stopping;
    std::deque<Job*> arrived;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      stopping = s->stop;
      arrived.swap(s->incoming);
    }
    for (Job* j : arrived) {
      if (stopping) {
        set_state(s, j, DSMC_JOB_FAILED, DSMC_ECANCELLED);
        continue;
      }
      const std::pair<int, int> key(j->job.N, padded_dx(j->dx));
      auto it = s->classes.find(key);
      if (it == s->classes.end()) {
        if ((int)s->classes.size() >= s->d.max_classes) {
          fail(DSMC_ENOMEM, "server has no room for another (N, d_x) class");
          set_state(s, j, DSMC_JOB_FAILED, DSMC_ENOMEM);
          continue;
        }
        std::unique_ptr<Class> c;
        int rc = make_class(s, key.first, key.second, &c);
        if (rc) {
          set_state(s, j, DSMC_JOB_FAILED, rc);
          continue;
        }
        it = s->classes.emplace(key, std::move(c)).first;
      }
      it->second->queue.push_back(j);
    }
    bool busy = false, did = false;
    for (auto& kv : s->classes) {
      Class* c = kv.second.get();
      if (stopping) {
        for (Job* j : c->queue) set_state(s, j, DSMC_JOB_FAILED, DSMC_ECANCELLED);
        c->queue.clear();
      }
      did |= service_class(s, c, !stopping);
      busy |= !c->queue.empty() || !c->running.empty() || !c->finishing.empty();
    }
    if (stopping && !busy) break;
    if (!did) {
      std::unique_lock<std::mutex> lk(s->mu);
      if (busy)
        s->cv.wait_for(lk, std::chrono::microseconds(50));
      else
        s->cv.wait_for(lk, std::chrono::milliseconds(2), [s] { return s->stop || !s->incoming.empty(); });
    }
  }
}

}  // namespace

extern "C" int dsmc_server_create(const dsmc_server_desc* d, dsmc_server_t** out) {
  if (!d || !out) return fail(DSMC_EINVAL, "null argument");
  *out = nullptr;
  if (d->precision != DSMC_FP32 && d->precision != DSMC_FP64)
    return fail(DSMC_EUNSUPPORTED, "precision %d not supported", d->precision);
  auto* s = new dsmc_server_t;
  s->d = *d;
  if (!s->d.mem_budget) s->d.mem_budget = (size_t)16 << 30;
  if (s->d.max_jobs <= 0) s->d.max_jobs = 1024;
  if (s->d.max_classes <= 0) s->d.max_classes = 4;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(DSMC_EDEVICE, "hipGetDevice failed");
  }
  s->th = std::thread(scheduler, s);
  *out = s;
  return DSMC_OK;
}

extern "C" void dsmc_server_destroy(dsmc_server_t* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();
  s->classes.clear();
  delete s;
}

extern "C" int dsmc_submit(dsmc_server_t* s, const dsmc_job* job, uint64_t* job_id) {
  if (!s || !job || !job_id) return fail(DSMC_EINVAL, "null argument");
  if (!job->model) return fail(DSMC_EINVAL, "null model");
  if (job->N < 1 || job->N > DSMC_MAX_N) return fail(DSMC_EUNSUPPORTED, "N must be in 1..%d", DSMC_MAX_N);
  if (!(job->admit_deadline >= 0.0)) return fail(DSMC_EINVAL, "admit_deadline must be >= 0");
  int rc = check_output(&job->out);
  if (rc) return rc;
  auto j = std::make_unique<Job>();
  j->job = *job;
  j->K = job->model->K;
  j->dx = job->model->dx;
  j->t_submit = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(DSMC_ECANCELLED, "server is stopping");
  j->id = s->next_id++;
  *job_id = j->id;
  s->incoming.push_back(j.get());
  s->jobs.emplace(j->id, std::move(j));
  s->cv.notify_all();
  return DSMC_OK;
}

extern "C" int dsmc_cancel(dsmc_server_t* s, uint64_t job_id) {
  if (!s) return fail(DSMC_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return fail(DSMC_EINVAL, "unknown job %llu", (unsigned long long)job_id);
  Job* j = it->second.get();
  if (j->state != DSMC_JOB_QUEUED) return DSMC_EAGAIN;
  j->cancel = true;
  s->cv.notify_all();
  return DSMC_OK;
}

extern "C" int dsmc_poll(dsmc_server_t* s, uint64_t job_id, int* state) {
  if (!s) return fail(DSMC_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return fail(DSMC_EINVAL, "unknown job %llu", (unsigned long long)job_id);
  const Job* j = it->second.get();
  if (state) *state = j->state;
  if (j->state == DSMC_JOB_DONE) return DSMC_OK;
  if (j->state == DSMC_JOB_FAILED) return j->code;
  return DSMC_EAGAIN;
}

extern "C" int dsmc_job_times(dsmc_server_t* s, uint64_t job_id, double* t_submit, double* t_start,
                              double* t_done) {
  if (!s) return fail(DSMC_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return fail(DSMC_EINVAL, "unknown job %llu", (unsigned long long)job_id);
  const Job* j = it->second.get();
  if (t_submit) *t_submit = j->t_submit;
  if (t_start) *t_start = j->t_start;
  if (t_done) *t_done = j->t_done;
  return DSMC_OK;
}

extern "C" int dsmc_job_release(dsmc_server_t* s, uint64_t job_id) {
  if (!s) return fail(DSMC_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(job_id);
  if (it == s->jobs.end()) return fail(DSMC_EINVAL, "unknown job %llu", (unsigned long long)job_id);
  const int st = it->second->state;
  if (st != DSMC_JOB_DONE && st != DSMC_JOB_FAILED) return DSMC_EAGAIN;
  s->jobs.erase(it);  // the scheduler holds no reference to a finished job
  return DSMC_OK;
}
