// Continuous-batching request server.
//
// Requests are independent sample solves (one KL input, one mesh, one time
// grid).  Each mesh size is a class with its own set-up and a few lanes; a lane
// is a stream with its own problem handle (work buffer, work counter).  A
// request's tables, state a, resume record and QoI live in a device slot of
// its class from admission to completion.  The scheduler thread advances every
// admitted request in launches of at most `chunk_steps` steps: whenever a lane
// is idle it launches one persistent kernel over all admitted requests of its
// class that are not running elsewhere, so requests that arrive while others
// run join the next launch and overlap on the device with the launches of the
// other lanes and classes.  Launch boundaries sit at fixed request-relative
// steps and the kernels resume bit for bit (Inst::carry), so a request's
// result does not depend on what else the server is running.
//
// Requests on large multigrid meshes (n_nodes >= wide_min_nodes) go instead to
// the wide lane while the device has room and its queue is short: a worker
// thread that runs them one at a time, each over the whole device (the wide
// path), which cuts their latency from one workgroup's pace to the device's.
// Batched, such a request costs one workgroup; wide, it takes every compute
// unit at a lower efficiency (and its stream of short kernels keeps the
// batched launches' large workgroups from finding free compute units), so a
// large request is routed to the lane only while fewer than wide_load_limit
// batched requests are admitted and at most wide_queue wait for it, and the
// lane pauses between time steps while the batched load is at or above that
// limit.  A request runs on one path from start to end, so its result stays
// the same bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "problem.h"

using namespace mq;

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

constexpr int SLAB = 16;          // request slots allocated at a time
constexpr int XI_SLOT = 16;       // doubles reserved for a request's input

// Pinned host memory (asynchronous copies that never wait for the device).
template <typename T>
struct PinnedPtr {
  T* p = nullptr;
  PinnedPtr() = default;
  PinnedPtr(const PinnedPtr&) = delete;
  PinnedPtr& operator=(const PinnedPtr&) = delete;
  ~PinnedPtr() {
    if (p) (void)hipHostFree(p);
  }
  T* get() const { return p; }
};
template <typename T>
hipError_t pinned_alloc(PinnedPtr<T>& h, size_t count) {
  return hipHostMalloc((void**)&h.p, (count > 0 ? count : 1) * sizeof(T), hipHostMallocDefault);
}

struct Req {
  mq_request rq;
  uint64_t ticket = 0;
  int64_t t_submit = 0, t_start = 0;
  int slot = -1;
  int64_t n_total = 0, done_steps = 0;
  int64_t iters = 0, sweeps = 0;
  int path = 0;
  int flags = 0;
  bool running = false;
  bool initialised = false;
};

// The scheduler thread never waits for a stream: a lane's instance table and
// the inputs of new requests go up from pinned buffers, and the launch's
// statistics and the QoI of the requests it completes come back into pinned
// buffers before its `done` event, all sized for max_batch requests when the
// lane is activated.  (Streams share the process's hardware queues, so a
// blocking copy could wait for another lane's whole launch.)
struct Lane {
  mq_problem* p = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<Req*> running;
  std::vector<Inst> insts;
  DevPtr<Inst> dinst;
  DevPtr<int> dstat;
  PinnedPtr<Inst> hinst;
  PinnedPtr<int> hstat;
  PinnedPtr<double> hq;   // QoI of the requests that complete in the launch, by launch position
  PinnedPtr<double> hxi;  // inputs of the requests initialised by the launch
  size_t cap = 0;
};

// J(t_k) of one time grid: FP64 on the host, uploaded once per class from a
// pinned copy on the stream of the lane that first needs it; other lanes wait
// for `ready` before using it.
struct SrcTable {
  DevPtr<double> dev;
  PinnedPtr<double> host;
  hipEvent_t ready = nullptr;
  ~SrcTable() {
    if (ready) (void)hipEventDestroy(ready);
  }
};

struct Class {
  int n_nodes = 0;
  size_t FS = 0, tab = 0, slot_d = 0;  // per slot: tables | a (FS) | carry (2 FS + 1) | q | xi
  std::vector<DevPtr<double>> slabs;
  std::vector<double*> slot_ptr;
  std::vector<int> free_slots;
  std::vector<std::unique_ptr<Lane>> lanes;
  std::map<std::pair<int, int64_t>, std::unique_ptr<SrcTable>> src;  // (steps/period, steps) -> J(t_k)
  std::vector<Req*> active;                                // admitted, in admission order
  size_t lane_slots = 0;
  int64_t fixed_bytes = 0;  // lane work buffers
  bool ready = false;       // work buffers allocated (counted in the budget)
};

}  // namespace

struct mq_server {
  mq_server_desc sd{};
  int device = 0;
  int n_xi = 0;
  int chunk = 32;
  int lanes = 2;
  int max_batch = 4096;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req*> queue;             // submitted, not yet admitted
  std::deque<mq_result> done;         // finished, not yet polled
  int64_t n_pending = 0;              // queued + admitted
  uint64_t next_ticket = 1;
  std::atomic<bool> stop{false};
  std::thread th;
  // scheduler-thread state
  std::map<int, std::unique_ptr<Class>> classes;
  int64_t used_bytes = 0;
  std::atomic<int> inflight{0};  // admitted batched requests (written by the scheduler only)
  // wide lane (queue and count guarded by mu)
  int wide_min = 0;  // 0: no wide lane
  int wide_queue = 8;
  int wide_load = 128;
  bool wide_mg = false;  // the base description allows multigrid
  std::deque<Req*> wq;
  int wide_count = 0;  // queued + running on the wide lane
  std::condition_variable wcv;
  std::thread wth;
};

namespace {

void finish(mq_server* s, Req* r, int status, double q, const std::string& msg = std::string()) {
  mq_result res{};
  if (status < 0) {
    const std::string m = msg.empty() ? last_error() : msg;
    std::snprintf(res.message, sizeof(res.message), "%s", m.c_str());
  }
  res.ticket = r->ticket;
  res.user_id = r->rq.user_id;
  res.q = q;
  res.status = status;
  res.inner_iters = (int32_t)std::min<int64_t>(r->iters, INT32_MAX);
  res.sweeps = (int32_t)std::min<int64_t>(r->sweeps, INT32_MAX);
  res.path = r->path;
  res.t_submit_ns = r->t_submit;
  res.t_start_ns = r->t_start;
  res.t_done_ns = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->done.push_back(res);
    s->n_pending--;
  }
  delete r;
}

void destroy_class(Class& c) {
  for (auto& L : c.lanes)
    if (L->stream) (void)hipStreamSynchronize(L->stream);
  for (auto& L : c.lanes) {
    L->dinst.reset();
    L->dstat.reset();
    if (L->p) mq_problem_destroy(L->p);
    if (L->done) (void)hipEventDestroy(L->done);
    if (L->stream) (void)hipStreamDestroy(L->stream);
  }
  c.lanes.clear();
  c.src.clear();
  c.slabs.clear();
}

// Set-up of one mesh class: one problem handle and stream per lane.  The
// lanes' work buffers (sized for a lane's largest launch) are allocated by
// activate() once they fit the budget.
int make_class(mq_server* s, int n_nodes, std::unique_ptr<Class>* out) {
  auto c = std::make_unique<Class>();
  c->n_nodes = n_nodes;
  mq_problem_desc d = s->sd.base;
  d.mem_kind = MQ_MEM_DEVICE;  // the server passes device buffers
  d.n_nodes = n_nodes;
  int64_t bytes = 0;
  for (int l = 0; l < s->lanes; ++l) {
    auto L = std::make_unique<Lane>();
    hipError_t e = hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&L->done, hipEventDisableTiming);
    if (e != hipSuccess) {
      c->lanes.push_back(std::move(L));
      destroy_class(*c);
      return fail(MQ_ERR_DEVICE, std::string("server stream: ") + hipGetErrorString(e));
    }
    int rc = fem_setup(&d, (void*)L->stream, &L->p);
    if (rc == MQ_OK) {
      const size_t slots = std::min<size_t>((size_t)s->max_batch, max_slots(L->p));
      c->lane_slots = slots;
      bytes += (int64_t)work_bytes(L->p, slots);
    }
    c->lanes.push_back(std::move(L));
    if (rc != MQ_OK) {
      destroy_class(*c);
      return rc;
    }
  }
  const Geom& g = c->lanes[0]->p->hm.g;
  c->FS = (size_t)g.N * g.P;
  c->tab = tab_stride(g);
  c->slot_d = c->tab + 3 * c->FS + 2 + XI_SLOT;
  c->fixed_bytes = bytes;
  *out = std::move(c);
  return MQ_OK;
}

int64_t slab_bytes(const Class& c) { return (int64_t)(SLAB * c.slot_d * sizeof(double)); }

// Work buffers and per-lane tables (the work buffer is cleared on each lane's
// own stream, ahead of its first launch).
int activate(mq_server* s, Class& c) {
  const size_t cap = (size_t)s->max_batch;
  for (auto& L : c.lanes) {
    int rc = ensure_work(L->p, c.lane_slots);
    if (rc) return rc;
    if (L->cap < cap) {
      HIP_TRY(dev_alloc(L->dinst, cap));
      HIP_TRY(dev_alloc(L->dstat, cap * STAT_N));
      HIP_TRY(pinned_alloc(L->hinst, cap));
      HIP_TRY(pinned_alloc(L->hstat, cap * STAT_N));
      HIP_TRY(pinned_alloc(L->hq, cap));
      HIP_TRY(pinned_alloc(L->hxi, cap * XI_SLOT));
      L->cap = cap;
    }
  }
  c.ready = true;
  return MQ_OK;
}

// Source table for one time grid, enqueued on lane L's stream.
int source_for(Class& c, Lane& L, const mq_problem_desc& d, int spp, int64_t n_total, const double** out) {
  auto key = std::make_pair(spp, n_total);
  auto it = c.src.find(key);
  if (it == c.src.end()) {
    auto h = source_table(d, 1.0 / (d.freq * spp), (int)n_total);
    auto t = std::make_unique<SrcTable>();
    HIP_TRY(dev_alloc(t->dev, h.size()));
    HIP_TRY(pinned_alloc(t->host, h.size()));
    std::memcpy(t->host.get(), h.data(), h.size() * sizeof(double));
    HIP_TRY(hipEventCreateWithFlags(&t->ready, hipEventDisableTiming));
    HIP_TRY(hipMemcpyAsync(t->dev.get(), t->host.get(), h.size() * sizeof(double), hipMemcpyHostToDevice, L.stream));
    HIP_TRY(hipEventRecord(t->ready, L.stream));
    it = c.src.emplace(key, std::move(t)).first;
  } else {
    HIP_TRY(hipStreamWaitEvent(L.stream, it->second->ready, 0));
  }
  *out = it->second->dev.get();
  return MQ_OK;
}

// Retire a lane whose launch has ended: accumulate counters, complete the
// requests that reached their last step.
void retire(mq_server* s, Class& c, Lane& L, hipError_t q) {
  L.busy = false;
  const int rc = q == hipSuccess ? MQ_OK : MQ_ERR_DEVICE;
  const std::string qmsg = q == hipSuccess ? std::string() : std::string("launch: ") + hipGetErrorString(q);
  const size_t n = L.running.size();
  std::vector<Req*> fin;
  std::vector<double> qh;
  for (size_t i = 0; i < n; ++i) {
    Req* r = L.running[i];
    r->running = false;
    if (rc != MQ_OK) {
      r->flags |= FLAG_FAILED;
      r->done_steps = r->n_total;
    } else {
      const int* st = L.hstat.get() + i * STAT_N;
      r->done_steps += L.insts[i].n_steps;
      r->iters += st[0];
      r->sweeps += st[1];
      r->path = L.p->path;
      r->flags |= st[3];
    }
    if (r->done_steps >= r->n_total) {
      fin.push_back(r);
      qh.push_back(rc == MQ_OK ? L.hq.get()[i] : NAN);
    }
  }
  L.running.clear();
  for (size_t i = 0; i < fin.size(); ++i) {
    Req* r = fin[i];
    c.active.erase(std::find(c.active.begin(), c.active.end(), r));
    c.free_slots.push_back(r->slot);
    s->inflight--;
    int status = MQ_OK;
    if (rc != MQ_OK) status = rc;
    else if (r->flags & FLAG_FAILED) status = MQ_ERR_NONFINITE;
    else if (r->flags & FLAG_NOT_CONVERGED) status = MQ_WARN_NOT_CONVERGED;
    finish(s, r, status, status < 0 ? NAN : qh[i],
           rc != MQ_OK ? qmsg : (status == MQ_ERR_NONFINITE ? "the solve produced NaN or Inf" : ""));
  }
}

// Admitted requests of class c that no lane is running, in admission order.
std::vector<Req*> idle_requests(mq_server* s, Class& c) {
  std::vector<Req*> pick;
  for (Req* r : c.active) {
    if (r->running) continue;
    pick.push_back(r);
    if ((int)pick.size() >= s->max_batch) break;
  }
  return pick;
}

// Launch the next step chunk of the requests `pick` (class c) on lane L.
int launch_lane(mq_server* s, Class& c, Lane& L, const std::vector<Req*>& pick) {
  const mq_problem_desc& d = L.p->d;
  const Geom& g = L.p->hm.g;
  L.insts.clear();
  for (Req* r : pick) {
    double* base = c.slot_ptr[r->slot];
    double* tab = base;
    double* a = base + c.tab;
    double* carry = a + c.FS;
    double* q = carry + 2 * c.FS + 1;
    double* xi = q + 1;
    if (!r->initialised) {
      // request input -> device (through the lane's pinned buffer), per-sample
      // tables, zero initial state
      double* hx = L.hxi.get() + L.insts.size() * XI_SLOT;
      std::memcpy(hx, r->rq.xi, sizeof(double) * s->n_xi);
      HIP_TRY(hipMemcpyAsync(xi, hx, sizeof(double) * s->n_xi, hipMemcpyHostToDevice, L.stream));
      HIP_TRY(launch_assemble(g, L.p->hm.cr, L.p->dcond.get(), L.p->dkl.get(), L.p->hm.n_modes, d.material, xi,
                              s->n_xi, 1, L.p->mat, tab, L.stream));
      if (d.mass == MQ_MASS_LUMPED) HIP_TRY(launch_lump_mass(g, 1, tab, L.stream));
      HIP_TRY(launch_fill_zero(a, c.FS, L.stream));
      r->initialised = true;
    }
    const double* src = nullptr;
    int rc = source_for(c, L, d, r->rq.steps_per_period, r->n_total, &src);
    if (rc) return rc;
    Inst in{};
    in.tab = tab;
    in.src = src;
    in.a_init = a;
    in.a_out = a;
    in.q_out = q;
    in.q_scale = 1.0 / (r->rq.n_periods / d.freq);  // 1 / T, as in the level runs
    in.dt = 1.0 / (d.freq * r->rq.steps_per_period);
    in.k0 = (int)r->done_steps;
    in.n_steps = (int)std::min<int64_t>(s->chunk, r->n_total - r->done_steps);
    in.carry = carry;
    in.carry_in = r->done_steps > 0;
    L.insts.push_back(in);
  }
  // longest remaining work first (the kernel's work queue takes instances in order)
  std::vector<size_t> ord(pick.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return L.insts[x].n_steps > L.insts[y].n_steps; });
  std::vector<Inst> ins(ord.size());
  L.running.resize(ord.size());
  for (size_t i = 0; i < ord.size(); ++i) {
    ins[i] = L.insts[ord[i]];
    L.running[i] = pick[ord[i]];
  }
  L.insts.swap(ins);
  const size_t n = L.insts.size();
  if (n > L.cap) return fail(MQ_ERR_INVALID_ARG, "launch larger than the lane's tables");
  for (size_t i = 0; i < n; ++i) L.insts[i].stat = L.dstat.get() + STAT_N * i;
  std::memcpy(L.hinst.get(), L.insts.data(), n * sizeof(Inst));
  HIP_TRY(launch_fill_zero_i(L.dstat.get(), n * STAT_N, L.stream));
  HIP_TRY(hipMemcpyAsync(L.dinst.get(), L.hinst.get(), n * sizeof(Inst), hipMemcpyHostToDevice, L.stream));
  int grid = 0, block = 0;
  int rc = launch_persistent(L.p, L.dinst.get(), (int)n, &grid, &block);
  if (rc) return rc;
  // statistics, and the QoI of every request this launch completes, come back
  // ahead of the event
  HIP_TRY(hipMemcpyAsync(L.hstat.get(), L.dstat.get(), n * STAT_N * sizeof(int), hipMemcpyDeviceToHost, L.stream));
  for (size_t i = 0; i < n; ++i) {
    Req* r = L.running[i];
    if (r->done_steps + L.insts[i].n_steps < r->n_total) continue;
    const double* qd = c.slot_ptr[r->slot] + c.tab + 3 * c.FS + 1;
    HIP_TRY(hipMemcpyAsync(L.hq.get() + i, qd, sizeof(double), hipMemcpyDeviceToHost, L.stream));
  }
  HIP_TRY(hipEventRecord(L.done, L.stream));
  // the pinned tables and inputs are read by the stream: they are not
  // rewritten before the launch has been retired
  const int64_t t = now_ns();
  for (Req* r : L.running) {
    r->running = true;
    if (!r->t_start) r->t_start = t;
  }
  L.busy = true;
  return MQ_OK;
}

// Large meshes with a multigrid hierarchy (n_nodes = 2^k + 1) may use the wide lane.
bool wide_eligible(const mq_server* s, int n_nodes) {
  if (s->wide_min <= 0 || !s->wide_mg || n_nodes < s->wide_min) return false;
  const int m = n_nodes - 1;
  return m >= 2 && (m & (m - 1)) == 0;
}

// The wide lane: runs its requests one at a time with mlmc_level_run on a
// wide-path problem per mesh size (set up on first use, kept until the
// server ends).
void wide_worker(mq_server* s) {
  (void)hipSetDevice(s->device);
  hipStream_t st = nullptr;
  std::map<int, mq_problem*> probs;
  DevPtr<double> buf;  // xi | q
  bool ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
            dev_alloc(buf, XI_SLOT + 1) == hipSuccess;
  for (;;) {
    Req* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->wcv.wait(lk, [&] { return s->stop.load() || !s->wq.empty(); });
      if (s->stop.load()) break;
      r = s->wq.front();
      s->wq.pop_front();
    }
    r->t_start = now_ns();
    int status = MQ_ERR_DEVICE;
    double q = NAN;
    std::string msg = ok ? std::string() : std::string("wide lane set-up failed");
    if (ok) {
      mq_problem*& p = probs[r->rq.n_nodes];
      int rc = MQ_OK;
      if (!p) {
        mq_problem_desc d = s->sd.base;
        d.mem_kind = MQ_MEM_DEVICE;  // the server passes device buffers
        d.n_nodes = r->rq.n_nodes;
        d.path = MQ_PATH_WIDE;
        rc = fem_setup(&d, (void*)st, &p);
        if (rc != MQ_OK) p = nullptr;
        else
          p->wide_yield = [s] {
            while (s->inflight.load() >= s->wide_load && !s->stop.load())
              std::this_thread::sleep_for(std::chrono::microseconds(500));
          };
      }
      if (rc == MQ_OK &&
          hipMemcpyAsync(buf.get(), r->rq.xi, sizeof(double) * s->n_xi, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = MQ_ERR_DEVICE;
      if (rc == MQ_OK) {
        const mq_level_desc lv{r->rq.steps_per_period, 0, r->rq.n_periods, 0};
        mq_run_stats rs{};
        rc = mlmc_level_run(p, &lv, 1, buf.get(), buf.get() + XI_SLOT, nullptr, nullptr, &rs);
        r->iters = rs.inner_iters;
        r->sweeps = rs.sweeps;
        r->path = MQ_PATH_WIDE;
        if (rc >= 0 && (hipMemcpyAsync(&q, buf.get() + XI_SLOT, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
                        hipStreamSynchronize(st) != hipSuccess))
          rc = MQ_ERR_DEVICE;
      }
      status = rc;
      if (status < 0) msg = std::string("wide lane: ") + last_error();
      if (status >= 0 && !std::isfinite(q)) {
        status = MQ_ERR_NONFINITE;
        msg = "wide lane: the solve produced NaN or Inf";
      }
    }
    finish(s, r, status, status < 0 ? NAN : q, msg);
    std::lock_guard<std::mutex> lk(s->mu);
    s->wide_count--;
  }
  for (auto& kv : probs)
    if (kv.second) mq_problem_destroy(kv.second);
  if (st) (void)hipStreamDestroy(st);
}

// Admit queued requests in arrival order while they fit.
void admit(mq_server* s) {
  for (;;) {
    Req* r = nullptr;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->queue.empty()) return;
      r = s->queue.front();
    }
    if (wide_eligible(s, r->rq.n_nodes)) {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->wide_count < s->wide_queue + 1 && s->inflight < s->wide_load) {
        s->queue.pop_front();
        s->wq.push_back(r);
        s->wide_count++;
        s->wcv.notify_one();
        continue;
      }
    }
    if (s->inflight >= s->sd.max_inflight) return;
    auto it = s->classes.find(r->rq.n_nodes);
    int rc = MQ_OK;
    if (it == s->classes.end()) {
      std::unique_ptr<Class> c;
      rc = make_class(s, r->rq.n_nodes, &c);
      if (rc == MQ_OK) it = s->classes.emplace(r->rq.n_nodes, std::move(c)).first;
    }
    if (rc == MQ_OK && !it->second->ready) {
      Class& c = *it->second;
      if (s->used_bytes + c.fixed_bytes + slab_bytes(c) > s->sd.hbm_budget_bytes) {
        if (s->inflight > 0) return;  // wait for memory to free up
        rc = MQ_ERR_BUSY;
      } else {
        rc = activate(s, c);
        if (rc == MQ_OK) s->used_bytes += c.fixed_bytes;
      }
    }
    if (rc != MQ_OK) {
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->queue.pop_front();
      }
      finish(s, r, rc, NAN);
      continue;
    }
    Class& c = *it->second;
    if (c.free_slots.empty()) {
      const int64_t need = slab_bytes(c);
      if (s->used_bytes + need > s->sd.hbm_budget_bytes) {
        if (s->inflight > 0) return;  // wait for a slot
        {
          std::lock_guard<std::mutex> lk(s->mu);
          s->queue.pop_front();
        }
        finish(s, r, MQ_ERR_BUSY, NAN, "the request alone does not fit the memory budget");
        continue;
      }
      DevPtr<double> slab;
      if (dev_alloc(slab, SLAB * c.slot_d) != hipSuccess) {
        if (s->inflight > 0) return;
        {
          std::lock_guard<std::mutex> lk(s->mu);
          s->queue.pop_front();
        }
        finish(s, r, MQ_ERR_OUT_OF_MEMORY, NAN, "request slots: out of device memory");
        continue;
      }
      for (int k = SLAB - 1; k >= 0; --k) {
        c.slot_ptr.push_back(slab.get() + (size_t)k * c.slot_d);
        c.free_slots.push_back((int)c.slot_ptr.size() - 1);
      }
      c.slabs.push_back(std::move(slab));
      s->used_bytes += need;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->queue.pop_front();
    }
    r->slot = c.free_slots.back();
    c.free_slots.pop_back();
    c.active.push_back(r);
    s->inflight++;
  }
}

void scheduler(mq_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    bool progress = false;
    for (auto& kv : s->classes) {
      for (auto& L : kv.second->lanes) {
        if (!L->busy) continue;
        const hipError_t q = hipEventQuery(L->done);
        if (q == hipErrorNotReady) continue;
        retire(s, *kv.second, *L, q);
        progress = true;
      }
    }
    if (s->stop.load()) {
      bool any = false;
      for (auto& kv : s->classes)
        for (auto& L : kv.second->lanes) any |= L->busy;
      if (!any) break;
      std::this_thread::sleep_for(std::chrono::microseconds(100));
      continue;
    }
    admit(s);
    for (auto& kv : s->classes) {
      Class& c = *kv.second;
      for (auto& L : c.lanes) {
        if (L->busy) continue;
        const std::vector<Req*> pick = idle_requests(s, c);
        if (pick.empty()) break;
        const int rc = launch_lane(s, c, *L, pick);
        if (rc != MQ_OK) {
          // the picked requests fail; the lane stays usable
          (void)hipStreamSynchronize(L->stream);
          for (Req* r : pick) {
            r->running = false;
            c.active.erase(std::find(c.active.begin(), c.active.end(), r));
            c.free_slots.push_back(r->slot);
            s->inflight--;
            finish(s, r, rc, NAN);
          }
          L->running.clear();
          L->busy = false;
        }
        progress = true;
      }
    }
    if (!progress) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait_for(lk, std::chrono::microseconds(200));
    }
  }
}

}  // namespace

extern "C" {

int mq_server_create(const mq_server_desc* sd, void* stream, mq_server** out) {
  (void)stream;
  if (!sd || !out) return fail(MQ_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (sd->base.material == MQ_MAT_NONLINEAR)
    return fail(MQ_ERR_INVALID_ARG, "the server runs linear materials");
  if (sd->base.path == MQ_PATH_WIDE)
    return fail(MQ_ERR_INVALID_ARG, "the server batches requests: resident or streaming path");
  if (sd->hbm_budget_bytes <= 0 || sd->max_inflight < 1 || sd->n_streams < 0 || sd->n_streams > 8 ||
      sd->max_batch < 0 || sd->chunk_steps < 0 || sd->wide_min_nodes < -1 || sd->wide_queue < 0 ||
      sd->wide_load_limit < 0)
    return fail(MQ_ERR_INVALID_ARG, "bad server limits");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(MQ_ERR_NO_DEVICE, "no HIP device");
  // validate the base description once on a tiny mesh
  mq_problem_desc d = sd->base;
  d.mem_kind = MQ_MEM_DEVICE;
  d.n_nodes = 5;
  mq_problem* probe = nullptr;
  int rc = fem_setup(&d, nullptr, &probe);
  if (rc) return rc;
  auto s = new mq_server();
  s->n_xi = probe->n_xi;
  mq_problem_destroy(probe);
  s->sd = *sd;
  (void)hipGetDevice(&s->device);
  s->chunk = sd->chunk_steps > 0 ? sd->chunk_steps : 32;
  s->lanes = sd->n_streams > 0 ? sd->n_streams : 2;
  s->max_batch = sd->max_batch > 0 ? sd->max_batch : 4096;
  s->wide_min = sd->wide_min_nodes == 0 ? 513 : (sd->wide_min_nodes < 0 ? 0 : sd->wide_min_nodes);
  s->wide_queue = sd->wide_queue > 0 ? sd->wide_queue : 8;
  s->wide_mg = sd->base.precond != MQ_PRECOND_JACOBI;
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess || n_cu < 2)
    n_cu = 256;
  s->wide_load = sd->wide_load_limit > 0 ? sd->wide_load_limit : n_cu / 2;
  s->th = std::thread(scheduler, s);
  if (s->wide_min > 0) s->wth = std::thread(wide_worker, s);
  *out = s;
  return MQ_OK;
}

int mq_submit(mq_server* s, const mq_request* rq, uint64_t* ticket) {
  if (!s || !rq || !ticket) return fail(MQ_ERR_INVALID_ARG, "null argument");
  if (rq->n_nodes < 3 || rq->n_nodes > 8193) return fail(MQ_ERR_INVALID_ARG, "n_nodes must be in [3, 8193]");
  if (rq->steps_per_period < 1 || rq->n_periods < 1) return fail(MQ_ERR_INVALID_ARG, "steps >= 1 required");
  const int64_t n_total = (int64_t)rq->steps_per_period * rq->n_periods;
  if (n_total > (1 << 24)) return fail(MQ_ERR_INVALID_ARG, "too many steps");
  if (rq->n_xi != s->n_xi) return fail(MQ_ERR_INVALID_ARG, "n_xi does not match the server's material");
  for (int i = 0; i < rq->n_xi; ++i)
    if (!std::isfinite(rq->xi[i])) return fail(MQ_ERR_NONFINITE, "xi contains NaN or Inf");
  auto r = new Req();
  r->rq = *rq;
  r->n_total = n_total;
  r->t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    s->queue.push_back(r);
    s->n_pending++;
  }
  s->cv.notify_one();
  *ticket = r->ticket;
  return MQ_OK;
}

int mq_poll(mq_server* s, mq_result* out, int32_t cap, int32_t* n_out) {
  if (!s || !n_out || cap < 0 || (cap > 0 && !out)) return fail(MQ_ERR_INVALID_ARG, "bad poll arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t k = 0;
  while (k < cap && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n_out = k;
  return MQ_OK;
}

int mq_server_pending(const mq_server* s, int32_t* n) {
  if (!s || !n) return fail(MQ_ERR_INVALID_ARG, "null argument");
  auto* m = const_cast<mq_server*>(s);
  std::lock_guard<std::mutex> lk(m->mu);
  *n = (int32_t)m->n_pending;
  return MQ_OK;
}

int mq_server_destroy(mq_server* s) {
  if (!s) return MQ_OK;
  s->stop.store(true);
  {
    std::lock_guard<std::mutex> lk(s->mu);  // no wake-up is lost between the workers' test and wait
  }
  s->cv.notify_all();
  s->wcv.notify_all();
  if (s->th.joinable()) s->th.join();
  if (s->wth.joinable()) s->wth.join();
  for (Req* r : s->wq) delete r;
  s->wq.clear();
  for (auto& kv : s->classes) {
    destroy_class(*kv.second);
    for (Req* r : kv.second->active) delete r;
  }
  s->classes.clear();
  for (Req* r : s->queue) delete r;
  s->queue.clear();
  delete s;
  return MQ_OK;
}

}  // extern "C"
