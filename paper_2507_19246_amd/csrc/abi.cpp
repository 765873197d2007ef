// C ABI of libmq: argument validation, device memory, instance tables and
// launch orchestration for MLMC level runs (Section II-B), Parareal
// (Section II-C) and the MLMC estimator (Eq. (9)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <memory>
#include <queue>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "problem.h"

using namespace mq;

namespace mq {
std::string& last_error() {
  thread_local std::string e;
  return e;
}
// per-instance FLAG_* bits of the calling thread's last level, multilevel or
// Parareal run (empty after any other run call)
std::vector<int32_t>& last_flags() {
  thread_local std::vector<int32_t> f;
  return f;
}
}  // namespace mq

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

namespace mq {

Solver solver_of(const mq_problem* p) {
  Solver sv;
  sv.precond = p->precond == MQ_PRECOND_MULTIGRID ? 1 : 0;
  sv.mg_omega = p->d.mg_omega > 0 ? p->d.mg_omega : 0.8;
  sv.precision = p->d.precision;
  sv.tol = p->d.tol;
  sv.inner_rtol = p->d.inner_rtol;
  sv.max_iter = p->d.max_iter;
  sv.max_sweeps = p->d.max_sweeps;
  sv.nonlinear = p->d.material == MQ_MAT_NONLINEAR;
  sv.picard_tol = p->d.picard_tol;
  sv.picard_max = p->d.picard_max;
  sv.tile = p->tile;
  sv.mg_levels = p->d.mg_levels;
  sv.mg_coarse_sweeps = p->d.mg_coarse_sweeps;
  sv.mg_block_min = p->d.mg_block_min > 0 ? p->d.mg_block_min : 15;
  sv.lds_limit = p->lds_limit;
  return sv;
}

size_t slot_doubles(const mq_problem* p) {
  // FP64 slot planes + the streaming path's vector workspace (8-byte upper bound)
  const bool smg = (p->path == MQ_PATH_STREAMING || p->path == MQ_PATH_WIDE) && p->mg.nlev > 0;
  return ie_work_doubles(p->hm.g) + stream_vwork_elems(p->hm.g, smg ? &p->mg : nullptr);
}

int ensure_work(mq_problem* p, size_t slots) {
  if (p->work_slots >= slots) return MQ_OK;
  p->work.reset();
  p->work_slots = 0;
  const size_t nd = slots * slot_doubles(p);
  HIP_TRY(dev_alloc(p->work, nd));
  HIP_TRY(launch_fill_zero(p->work.get(), nd, p->stream));
  p->work_slots = slots;
  return MQ_OK;
}

size_t work_bytes(const mq_problem* p, size_t slots) { return slots * slot_doubles(p) * sizeof(double); }

size_t max_slots(const mq_problem* p) {
  if (p->path == MQ_PATH_WIDE) return 1;
  const int per_cu = ie_slots_per_cu(p->hm.g, p->mg.nlev > 0 ? &p->mg : nullptr, p->path, p->d.precision, p->tile);
  return (size_t)p->num_cu * per_cu;
}

int launch_persistent(mq_problem* p, const Inst* dinst, int n, int* grid, int* block, double* work,
                      size_t work_slots, int n_first, int grid_first, bool para) {
  if (!work) {
    work = p->work.get();
    work_slots = p->work_slots;
  }
  size_t slots = std::min<size_t>((size_t)n, max_slots(p));
  slots = std::min(slots, work_slots);
  if (slots < 1) return fail(MQ_ERR_INVALID_ARG, "work buffer smaller than the launch");
  // one queue unless asked: every entry in queue 0, every workgroup starts there
  HIP_TRY(launch_queue_init(p->dcounter.get(), n_first >= 0 ? n_first : n, grid_first >= 0 ? grid_first : INT_MAX,
                            p->stream));
  Solver sv = solver_of(p);
  sv.para = para ? 1 : 0;
  // the slot layout of the work buffer is fixed by its allocation (work_slots);
  // the grid is the occupancy-limited slot count
  hipError_t le = launch_ie(p->hm.g, p->mg, sv, dinst, n, p->dcounter.get(), work, (int)work_slots,
                            (int)slots, p->dS.get(), p->path, p->d.precision, p->hm.cr, p->dcond.get(), p->mat,
                            grid, block, p->stream);
  if (le != hipSuccess) return fail(MQ_ERR_DEVICE, std::string("time-stepping launch: ") + hipGetErrorString(le));
  return MQ_OK;
}

// J(t_k) = J0 sin(2 pi f k dt), k = 0..n_total (FP64 on the host).
std::vector<double> source_table(const mq_problem_desc& d, double dt, int n_total) {
  std::vector<double> s(n_total + 1);
  for (int k = 0; k <= n_total; ++k) s[k] = d.J0 * std::sin(2.0 * M_PI * d.freq * (k * dt));
  return s;
}

}  // namespace mq

namespace {

int n_xi_of(const mq_problem_desc& d) {
  if (d.material == MQ_MAT_LOGNORMAL_SCALAR) return 2;
  if (d.material == MQ_MAT_KL) return d.n_modes;
  return 3;
}

int validate_desc(const mq_problem_desc* d) {
  if (!d) return fail(MQ_ERR_INVALID_ARG, "null problem description");
  if (d->n_nodes < 3 || d->n_nodes > 8193) return fail(MQ_ERR_INVALID_ARG, "n_nodes must be in [3, 8193]");
  if (d->material < 0 || d->material > 2) return fail(MQ_ERR_INVALID_ARG, "unknown material kind");
  if (d->precision != MQ_PREC_FP64 && d->precision != MQ_PREC_MIXED)
    return fail(MQ_ERR_INVALID_ARG, "unknown precision");
  if (d->path < 0 || d->path > 3) return fail(MQ_ERR_INVALID_ARG, "unknown path");
  if (d->mem_kind != MQ_MEM_DEVICE && d->mem_kind != MQ_MEM_HOST) return fail(MQ_ERR_INVALID_ARG, "unknown mem_kind");
  if (d->mass != MQ_MASS_CONSISTENT && d->mass != MQ_MASS_LUMPED) return fail(MQ_ERR_INVALID_ARG, "unknown mass kind");
  if (!(d->conductor[0] < d->conductor[1]) || !(d->conductor[2] < d->conductor[3]))
    return fail(MQ_ERR_INVALID_ARG, "empty conductor box");
  if (!(d->strip[0] <= d->strip[1])) return fail(MQ_ERR_INVALID_ARG, "bad strip");
  if (!(d->freq > 0) || !std::isfinite(d->J0)) return fail(MQ_ERR_INVALID_ARG, "bad source");
  if (!(d->sigma0 >= 0) || !(d->nu_cond > 0) || !(d->nu_air > 0))
    return fail(MQ_ERR_INVALID_ARG, "bad material constants");
  if (d->material == MQ_MAT_KL && (d->n_modes < 1 || d->n_modes > 16 || !(d->corr_len > 0)))
    return fail(MQ_ERR_INVALID_ARG, "KL needs 1..16 modes and corr_len > 0");
  if (!(d->tol > 0) || !(d->inner_rtol > 0) || !(d->inner_rtol < 1))
    return fail(MQ_ERR_INVALID_ARG, "tolerances must be positive (inner_rtol < 1)");
  if (d->max_iter < 1 || d->max_sweeps < 1) return fail(MQ_ERR_INVALID_ARG, "max_iter and max_sweeps must be >= 1");
  if (d->material == MQ_MAT_NONLINEAR && (d->picard_max < 1 || !(d->picard_tol > 0)))
    return fail(MQ_ERR_INVALID_ARG, "bad Picard parameters");
  if (d->precond < 0 || d->precond > 2) return fail(MQ_ERR_INVALID_ARG, "unknown preconditioner");
  if (!(d->mg_omega >= 0) || !(d->mg_omega < 1)) return fail(MQ_ERR_INVALID_ARG, "mg_omega must be in [0, 1)");
  if (d->tile < 0 || d->tile > 2) return fail(MQ_ERR_INVALID_ARG, "tile must be 0, 1 or 2");
  if (d->mg_levels < 0 || d->mg_coarse_sweeps < 0 || d->mg_coarse_sweeps > 64)
    return fail(MQ_ERR_INVALID_ARG, "mg_levels >= 0 and 0 <= mg_coarse_sweeps <= 64 required");
  if (d->split_steps < -1) return fail(MQ_ERR_INVALID_ARG, "split_steps must be >= -1");
  if (d->mg_block_min < 0) return fail(MQ_ERR_INVALID_ARG, "mg_block_min must be >= 0");
  return MQ_OK;
}

int check_finite(mq_problem* p, const double* x, size_t n) {
  HIP_TRY(launch_fill_zero_i(p->dflag.get(), 1, p->stream));
  HIP_TRY(launch_check_finite(x, n, p->dflag.get(), p->stream));
  int bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, p->dflag.get(), sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (bad) return fail(MQ_ERR_NONFINITE, "xi contains NaN or Inf");
  return MQ_OK;
}

struct RunOut {
  int status = MQ_OK;
  // host time (now_ms) of the call's start: when > 0, run_instances reports
  // latency as the time from it until a sample's Q is readable in host memory
  double t_submit_ms = 0;
  // two work queues in one launch: entries [0, queue0) form the first queue,
  // taken first by workgroups [0, grid0); -1: one queue
  int queue0 = -1, grid0 = -1;
  // device time from the launch's first start to the last end of each queue's entries
  double done_ms[2] = {0, 0};
  std::vector<int> flags;  // FLAG_* bits per instance, appended by each run_instances call in its order
  double kernel_ms = 0;
  int grid = 0, block = 0;
};

// Launch one persistent time-stepping kernel over `insts` (host copy).
// Makespan, in steps, of the greedy work queue over `slots` workgroups: each
// item starts when a workgroup is free and its predecessor (dep >= 0) is done.
double queue_makespan(const std::vector<std::pair<int, int>>& items, size_t slots) {
  std::priority_queue<double, std::vector<double>, std::greater<double>> freeq;
  for (size_t s = 0; s < slots; ++s) freeq.push(0.0);
  std::vector<double> end(items.size());
  double mk = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    double t = freeq.top();
    freeq.pop();
    if (items[i].second >= 0) t = std::max(t, end[items[i].second]);
    end[i] = t + items[i].first;
    mk = std::max(mk, end[i]);
    freeq.push(end[i]);
  }
  return mk;
}

// Tail splitting: with more instances than slots, instances of at most a
// quarter (or half) of the longest one's steps become chains of S-step pieces,
// queued after the other instances one round of pieces at a time; the threshold
// whose simulated makespan is shortest (by more than 2%, counting two steps per
// piece for its set-up) is used.  Entry e of the plan runs steps
// [first, first + len) of instance orig and waits for entry dep (-1: none).
struct PiecePlan {
  std::vector<int> orig, first, len, dep;
  double mk0 = 0, mk = 0;
  bool split = false;
};

PiecePlan plan_pieces(const std::vector<int>& steps, size_t slots, int S) {
  PiecePlan pl;
  const size_t n = steps.size();
  std::vector<std::pair<int, int>> base;
  int max_steps = 0;
  for (int s : steps) {
    base.push_back({s, -1});
    max_steps = std::max(max_steps, s);
  }
  pl.mk0 = pl.mk = queue_makespan(base, std::max<size_t>(slots, 1));
  auto whole = [&]() {
    for (size_t i = 0; i < n; ++i) {
      pl.orig.push_back((int)i);
      pl.first.push_back(0);
      pl.len.push_back(steps[i]);
      pl.dep.push_back(-1);
    }
  };
  if (S < 1 || n <= slots) {
    whole();
    return pl;
  }
  constexpr int SETUP = 2;
  auto build = [&](int th, PiecePlan& out) {
    std::vector<size_t> sp;
    for (size_t i = 0; i < n; ++i) {
      if (steps[i] <= th && steps[i] >= 2 * S) {
        sp.push_back(i);
      } else {
        out.orig.push_back((int)i);
        out.first.push_back(0);
        out.len.push_back(steps[i]);
        out.dep.push_back(-1);
      }
    }
    std::vector<int> last(sp.size(), -1);
    for (int k = 0;; ++k) {
      bool any = false;
      for (size_t a = 0; a < sp.size(); ++a) {
        const int done = k * S;
        if (done >= steps[sp[a]]) continue;
        any = true;
        out.orig.push_back((int)sp[a]);
        out.first.push_back(done);
        out.len.push_back(std::min(S, steps[sp[a]] - done));
        out.dep.push_back(last[a]);
        last[a] = (int)out.orig.size() - 1;
      }
      if (!any) break;
    }
    return !sp.empty();
  };
  double best = pl.mk0 * 0.98;
  int best_th = 0;
  for (int th : {max_steps / 4, max_steps / 2}) {
    PiecePlan c;
    if (!build(th, c)) continue;
    std::vector<std::pair<int, int>> q;
    for (size_t e = 0; e < c.orig.size(); ++e) {
      const bool piece = c.len[e] != steps[c.orig[e]];
      q.push_back({c.len[e] + (piece ? SETUP : 0), c.dep[e]});
    }
    const double mk = queue_makespan(q, slots);
    if (mk < best) {
      best = mk;
      best_th = th;
    }
  }
  if (best_th == 0) {
    whole();
    return pl;
  }
  build(best_th, pl);
  pl.mk = best;
  pl.split = true;
  return pl;
}

// Launch entries of a tail-split plan (resident path, linear material, plain
// instances).  The pieces of an instance carry the state through `buf` (per
// split instance: a, then the carry record) and order themselves through
// `flags` (one per piece but the last).
struct Split {
  std::vector<Inst> pieces;
  std::vector<int> orig;  // original instance of each entry
  TmpPtr<double> buf;
  TmpPtr<int> flags;
};

int plan_split(mq_problem* p, const std::vector<Inst>& insts, Split& out, bool* used) {
  *used = false;
  const size_t n = insts.size();
  size_t slots = std::min(n, max_slots(p));
  const int S = p->d.split_steps == 0 ? 32 : p->d.split_steps;
  if (p->d.split_steps < 0 || p->path != MQ_PATH_RESIDENT || p->d.material == MQ_MAT_NONLINEAR || n <= slots)
    return MQ_OK;
  std::vector<int> steps;
  for (const Inst& in : insts) {
    if (in.n_chain > 0 || in.carry || in.dep_wait || in.dep_done) return MQ_OK;
    steps.push_back(in.n_steps);
  }
  const PiecePlan pl = plan_pieces(steps, slots, S);
  if (!pl.split) return MQ_OK;
  const size_t m = pl.orig.size();
  // per split instance a state buffer; per entry with a successor a flag
  const Geom& g = p->hm.g;
  const size_t FS = (size_t)g.N * g.P, per = 3 * FS + 1;
  std::vector<int> buf_of(n, -1), flag_of(m, -1);
  int n_buf = 0, n_flags = 0;
  for (size_t e = 0; e < m; ++e) {
    const int o = pl.orig[e];
    if (pl.len[e] == steps[o]) continue;
    if (buf_of[o] < 0) buf_of[o] = n_buf++;
    if (pl.first[e] + pl.len[e] < steps[o]) flag_of[e] = n_flags++;
  }
  if (per * (size_t)n_buf * sizeof(double) > ((size_t)8 << 30)) return MQ_OK;  // keep the state buffers modest
  HIP_TRY(tmp_alloc(out.buf, per * (size_t)n_buf, p->stream));
  HIP_TRY(tmp_alloc(out.flags, (size_t)n_flags, p->stream));
  HIP_TRY(launch_fill_zero_i(out.flags.get(), (size_t)n_flags, p->stream));
  for (size_t e = 0; e < m; ++e) {
    const Inst& o = insts[pl.orig[e]];
    out.orig.push_back(pl.orig[e]);
    if (pl.len[e] == o.n_steps) {
      out.pieces.push_back(o);
      continue;
    }
    const bool first = pl.first[e] == 0, lastp = pl.first[e] + pl.len[e] == o.n_steps;
    double* abuf = out.buf.get() + per * (size_t)buf_of[pl.orig[e]];
    Inst pc = o;
    pc.k0 = o.k0 + pl.first[e];
    pc.n_steps = pl.len[e];
    pc.a_init = first ? o.a_init : abuf;
    pc.a_out = lastp ? o.a_out : abuf;
    pc.q_out = lastp ? o.q_out : nullptr;
    pc.carry = abuf + FS;
    pc.carry_in = first ? 0 : 1;
    pc.dep_wait = pl.dep[e] >= 0 ? out.flags.get() + flag_of[pl.dep[e]] : nullptr;
    pc.dep_done = lastp ? nullptr : out.flags.get() + flag_of[e];
    out.pieces.push_back(pc);
  }
  *used = true;
  return MQ_OK;
}

// fixed (nullable): a CallMem over a fixed region; the launch then takes its
// instance table, statistics and work slots from it (as many slots as fit),
// splits nothing, creates no events and allocates nothing.
int run_instances(mq_problem* p, std::vector<Inst>& insts, mq_run_stats* st, RunOut* ro,
                  std::vector<int>* stat_host, CallMem* fixed = nullptr) {
  const int n = (int)insts.size();
  if (n == 0) return MQ_OK;
  if (fixed && !fixed->fixed()) fixed = nullptr;
  if (p->path == MQ_PATH_WIDE) {
    if (fixed) return fail(MQ_ERR_INVALID_ARG, "the wide path allocates its own workspace");
    (void)stat_host;
    int status = MQ_OK;
    const int rc = run_wide(p, insts, st, &status, &ro->flags);
    if (rc) return rc;
    ro->status = std::max(ro->status, status);
    return MQ_OK;
  }
  Split spl;
  bool split = false;
  int rc = (stat_host || fixed) ? MQ_OK : plan_split(p, insts, spl, &split);
  if (rc) return rc;
  std::vector<Inst>& run = split ? spl.pieces : insts;
  const int nr = (int)run.size();
  CallMem own;
  own.use_stream(p->stream);
  CallMem& mem = fixed ? *fixed : own;
  int* dstat = nullptr;
  HIP_TRY(mem.get(dstat, (size_t)nr * STAT_N));
  HIP_TRY(launch_fill_zero_i(dstat, (size_t)nr * STAT_N, p->stream));
  for (int i = 0; i < nr; ++i) run[i].stat = dstat + STAT_N * i;
  // host-visible completion records (coherent pinned memory)
  HostDone* rec = nullptr;
  if (ro->t_submit_ms > 0 && !fixed) {
    if (p->done_cap < (size_t)nr) {
      HIP_TRY(hipStreamSynchronize(p->stream));
      p->done_rec.reset();
      p->done_cap = 0;
      HostDone* h = nullptr;
      HIP_TRY(hipHostMalloc((void**)&h, (size_t)nr * sizeof(HostDone), hipHostMallocCoherent | hipHostMallocMapped));
      p->done_rec.reset(h);
      p->done_cap = (size_t)nr;
    }
    rec = p->done_rec.get();
    std::memset((void*)rec, 0, (size_t)nr * sizeof(HostDone));
    HostDone* drec = nullptr;
    HIP_TRY(hipHostGetDevicePointer((void**)&drec, rec, 0));
    for (int i = 0; i < nr; ++i) run[i].host_done = drec + i;
  }
  Inst* dinst = nullptr;
  HIP_TRY(mem.get(dinst, nr));
  HIP_TRY(hipMemcpyAsync(dinst, run.data(), nr * sizeof(Inst), hipMemcpyHostToDevice, p->stream));
  size_t slots = std::min<size_t>((size_t)nr, max_slots(p));
  double* fwork = nullptr;
  if (fixed) {
    // as many work slots as the region has left (zeroed: the kernels rely on a
    // zero boundary ring, and the region holds whatever the last call left)
    const size_t sd = slot_doubles(p);
    slots = std::min(slots, mem.left() / CallMem::rounded(sd * sizeof(double)));
    if (slots < 1) return fail(MQ_ERR_INVALID_ARG, "the fixed workspace has no room for a work slot");
    HIP_TRY(mem.get(fwork, slots * sd));
    HIP_TRY(launch_fill_zero(fwork, slots * sd, p->stream));
  } else {
    rc = ensure_work(p, slots);
    if (rc) return rc;
  }
  // launch timing: events on the stream, or (fixed) the host clock around the
  // launch and the stream's end
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double t_launch = 0;
  if (!fixed) {
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, p->stream));
  } else {
    HIP_TRY(hipStreamSynchronize(p->stream));
    t_launch = now_ms();
  }
  const bool para = std::any_of(run.begin(), run.end(), [](const Inst& in) { return in.para != nullptr; });
  rc = launch_persistent(p, dinst, nr, &ro->grid, &ro->block, fwork, fixed ? slots : 0, ro->queue0, ro->grid0, para);
  if (rc) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
  }
  if (e1) HIP_TRY(hipEventRecord(e1, p->stream));
  // host time at which each entry's record became visible (polled while the
  // launch runs; the stream's end also ends the wait)
  std::vector<double> seen;
  if (rec) {
    seen.assign(nr, -1.0);
    int left = nr;
    for (;;) {
      for (int i = 0; i < nr; ++i)
        if (seen[i] < 0 && __atomic_load_n(&rec[i].done, __ATOMIC_ACQUIRE)) {
          seen[i] = now_ms();
          --left;
        }
      if (left == 0) break;
      const hipError_t q = hipStreamQuery(p->stream);
      if (q != hipErrorNotReady) {
        const double t = now_ms();
        for (int i = 0; i < nr; ++i)
          if (seen[i] < 0) seen[i] = t;
        break;
      }
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
  std::vector<int> sh((size_t)nr * STAT_N);
  float ms = 0;
  if (fixed) {
    HIP_TRY(hipStreamSynchronize(p->stream));
    ms = (float)(now_ms() - t_launch);
  }
  HIP_TRY(hipMemcpyAsync(sh.data(), dstat, sh.size() * sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (!fixed) {
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  ro->kernel_ms += ms;
  // per-entry device wall-clock stamps -> per-group completion latency
  auto stamp = [&](int i, int w) {
    const int* q = &sh[(size_t)STAT_N * i + 4 + 2 * w];
    return (uint64_t)(uint32_t)q[0] | ((uint64_t)(uint32_t)q[1] << 32);
  };
  uint64_t t_first = ~0ull;
  for (int i = 0; i < nr; ++i) t_first = std::min(t_first, stamp(i, 0));
  for (int i = 0; i < nr; ++i) {
    const int qq = (ro->queue0 >= 0 && i >= ro->queue0) ? 1 : 0;
    ro->done_ms[qq] = std::max(ro->done_ms[qq], (double)(stamp(i, 1) - t_first) / p->wall_khz);
  }
  {
    // per group (sample): host-visible completion after the call's start, or
    // device time after the first entry started
    std::vector<std::pair<int, double>> done;
    for (int i = 0; i < nr; ++i)
      done.push_back({run[i].group, rec ? seen[i] - ro->t_submit_ms : (double)(stamp(i, 1) - t_first) / p->wall_khz});
    std::sort(done.begin(), done.end());
    std::vector<double> lat;
    for (size_t a = 0; a < done.size();) {
      double e = 0;
      size_t b = a;
      for (; b < done.size() && done[b].first == done[a].first; ++b) e = std::max(e, done[b].second);
      lat.push_back(e);
      a = b;
    }
    if (st && !lat.empty()) {
      std::sort(lat.begin(), lat.end());
      auto pct = [&](double f) {
        const size_t k = (size_t)std::min<double>(lat.size() - 1, std::ceil(f * lat.size()) - 1);
        return lat[k];
      };
      st->lat_p50_ms = pct(0.50);
      st->lat_p99_ms = pct(0.99);
      st->lat_max_ms = lat.back();
    }
  }
  // counters per entry; flags per original instance (its pieces OR-ed)
  std::vector<int> oflags(n, 0);
  for (int i = 0; i < nr; ++i) {
    const int* s4 = &sh[(size_t)STAT_N * i];
    oflags[split ? spl.orig[i] : i] |= s4[3];
    if (st) {
      st->sample_steps += (int64_t)run[i].n_steps * std::max(1, run[i].n_chain);
      st->inner_iters += s4[0];
      st->sweeps += s4[1];
      st->max_inner_per_step = std::max(st->max_inner_per_step, s4[2]);
      for (int q = 0; q < 8; ++q) st->phase_ms[q] += (double)(uint32_t)s4[8 + q] * 16.0 / p->wall_khz;
      st->busy_ms += (double)(stamp(i, 1) - stamp(i, 0)) / p->wall_khz;
      st->picard_iters += s4[16];
    }
  }
  for (int i = 0; i < n; ++i) {
    if (st) {
      st->n_instances += 1;
      if (oflags[i] & (FLAG_NOT_CONVERGED | FLAG_PICARD_CAP)) st->n_not_converged++;
      if (oflags[i] & FLAG_FAILED) st->n_failed++;
    }
    if (oflags[i] & FLAG_WARN) ro->status = MQ_WARN_NOT_CONVERGED;
  }
  ro->flags.insert(ro->flags.end(), oflags.begin(), oflags.end());
  if (st) {
    st->path = p->path;
    st->grid = ro->grid;
    st->block = ro->block;
    st->kernel_ms += ms;
    st->n_pieces += split ? nr : 0;
  }
  if (stat_host) *stat_host = std::move(sh);
  return MQ_OK;
}

// Assemble the tables of n samples into `tables` ([n][tab_stride], device).
int assemble_into(mq_problem* p, const double* xi, int n, double* tables) {
  const Geom& g = p->hm.g;
  HIP_TRY(launch_assemble(g, p->hm.cr, p->dcond.get(), p->dkl.get(), p->hm.n_modes, p->d.material, xi,
                          p->n_xi, n, p->mat, tables, p->stream));
  if (p->d.mass == MQ_MASS_LUMPED) HIP_TRY(launch_lump_mass(g, n, tables, p->stream));
  return MQ_OK;
}

int assemble(mq_problem* p, const double* xi, int n, TmpPtr<double>& tables) {
  HIP_TRY(tmp_alloc(tables, (size_t)n * tab_stride(p->hm.g), p->stream));
  return assemble_into(p, xi, n, tables.get());
}

// Inputs of one level run; `mem` owns them (or slices a fixed region).
struct LevelBufs {
  CallMem mem;
  double* tables = nullptr;
  double* src_f = nullptr;
  double* src_c = nullptr;
  double* afull = nullptr;
  std::vector<double*> afull_ptr;
};

// Append the instances of one level (fine first) and allocate their inputs.
int prepare_level(mq_problem* p, const mq_level_desc* lv, int n, const double* xi, double* qf,
                  double* qc, bool want_state, LevelBufs& lb, std::vector<Inst>& fine,
                  std::vector<Inst>& coarse, int group0) {
  if (!lv) return fail(MQ_ERR_INVALID_ARG, "null level description");
  if (n < 1) return fail(MQ_ERR_INVALID_ARG, "n_samples must be >= 1");
  if (lv->steps_per_period < 1 || lv->n_periods < 1 || lv->coarse_steps_per_period < 0)
    return fail(MQ_ERR_INVALID_ARG, "steps_per_period, n_periods >= 1 and coarse_steps_per_period >= 0 required");
  if (!xi || !qf) return fail(MQ_ERR_INVALID_ARG, "xi and q_fine are required");
  if (lv->coarse_steps_per_period > 0 && !qc) return fail(MQ_ERR_INVALID_ARG, "q_coarse required for a coupled level");
  const int64_t nf = (int64_t)lv->steps_per_period * lv->n_periods;
  const int64_t nc = (int64_t)lv->coarse_steps_per_period * lv->n_periods;
  if (nf > (1 << 24) || nc > (1 << 24)) return fail(MQ_ERR_INVALID_ARG, "too many steps");
  int rc = check_finite(p, xi, (size_t)n * p->n_xi);
  if (rc) return rc;
  if (!lb.mem.fixed()) lb.mem.use_stream(p->stream);
  const Geom& g = p->hm.g;
  HIP_TRY(lb.mem.get(lb.tables, (size_t)n * tab_stride(g)));
  rc = assemble_into(p, xi, n, lb.tables);
  if (rc) return rc;
  const double T = lv->n_periods / p->d.freq;
  const double dtf = 1.0 / (p->d.freq * lv->steps_per_period);
  auto sf = source_table(p->d, dtf, (int)nf);
  HIP_TRY(lb.mem.get(lb.src_f, sf.size()));
  HIP_TRY(hipMemcpyAsync(lb.src_f, sf.data(), sf.size() * sizeof(double), hipMemcpyHostToDevice, p->stream));
  double dtc = 0;
  if (nc > 0) {
    dtc = 1.0 / (p->d.freq * lv->coarse_steps_per_period);
    auto sc = source_table(p->d, dtc, (int)nc);
    HIP_TRY(lb.mem.get(lb.src_c, sc.size()));
    HIP_TRY(hipMemcpyAsync(lb.src_c, sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, p->stream));
    // the copy's host vector must outlive the async copy
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  const size_t FS = (size_t)g.N * g.P;
  if (want_state) {
    HIP_TRY(lb.mem.get(lb.afull, FS * n));
    lb.afull_ptr.resize(n);
    for (int s = 0; s < n; ++s) lb.afull_ptr[s] = lb.afull + FS * s;
  }
  for (int s = 0; s < n; ++s) {
    Inst in{};
    in.tab = lb.tables + (size_t)s * tab_stride(g);
    in.src = lb.src_f;
    in.a_init = p->a0.get();  // null: a_0 = 0
    in.a_out = want_state ? lb.afull_ptr[s] : nullptr;
    in.q_out = qf + s;
    in.q_scale = 1.0 / T;
    in.dt = dtf;
    in.n_steps = (int)nf;
    in.sample = s;
    in.group = group0 + s;
    fine.push_back(in);
    if (nc > 0) {
      Inst ic = in;
      ic.src = lb.src_c;
      ic.a_out = nullptr;
      ic.q_out = qc + s;
      ic.dt = dtc;
      ic.n_steps = (int)nc;
      coarse.push_back(ic);
    }
  }
  return MQ_OK;
}

// Handles set up with mem_kind = MQ_MEM_HOST take host arrays in the staged calls.
bool host_mode(const mq_problem* p) { return p && p->d.mem_kind == MQ_MEM_HOST; }

// mq_last_flags reports level, multilevel and Parareal runs only: the other run
// calls leave its list empty whichever inner runs they made.
struct FlagsClearedOnReturn {
  ~FlagsClearedOnReturn() { last_flags().clear(); }
};

int refuse_host(const mq_problem* p) {
  if (host_mode(p))
    return fail(MQ_ERR_INVALID_ARG, "this call takes device pointers (the handle was set up with mem_kind = MQ_MEM_HOST)");
  return MQ_OK;
}

}  // namespace

extern "C" {

const char* mq_last_error(void) { return last_error().c_str(); }

int mq_last_flags(int32_t* flags, int64_t cap, int64_t* n_out) {
  if (!n_out || cap < 0 || (cap > 0 && !flags)) return fail(MQ_ERR_INVALID_ARG, "invalid arguments");
  const std::vector<int32_t>& f = last_flags();
  *n_out = (int64_t)f.size();
  for (int64_t i = 0; i < cap && i < (int64_t)f.size(); ++i) flags[i] = f[i];
  return MQ_OK;
}

int mq_version(void) { return 1; }

int fem_setup(const mq_problem_desc* d, void* stream, mq_problem** out) {
  if (!out) return fail(MQ_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  int rc = validate_desc(d);
  if (rc) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(MQ_ERR_NO_DEVICE, "no HIP device");
  std::unique_ptr<mq_problem> p(new mq_problem());
  p->d = *d;
  try {
    p->hm = build_host_mesh(*d);
  } catch (const std::exception& ex) {
    return fail(MQ_ERR_INVALID_ARG, std::string("mesh set-up: ") + ex.what());
  }
  HIP_TRY(hipGetDevice(&p->device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, p->device));
  p->num_cu = prop.multiProcessorCount;
  p->lds_limit = (int)prop.sharedMemPerBlock;
  int optin = 0;
  if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, p->device) == hipSuccess && optin > p->lds_limit)
    p->lds_limit = optin;
  p->stream = (hipStream_t)stream;
  int wk = 0;
  if (hipDeviceGetAttribute(&wk, hipDeviceAttributeWallClockRate, p->device) == hipSuccess && wk > 0)
    p->wall_khz = wk;
  p->n_xi = n_xi_of(*d);
  // multigrid hierarchy (resident path only); fall back to Jacobi if it does not fit
  // path and preconditioner: the resident path (with multigrid if its LDS
  // holds the hierarchy, else Jacobi) where it fits, else the streaming path
  // (with multigrid on 2^k + 1 meshes)
  p->tile = d->tile > 0 ? d->tile : 1;
  const Geom& g0 = p->hm.g;
  const bool want_mg = d->precond != MQ_PRECOND_JACOBI;
  const int lp = resident_lp(g0, p->tile);
  MGGeom rmg{};
  const bool res_mg = want_mg && lp > 0 && d->path != MQ_PATH_STREAMING && build_mg(g0, lp, &rmg) &&
                      resident_supported(g0, &rmg, d->precision, p->lds_limit, nullptr, p->tile);
  p->resident_ok = resident_supported(g0, res_mg ? &rmg : nullptr, d->precision, p->lds_limit, &p->lds_bytes, p->tile);
  if (d->path == MQ_PATH_RESIDENT && !p->resident_ok)
    return fail(MQ_ERR_INVALID_ARG, "the resident path does not fit this mesh/precision");
  if (d->material == MQ_MAT_NONLINEAR && (!p->resident_ok || d->path == MQ_PATH_STREAMING))
    return fail(MQ_ERR_INVALID_ARG, "the nonlinear (Picard) material runs on the resident path only");
  p->path = (d->path == MQ_PATH_STREAMING || !p->resident_ok) ? MQ_PATH_STREAMING : MQ_PATH_RESIDENT;
  if (d->path == MQ_PATH_WIDE) {
    if (d->material == MQ_MAT_NONLINEAR) return fail(MQ_ERR_INVALID_ARG, "the wide path needs a linear material");
    p->path = MQ_PATH_WIDE;
  }
  p->mg = MGGeom{};
  if (p->path == MQ_PATH_RESIDENT) {
    if (res_mg) p->mg = rmg;
  } else if (want_mg && !build_mg(g0, 0, &p->mg)) {
    p->mg = MGGeom{};
  }
  if (d->precond == MQ_PRECOND_MULTIGRID && p->mg.nlev == 0)
    return fail(MQ_ERR_INVALID_ARG, "multigrid needs n_nodes = 2^k + 1 (and, on the resident path, room in LDS)");
  p->precond = p->mg.nlev > 0 ? MQ_PRECOND_MULTIGRID : MQ_PRECOND_JACOBI;
  const double m[10] = {d->sigma0, d->nu_cond, d->nu_air, d->s_sigma, d->s_nu, d->s_kl, d->k1, d->k2, d->k3, d->s_k};
  std::memcpy(p->mat, m, sizeof(m));
  const Geom& g = p->hm.g;
  HIP_TRY(dev_alloc(p->dS, p->hm.S.size()));
  HIP_TRY(copy_sync(p->dS.get(), p->hm.S.data(), p->hm.S.size() * sizeof(double), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(dev_alloc(p->dcond, p->hm.cond.size()));
  HIP_TRY(copy_sync(p->dcond.get(), p->hm.cond.data(), p->hm.cond.size(), hipMemcpyHostToDevice, p->stream));
  if (!p->hm.kl.empty()) {
    HIP_TRY(dev_alloc(p->dkl, p->hm.kl.size()));
    HIP_TRY(copy_sync(p->dkl.get(), p->hm.kl.data(), p->hm.kl.size() * sizeof(double), hipMemcpyHostToDevice, p->stream));
  }
  HIP_TRY(dev_alloc(p->dcounter, 4));  // work queue: two positions, split, first-queue workgroups
  HIP_TRY(dev_alloc(p->dflag, 1));
  HIP_TRY(noalloc_workspace(p->device, &p->scratch));
  (void)g;
  *out = p.release();
  return MQ_OK;
}

int mq_problem_destroy(mq_problem* p) {
  if (!p) return MQ_OK;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  else (void)hipDeviceSynchronize();
  delete p;
  return MQ_OK;
}

int mq_ndof(const mq_problem* p, int64_t* nd) {
  if (!p || !nd) return fail(MQ_ERR_INVALID_ARG, "null argument");
  *nd = (int64_t)p->hm.g.n * p->hm.g.n;
  return MQ_OK;
}

static int set_initial_state_dev(mq_problem* p, const double* a0) {
  if (!p) return fail(MQ_ERR_INVALID_ARG, "null problem");
  if (!a0) {
    HIP_TRY(hipStreamSynchronize(p->stream));
    p->a0.reset();
    return MQ_OK;
  }
  const Geom& g = p->hm.g;
  const size_t nd = (size_t)g.n * g.n, FS = (size_t)g.N * g.P;
  int rc = check_finite(p, a0, nd);
  if (rc == MQ_ERR_NONFINITE) return fail(rc, "a0 contains NaN or Inf");
  if (rc) return rc;
  if (!p->a0) HIP_TRY(dev_alloc(p->a0, FS));
  HIP_TRY(launch_fill_zero(p->a0.get(), FS, p->stream));
  TmpPtr<double*> dptr;
  HIP_TRY(tmp_alloc(dptr, 1, p->stream));
  double* full = p->a0.get();
  HIP_TRY(copy_sync(dptr.get(), &full, sizeof(double*), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(launch_to_full(g, 1, a0, dptr.get(), p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return MQ_OK;
}

int mq_problem_info_get(const mq_problem* p, mq_problem_info* info) {
  if (!p || !info) return fail(MQ_ERR_INVALID_ARG, "null argument");
  std::memset(info, 0, sizeof(*info));
  const Geom& g = p->hm.g;
  info->n_nodes = g.N;
  info->n_dof = g.n * g.n;
  info->pitch = g.P;
  info->n_xi = p->n_xi;
  info->box[0] = g.bx0;
  info->box[1] = g.bx1;
  info->box[2] = g.by0;
  info->box[3] = g.by1;
  info->resident_ok = p->resident_ok;
  info->lds_bytes = p->lds_bytes;
  info->precond = p->precond;
  info->mg_levels = p->mg.nlev;
  info->n_modes_used = p->hm.n_modes;
  for (int k = 0; k < p->hm.n_modes && k < 16; ++k) info->kl_lambda[k] = p->hm.kl_lambda[k];
  if (p->path == MQ_PATH_RESIDENT) info->tile = (p->tile == 2 && g.n >= 64 && g.n <= 127) ? 2 : 1;
  else info->tile = p->tile;
  info->block = ie_block_threads(p->hm.g, p->path, p->tile);
  return MQ_OK;
}

// region (nullable): take every per-call buffer from this fixed device region
// instead of allocating (the allocation-free entry point).
static int level_run_dev(mq_problem* p, const mq_level_desc* lv, int32_t n_samples, const double* xi,
                         double* q_fine, double* q_coarse, double* final_state, mq_run_stats* st,
                         char* region = nullptr, size_t region_bytes = 0) {
  last_flags().clear();
  if (!p) return fail(MQ_ERR_INVALID_ARG, "null problem");
  const double t0 = now_ms();
  if (st) std::memset(st, 0, sizeof(*st));
  LevelBufs lb;
  if (region) lb.mem.use_region(region, region_bytes);
  std::vector<Inst> fine, coarse;
  int rc = prepare_level(p, lv, n_samples, xi, q_fine, q_coarse, final_state != nullptr, lb, fine, coarse, 0);
  if (rc) return rc;
  double** dptr = nullptr;
  if (final_state) HIP_TRY(lb.mem.get(dptr, lb.afull_ptr.size()));
  std::vector<Inst> all = fine;
  all.insert(all.end(), coarse.begin(), coarse.end());
  RunOut ro;
  if (!region) ro.t_submit_ms = t0;
  rc = run_instances(p, all, st, &ro, nullptr, region ? &lb.mem : nullptr);
  if (rc) return rc;
  last_flags().assign(ro.flags.begin(), ro.flags.end());  // fine 0..n-1, then coarse 0..n-1
  if (final_state) {
    HIP_TRY(hipMemcpyAsync(dptr, lb.afull_ptr.data(), lb.afull_ptr.size() * sizeof(double*), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(launch_to_interior(p->hm.g, n_samples, dptr, final_state, p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  if (st) st->total_ms = now_ms() - t0;
  return ro.status;
}

// Bytes that a level run takes from the fixed workspace before its work slots
// (the slices level_run_dev carves, in its order), plus one work slot.
static size_t noalloc_need(const mq_problem* p, int64_t n, int64_t nf, int64_t nc, bool state) {
  const Geom& g = p->hm.g;
  const size_t FS = (size_t)g.N * g.P;
  const int64_t n_inst = nc > 0 ? 2 * n : n;
  size_t b = CallMem::rounded(n * tab_stride(g) * sizeof(double));
  b += CallMem::rounded((nf + 1) * sizeof(double));
  if (nc > 0) b += CallMem::rounded((nc + 1) * sizeof(double));
  if (state) b += CallMem::rounded(FS * n * sizeof(double)) + CallMem::rounded(n * sizeof(double*));
  b += CallMem::rounded(n_inst * STAT_N * sizeof(int)) + CallMem::rounded(n_inst * sizeof(Inst));
  b += CallMem::rounded(slot_doubles(p) * sizeof(double));
  return b;
}

static int multilevel_run_dev(mq_problem* p, int32_t n_levels, const mq_level_desc* lv,
                              const int32_t* n_samples, const double* const* xi, double* const* q_fine,
                              double* const* q_coarse, mq_run_stats* st) {
  last_flags().clear();
  if (!p || !lv || !n_samples || !xi || !q_fine || !q_coarse) return fail(MQ_ERR_INVALID_ARG, "null argument");
  if (n_levels < 1 || n_levels > 64) return fail(MQ_ERR_INVALID_ARG, "n_levels must be in [1, 64]");
  const double t0 = now_ms();
  if (st) std::memset(st, 0, sizeof(*st));
  std::vector<LevelBufs> lbs(n_levels);
  std::vector<Inst> all;
  // (steps, position in the caller's flag order, instance): per level its fine
  // instances, then its coarse ones
  struct Keyed {
    int64_t steps;
    int pos;
    Inst in;
  };
  std::vector<Keyed> keyed;
  int group0 = 0;
  for (int l = 0; l < n_levels; ++l) {
    std::vector<Inst> f, c;
    int rc = prepare_level(p, &lv[l], n_samples[l], xi[l], q_fine[l], q_coarse[l], false, lbs[l], f, c, group0);
    group0 += n_samples[l];
    if (rc) return rc;
    for (auto& i : f) keyed.push_back({i.n_steps, (int)keyed.size(), i});
    for (auto& i : c) keyed.push_back({i.n_steps, (int)keyed.size(), i});
  }
  // longest instances first; stable so that equal lengths keep their order
  std::stable_sort(keyed.begin(), keyed.end(), [](const Keyed& a, const Keyed& b) { return a.steps > b.steps; });
  for (auto& k : keyed) all.push_back(k.in);
  RunOut ro;
  ro.t_submit_ms = t0;
  int rc = run_instances(p, all, st, &ro, nullptr);
  if (rc) return rc;
  std::vector<int32_t>& lf = last_flags();
  lf.assign(keyed.size(), 0);
  for (size_t i = 0; i < keyed.size(); ++i) lf[keyed[i].pos] = ro.flags[i];
  if (st) st->total_ms = now_ms() - t0;
  return ro.status;
}

int mlmc_adaptive_run(mq_problem* p, int32_t n_levels, const mq_level_desc* lv, const int32_t* n_max,
                      const double* const* xi, double* const* q_fine, double* const* q_coarse,
                      const mq_adaptive_desc* ad, int32_t* n_used, double* out, mq_run_stats* st) {
  const FlagsClearedOnReturn no_flags;
  if (int rh = refuse_host(p)) return rh;
  if (!p || !lv || !n_max || !xi || !q_fine || !q_coarse || !ad || !n_used || !out)
    return fail(MQ_ERR_INVALID_ARG, "null argument");
  if (n_levels < 1 || n_levels > 64) return fail(MQ_ERR_INVALID_ARG, "n_levels must be in [1, 64]");
  if (!(ad->target_rmse > 0) || ad->n_pilot < 2 || ad->max_rounds < 0 || !(ad->var_fraction >= 0) ||
      !(ad->var_fraction < 1))
    return fail(MQ_ERR_INVALID_ARG, "target_rmse > 0, n_pilot >= 2, 0 <= var_fraction < 1 required");
  for (int l = 0; l < n_levels; ++l) {
    if (n_max[l] < ad->n_pilot) return fail(MQ_ERR_INVALID_ARG, "n_max must be >= n_pilot on every level");
    if (!xi[l] || !q_fine[l] || (l > 0 && !q_coarse[l]))
      return fail(MQ_ERR_INVALID_ARG, "null per-level pointer");
    if (lv[l].steps_per_period < 1 || lv[l].n_periods < 1 || lv[l].coarse_steps_per_period < 0 ||
        (l > 0 && lv[l].coarse_steps_per_period < 1))
      return fail(MQ_ERR_INVALID_ARG, "levels above 0 need a coupled coarse run");
  }
  const double t0 = now_ms();
  const double theta = ad->var_fraction > 0 ? ad->var_fraction : 0.5;
  const double budget = theta * ad->target_rmse * ad->target_rmse;
  const int max_rounds = ad->max_rounds > 0 ? ad->max_rounds : 10;
  const int L = n_levels;
  std::vector<int32_t> have(L, 0), need(L);
  std::vector<double> cost(L);
  for (int l = 0; l < L; ++l) {
    need[l] = ad->n_pilot;
    cost[l] = (double)lv[l].n_periods * (lv[l].steps_per_period + lv[l].coarse_steps_per_period);
  }
  if (st) std::memset(st, 0, sizeof(*st));
  TmpPtr<double> dout;
  HIP_TRY(tmp_alloc(dout, 1 + 2 * (size_t)L, p->stream));
  std::vector<double> host(1 + 2 * (size_t)L);
  int status = MQ_OK;
  for (int round = 1;; ++round) {
    // the new samples of every level that asks for more, in one launch
    std::vector<mq_level_desc> lvs;
    std::vector<int32_t> ns;
    std::vector<const double*> xs;
    std::vector<double*> qf, qc;
    for (int l = 0; l < L; ++l) {
      if (need[l] <= have[l]) continue;
      lvs.push_back(lv[l]);
      ns.push_back(need[l] - have[l]);
      xs.push_back(xi[l] + (size_t)have[l] * p->n_xi);
      qf.push_back(q_fine[l] + have[l]);
      qc.push_back(lv[l].coarse_steps_per_period > 0 ? q_coarse[l] + have[l] : nullptr);
    }
    if (!lvs.empty()) {
      mq_run_stats s{};
      const int rc = multilevel_run_dev(p, (int32_t)lvs.size(), lvs.data(), ns.data(), xs.data(), qf.data(),
                                         qc.data(), &s);
      if (rc < 0) return rc;
      if (rc > 0) status = rc;
      if (st) {
        st->n_instances += s.n_instances;
        st->sample_steps += s.sample_steps;
        st->inner_iters += s.inner_iters;
        st->sweeps += s.sweeps;
        st->picard_iters += s.picard_iters;
        st->max_inner_per_step = std::max(st->max_inner_per_step, s.max_inner_per_step);
        st->n_not_converged += s.n_not_converged;
        st->n_failed += s.n_failed;
      st->n_pieces += s.n_pieces;
        st->path = s.path;
        st->grid = s.grid;
        st->block = s.block;
        st->kernel_ms += s.kernel_ms;
        st->busy_ms += s.busy_ms;
        for (int q = 0; q < 8; ++q) st->phase_ms[q] += s.phase_ms[q];
      }
      for (int l = 0; l < L; ++l) have[l] = std::max(have[l], need[l]);
    }
    // level means and variances of all samples so far (device, fixed order)
    const int rc = mlmc_estimate(L, have.data(), q_fine, q_coarse, dout.get(), p->stream);
    if (rc) return rc;
    HIP_TRY(copy_sync(host.data(), dout.get(), host.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    // Eq. (11) at the current variance estimates
    double s = 0.0;
    for (int l = 0; l < L; ++l) s += std::sqrt(host[1 + L + l] * cost[l]);
    bool more = false, capped = false;
    for (int l = 0; l < L; ++l) {
      const double v = host[1 + L + l];
      const double opt = v > 0 ? std::ceil(std::sqrt(v / cost[l]) * s / budget) : 0.0;
      int32_t target = have[l];
      if (opt > (double)have[l]) {
        if (opt > (double)n_max[l]) capped = true;
        target = (int32_t)std::min<double>(opt, (double)n_max[l]);
      }
      need[l] = target;
      more |= need[l] > have[l];
    }
    if (!more || round >= max_rounds) {
      if (more || capped) {
        status = std::max(status, (int)MQ_WARN_NOT_CONVERGED);
        last_error() = "adaptive MLMC stopped at n_max or max_rounds before Eq. (11) was met";
      }
      break;
    }
  }
  for (int l = 0; l < L; ++l) n_used[l] = have[l];
  std::memcpy(out, host.data(), host.size() * sizeof(double));
  if (st) st->total_ms = now_ms() - t0;
  return status;
}

int mlmc_multimesh_run(int32_t n_levels, mq_problem* const* problems, const mq_level_desc* lv,
                       const int32_t* n_samples, const double* const* xi, double* const* q_fine,
                       double* const* q_coarse, mq_run_stats* st) {
  const FlagsClearedOnReturn no_flags;
  if (!problems || !lv || !n_samples || !xi || !q_fine || !q_coarse) return fail(MQ_ERR_INVALID_ARG, "null argument");
  if (n_levels < 1 || n_levels > 16) return fail(MQ_ERR_INVALID_ARG, "n_levels must be in [1, 16]");
  for (int m = 0; m < n_levels; ++m)
    if (int rh = refuse_host(problems[m])) return rh;
  const int L = n_levels;
  for (int l = 0; l < L; ++l) {
    mq_problem* p = problems[l];
    if (!p) return fail(MQ_ERR_INVALID_ARG, "null problem");
    for (int k = 0; k < l; ++k)
      if (problems[k] == p) return fail(MQ_ERR_INVALID_ARG, "every level needs its own problem handle");
    if (p->n_xi != problems[0]->n_xi || p->d.material != problems[0]->d.material ||
        p->d.precision != problems[0]->d.precision)
      return fail(MQ_ERR_INVALID_ARG, "the meshes must share material, input dimension and precision");
    if (l > 0 && (lv[l].coarse_steps_per_period < 1 || !q_coarse[l]))
      return fail(MQ_ERR_INVALID_ARG, "levels above 0 need a coupled coarse run");
  }
  const double t0 = now_ms();
  if (st) std::memset(st, 0, sizeof(*st));
  // per mesh m: the fine runs of level m and the coupled coarse runs of level m + 1
  std::vector<std::vector<LevelBufs>> bufs(L);
  std::vector<std::vector<Inst>> runs(L);
  for (int m = 0; m < L; ++m) {
    mq_problem* p = problems[m];
    bufs[m].resize(2);
    std::vector<Inst> a, unused;
    const mq_level_desc f{lv[m].steps_per_period, 0, lv[m].n_periods, 0};
    int rc = prepare_level(p, &f, n_samples[m], xi[m], q_fine[m], nullptr, false, bufs[m][0], a, unused, 0);
    if (rc) return rc;
    if (m + 1 < L) {
      const mq_level_desc c{lv[m + 1].coarse_steps_per_period, 0, lv[m + 1].n_periods, 0};
      std::vector<Inst> b;
      rc = prepare_level(p, &c, n_samples[m + 1], xi[m + 1], q_coarse[m + 1], nullptr, false, bufs[m][1], b,
                         unused, n_samples[m]);
      if (rc) return rc;
      a.insert(a.end(), b.begin(), b.end());
    }
    std::stable_sort(a.begin(), a.end(), [](const Inst& x, const Inst& y) { return x.n_steps > y.n_steps; });
    runs[m] = std::move(a);
    // size the work buffer now: no allocation while other meshes run
    rc = ensure_work(p, std::min<size_t>(runs[m].size(), max_slots(p)));
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  // one persistent launch per mesh, all meshes at once (a host thread each)
  std::vector<int> rcs(L, MQ_OK);
  std::vector<std::string> errs(L);
  std::vector<mq_run_stats> sts(L);
  std::vector<RunOut> ros(L);
  std::vector<std::thread> th;
  for (int m = 0; m < L; ++m) {
    th.emplace_back([&, m] {
      (void)hipSetDevice(problems[m]->device);
      rcs[m] = run_instances(problems[m], runs[m], &sts[m], &ros[m], nullptr);
      if (rcs[m] < 0) errs[m] = last_error();
    });
  }
  for (auto& t : th) t.join();
  int status = MQ_OK;
  for (int m = 0; m < L; ++m) {
    if (rcs[m] < 0) return fail(rcs[m], errs[m]);
    status = std::max(status, ros[m].status);
    if (st) {
      const mq_run_stats& s = sts[m];
      st->n_instances += s.n_instances;
      st->sample_steps += s.sample_steps;
      st->inner_iters += s.inner_iters;
      st->sweeps += s.sweeps;
      st->picard_iters += s.picard_iters;
      st->max_inner_per_step = std::max(st->max_inner_per_step, s.max_inner_per_step);
      st->n_not_converged += s.n_not_converged;
      st->n_failed += s.n_failed;
      st->n_pieces += s.n_pieces;
      st->kernel_ms = std::max(st->kernel_ms, s.kernel_ms);  // concurrent launches
      st->busy_ms += s.busy_ms;
      st->lat_p50_ms = std::max(st->lat_p50_ms, s.lat_p50_ms);
      st->lat_p99_ms = std::max(st->lat_p99_ms, s.lat_p99_ms);
      st->lat_max_ms = std::max(st->lat_max_ms, s.lat_max_ms);
      for (int q = 0; q < 8; ++q) st->phase_ms[q] += s.phase_ms[q];
    }
  }
  if (st) {
    st->path = problems[L - 1]->path;
    st->grid = ros[L - 1].grid;
    st->block = ros[L - 1].block;
    st->total_ms = now_ms() - t0;
  }
  return status;
}

// Parareal (Section II-C, Eq. (12)) for n_samples samples in ONE persistent
// launch.  The launch's work queue holds, per sample, the initial coarse chain,
// then per iteration j = 1..kcap the fine slices n = j..M and the coarse chain
// of iteration j, which first takes the stopping decision from the interface
// jumps of Section II-C and then corrects U_n = F_n + (C_new - C_old), n =
// j+1..M-1.  Entries wait on flags in device memory:
//   fine (j, n)   waits for U_{n-1}^(j-1): the chain of iteration j-1 (segment
//                 n-1, or its first step U_{j-1} = F_{j-1} for n = j; the
//                 initial chain for j = 1; U_0 needs no wait);
//   chain (j)     waits for the chain of iteration j-1, then for the fine slices
//                 n = j..M of iteration j, one by one, while it sums the jumps.
// Every wait is for an entry queued before the waiting one, so every wait ends;
// and the sweep of iteration j+1 overlaps the correction chain of iteration j
// (fine (j+1, n) starts once the chain has passed slice n-1).  A sample that
// stops at iteration K skips its later entries; the executed work is exactly
// the sequential algorithm's (Eqs. (13)-(14)).  Fine end states alternate
// between two buffers by the parity of j, because fine (j+1, n) can finish
// before chain (j) has read F_n^(j).
// Queue entries and buffers of a one-launch Parareal run (para_build), and
// its results after the launch (para_finish).
struct ParaRun {
  CallMem mem;
  int S = 0, M = 0, kcap = 0, fs = 0, cs = 0;
  double T = 0;
  double* Fb = nullptr;
  double* qb = nullptr;
  int* Kd = nullptr;
  int* pfl = nullptr;
  std::vector<Inst> insts;
};

static int para_validate(const mq_problem* p, const mq_parareal_desc* pd) {
  const int M = pd->n_slices, fs = pd->fine_steps_per_slice, cs = pd->coarse_steps_per_slice;
  if (M < 1 || fs < 1 || cs < 1 || pd->n_periods < 1 || pd->k_max < 1 || pd->fixed_k < 0 || !(pd->tol >= 0))
    return fail(MQ_ERR_INVALID_ARG, "invalid Parareal description");
  if ((int64_t)M * fs > (1 << 24) || (int64_t)M * cs > (1 << 24)) return fail(MQ_ERR_INVALID_ARG, "too many steps");
  if (p->path == MQ_PATH_WIDE) return fail(MQ_ERR_INVALID_ARG, "Parareal runs on the resident or streaming path");
  return MQ_OK;
}

// Entries of Parareal (Section II-C, Eq. (12)) for S samples whose tables are
// assembled in `tables` ([S][tab_stride]); appended to pr.insts (group and
// sample = the sample index).  The launch's work queue holds, per sample,
// the initial coarse chain, then per iteration j = 1..kcap the fine slices n =
// j..M and the coarse chain of iteration j, which first takes the stopping
// decision from the interface jumps of Section II-C and then corrects U_n =
// F_n + (C_new - C_old), n = j+1..M-1.  Entries wait on flags in device memory:
//   fine (j, n)   waits for U_{n-1}^(j-1): the chain of iteration j-1 (segment
//                 n-1, or its first step U_{j-1} = F_{j-1} for n = j; the
//                 initial chain for j = 1; U_0 needs no wait);
//   chain (j)     waits for the chain of iteration j-1, then for the fine slices
//                 n = j..M of iteration j, one by one, while it sums the jumps.
// Every wait is for an entry queued before the waiting one, so every wait ends
// (checked here before the launch); and the sweep of iteration j+1 overlaps
// the correction chain of iteration j (fine (j+1, n) starts once the chain has
// passed slice n-1).  A sample that stops at iteration K skips its later
// entries; the executed work is exactly the sequential algorithm's (Eqs.
// (13)-(14)).  Fine end states alternate between two buffers by the parity of
// j, because fine (j+1, n) can finish before chain (j) has read F_n^(j).
static int para_build(mq_problem* p, const mq_parareal_desc* pd, int S, const double* tables, ParaRun& pr) {
  const Geom& g = p->hm.g;
  const size_t FS = (size_t)g.N * g.P;
  const int M = pd->n_slices, fs = pd->fine_steps_per_slice, cs = pd->coarse_steps_per_slice;
  CallMem& mem = pr.mem;
  mem.use_stream(p->stream);
  const double T = pd->n_periods / p->d.freq;
  const double dtf = T / ((double)M * fs), dtc = T / ((double)M * cs);
  auto sf = source_table(p->d, dtf, M * fs);
  auto sc = source_table(p->d, dtc, M * cs);
  const int kcap = std::min(pd->fixed_k > 0 ? pd->fixed_k : pd->k_max, M);
  double *dsf, *dsc, *Ub, *Fb, *Cb, *qb, *Jb;
  int *segd, *fdone, *chd, *Kd, *pfl, *abortf;
  ParaCtl* dctl;
  HIP_TRY(mem.get(dsf, sf.size()));
  HIP_TRY(mem.get(dsc, sc.size()));
  HIP_TRY(copy_sync(dsf, sf.data(), sf.size() * sizeof(double), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(copy_sync(dsc, sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice, p->stream));
  const size_t nU = (size_t)S * M * FS, nF = 2 * (size_t)S * M * FS, nC = (size_t)S * M * FS;
  const size_t nq = (size_t)S * kcap * M;
  const size_t nseg = (size_t)(kcap + 1) * S * M, nfd = (size_t)(kcap + 1) * S * (M + 1), nch = (size_t)(kcap + 1) * S;
  HIP_TRY(mem.get(Ub, nU));
  HIP_TRY(mem.get(Fb, nF));
  HIP_TRY(mem.get(Cb, nC));
  HIP_TRY(mem.get(qb, nq));
  HIP_TRY(mem.get(Jb, (size_t)S * kcap));
  HIP_TRY(mem.get(segd, nseg));
  HIP_TRY(mem.get(fdone, nfd));
  HIP_TRY(mem.get(chd, nch));
  HIP_TRY(mem.get(Kd, S));
  HIP_TRY(mem.get(pfl, S));
  HIP_TRY(mem.get(abortf, 1));
  HIP_TRY(mem.get(dctl, 1));
  HIP_TRY(launch_fill_zero(Ub, nU, p->stream));
  HIP_TRY(launch_fill_zero(Fb, nF, p->stream));
  HIP_TRY(launch_fill_zero(Cb, nC, p->stream));
  HIP_TRY(launch_fill_zero(qb, nq, p->stream));
  HIP_TRY(launch_fill_zero(Jb, (size_t)S * kcap, p->stream));
  HIP_TRY(launch_fill_zero_i(segd, nseg, p->stream));
  HIP_TRY(launch_fill_zero_i(fdone, nfd, p->stream));
  HIP_TRY(launch_fill_zero_i(chd, nch, p->stream));
  HIP_TRY(launch_fill_zero_i(Kd, S, p->stream));
  HIP_TRY(launch_fill_zero_i(pfl, S, p->stream));
  HIP_TRY(launch_fill_zero_i(abortf, 1, p->stream));
  auto U = [&](int s_, int n_) { return Ub + ((size_t)s_ * M + n_) * FS; };                       // n = 0..M-1
  auto F = [&](int j_, int s_, int n_) { return Fb + (((size_t)(j_ & 1) * S + s_) * M + (n_ - 1)) * FS; };  // n = 1..M
  auto C = [&](int s_, int n_) { return Cb + ((size_t)s_ * M + n_) * FS; };                       // n = 1..M-1
  auto QS = [&](int s_, int j_, int n_) { return qb + ((size_t)s_ * kcap + (j_ - 1)) * M + (n_ - 1); };
  auto SEG = [&](int j_, int s_, int n_) { return segd + ((size_t)j_ * S + s_) * M + n_; };        // U_n^(j) written
  auto FD = [&](int j_, int s_, int n_) { return fdone + ((size_t)j_ * S + s_) * (M + 1) + n_; };   // fine (j, n) done
  auto CH = [&](int j_, int s_) { return chd + (size_t)j_ * S + s_; };                              // chain (j) done
  if (p->a0)  // U_0 = a_0 for every sample
    for (int s_ = 0; s_ < S; ++s_)
      HIP_TRY(hipMemcpyAsync(U(s_, 0), p->a0.get(), FS * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
  ParaCtl hctl{Kd, Jb, pfl, abortf, pd->tol, pd->fixed_k, kcap};
  HIP_TRY(copy_sync(dctl, &hctl, sizeof(ParaCtl), hipMemcpyHostToDevice, p->stream));

  // pointer arrays of the entries (one device array, offsets into it)
  std::vector<const void*> ptrs;
  std::vector<Inst> insts;
  std::vector<std::pair<size_t, const void*>> fix;  // (entry, field) resolved after the copy
  auto put = [&](const std::vector<const void*>& v) {
    const size_t o = ptrs.size();
    ptrs.insert(ptrs.end(), v.begin(), v.end());
    return o;
  };
  struct Arr {
    size_t cu = SIZE_MAX, cf = SIZE_MAX, cc = SIZE_MAX, sd = SIZE_MAX, jf = SIZE_MAX, ju = SIZE_MAX, jw = SIZE_MAX;
  };
  std::vector<Arr> arrs;
  auto base = [&](int s_) {
    Inst in{};
    in.tab = tables + (size_t)s_ * tab_stride(g);
    in.sample = s_;
    in.group = s_;
    in.para = dctl;
    return in;
  };
  // initial coarse chain U_n^(0) = C(U_{n-1}^(0)), n = 1..M-1
  if (M >= 2)
    for (int s_ = 0; s_ < S; ++s_) {
      Inst in = base(s_);
      in.src = dsc;
      in.a_init = U(s_, 0);
      in.dt = dtc;
      in.n_steps = cs;
      in.k0 = 0;
      in.n_chain = M - 1;
      in.para_iter = 0;
      in.para_chain = 1;
      in.dep_done = CH(0, s_);
      Arr a;
      std::vector<const void*> cu, cf, cc, sd;
      for (int n_ = 1; n_ <= M - 1; ++n_) {
        cu.push_back(U(s_, n_));
        cf.push_back(nullptr);
        cc.push_back(C(s_, n_));
        sd.push_back(SEG(0, s_, n_));
      }
      a.cu = put(cu);
      a.cf = put(cf);
      a.cc = put(cc);
      a.sd = put(sd);
      insts.push_back(in);
      arrs.push_back(a);
    }
  for (int j_ = 1; j_ <= kcap; ++j_) {
    // fine sweep of iteration j over slices n = j..M (slice-major: the earliest
    // inputs first)
    for (int n_ = j_; n_ <= M; ++n_)
      for (int s_ = 0; s_ < S; ++s_) {
        Inst in = base(s_);
        in.src = dsf;
        in.a_init = U(s_, n_ - 1);
        in.a_out = F(j_, s_, n_);
        in.q_out = QS(s_, j_, n_);
        in.q_scale = 1.0;
        in.dt = dtf;
        in.n_steps = fs;
        in.k0 = (n_ - 1) * fs;
        in.para_iter = j_;
        in.para_chain = 0;
        in.dep_wait = (n_ == 1) ? nullptr : SEG(j_ - 1, s_, n_ - 1);
        in.dep_done = FD(j_, s_, n_);
        insts.push_back(in);
        arrs.push_back(Arr{});
      }
    // coarse chain of iteration j: stopping decision, then the correction
    for (int s_ = 0; s_ < S; ++s_) {
      Inst in = base(s_);
      in.src = dsc;
      in.dt = dtc;
      in.n_steps = cs;
      in.k0 = j_ * cs;
      in.para_iter = j_;
      in.para_chain = 1;
      in.dep_wait = (j_ == 1 && M < 2) ? nullptr : CH(j_ - 1, s_);  // no initial chain when M = 1
      in.dep_done = CH(j_, s_);
      in.n_jump = M - j_;
      const bool last = j_ >= kcap;
      in.n_chain = last ? 0 : std::max(0, M - 1 - j_);
      if (!last && j_ <= M - 1) {
        in.a_init = U(s_, j_);
        in.u_first = U(s_, j_);
        in.f_first = F(j_, s_, j_);
        in.first_done = SEG(j_, s_, j_);
      }
      Arr a;
      std::vector<const void*> jf, ju, jw;
      for (int n_ = j_; n_ <= M - 1; ++n_) {
        jf.push_back(F(j_, s_, n_));
        ju.push_back(U(s_, n_));
      }
      for (int n_ = j_; n_ <= M; ++n_) jw.push_back(FD(j_, s_, n_));
      a.jf = put(jf);
      a.ju = put(ju);
      a.jw = put(jw);
      if (in.n_chain > 0) {
        std::vector<const void*> cu, cf, cc, sd;
        for (int n_ = j_ + 1; n_ <= M - 1; ++n_) {
          cu.push_back(U(s_, n_));
          cf.push_back(F(j_, s_, n_));
          cc.push_back(C(s_, n_));
          sd.push_back(SEG(j_, s_, n_));
        }
        a.cu = put(cu);
        a.cf = put(cf);
        a.cc = put(cc);
        a.sd = put(sd);
      }
      insts.push_back(in);
      arrs.push_back(a);
    }
  }
  // Every flag an entry waits on must be set by an entry queued before it.
  {
    std::unordered_map<const void*, size_t> setter;
    for (size_t e = 0; e < insts.size(); ++e) {
      const Inst& in = insts[e];
      if (in.dep_done) setter[in.dep_done] = e;
      if (in.first_done) setter[in.first_done] = e;
      if (arrs[e].sd != SIZE_MAX)
        for (int k = 0; k < in.n_chain; ++k) setter[ptrs[arrs[e].sd + k]] = e;
    }
    auto before = [&](const void* f, size_t e) {
      auto it = setter.find(f);
      return it != setter.end() && it->second < e;
    };
    for (size_t e = 0; e < insts.size(); ++e) {
      const Inst& in = insts[e];
      bool ok = !in.dep_wait || before(in.dep_wait, e);
      if (arrs[e].jw != SIZE_MAX)
        for (int k = 0; k <= in.n_jump; ++k) ok = ok && before(ptrs[arrs[e].jw + k], e);
      if (!ok) return fail(MQ_ERR_DEVICE, "internal: Parareal entry waits on a later entry");
    }
  }
  const void** dptrs = nullptr;
  HIP_TRY(mem.get(dptrs, ptrs.size()));
  HIP_TRY(copy_sync(dptrs, ptrs.data(), ptrs.size() * sizeof(void*), hipMemcpyHostToDevice, p->stream));
  for (size_t e = 0; e < insts.size(); ++e) {
    Inst& in = insts[e];
    const Arr& a = arrs[e];
    if (a.cu != SIZE_MAX) {
      in.chain_u = (double* const*)(dptrs + a.cu);
      in.chain_f = (const double* const*)(dptrs + a.cf);
      in.chain_c = (double* const*)(dptrs + a.cc);
      in.seg_done = (int* const*)(dptrs + a.sd);
    }
    if (a.jf != SIZE_MAX) {
      in.jump_f = (const double* const*)(dptrs + a.jf);
      in.jump_u = (const double* const*)(dptrs + a.ju);
      in.jump_wait = (const int* const*)(dptrs + a.jw);
    }
  }
  pr.S = S;
  pr.M = M;
  pr.kcap = kcap;
  pr.fs = fs;
  pr.cs = cs;
  pr.T = T;
  pr.Fb = Fb;
  pr.qb = qb;
  pr.Kd = Kd;
  pr.pfl = pfl;
  pr.insts = std::move(insts);
  return MQ_OK;
}

// After the launch: per-sample K, flags (entry_flags: FLAG_* per entry of
// pr.insts, in order), Q (device), K (device iters), final states (nullable),
// executed sample-steps.  Returns MQ_WARN_NOT_CONVERGED when a sample
// reached k_max above tol or an entry hit a solver cap.
static int para_finish(mq_problem* p, ParaRun& pr, const int* entry_flags, double* q, int32_t* iters,
                       double* final_state, std::vector<int32_t>& pflags, std::vector<int>& Kh, int64_t* steps_out) {
  const Geom& g = p->hm.g;
  const size_t FS = (size_t)g.N * g.P;
  const int S = pr.S, M = pr.M, kcap = pr.kcap, fs = pr.fs, cs = pr.cs;
  const double T = pr.T;
  double* const Fb = pr.Fb;
  auto F = [&](int j_, int s_, int n_) { return Fb + (((size_t)(j_ & 1) * S + s_) * M + (n_ - 1)) * FS; };
  Kh.assign(S, 0);
  std::vector<int> ph(S);
  HIP_TRY(hipMemcpyAsync(Kh.data(), pr.Kd, S * sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(ph.data(), pr.pfl, S * sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  bool warn = false;
  pflags.assign(S, 0);
  for (size_t e = 0; e < pr.insts.size(); ++e) pflags[pr.insts[e].sample] |= entry_flags[e];
  for (int s_ = 0; s_ < S; ++s_) {
    pflags[s_] |= ph[s_];
    if (Kh[s_] < 1 || Kh[s_] > kcap) {  // no decision reached (a timed-out wait)
      pflags[s_] |= FLAG_FAILED;
      Kh[s_] = std::max(1, std::min(kcap, Kh[s_]));
    }
    if (pflags[s_] & (FLAG_PARAREAL_KMAX | FLAG_WARN)) warn = true;
  }
  HIP_TRY(copy_sync(iters, Kh.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
  // Q = sum_n q_n / T with q_n of each slice's latest fine run, iteration min(n, K) (FP64, device)
  HIP_TRY(launch_para_qoi(pr.qb, iters, kcap, M, S, T, q, p->stream));
  if (final_state) {
    std::vector<const double*> fp(S);
    for (int s_ = 0; s_ < S; ++s_) fp[s_] = F(Kh[s_], s_, M);
    const double** dfp = nullptr;
    HIP_TRY(pr.mem.get(dfp, S));
    HIP_TRY(copy_sync(dfp, fp.data(), S * sizeof(double*), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(launch_to_interior(g, S, dfp, final_state, p->stream));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  // executed work of the sequential algorithm with these K (entries that
  // skipped ran nothing): initial chain (M-1) C, per iteration j <= K the fine
  // slices j..M, per correction j < K the slices j+1..M-1
  int64_t steps = 0;
  for (int s_ = 0; s_ < S; ++s_) {
    steps += (int64_t)(M - 1) * cs;
    for (int j_ = 1; j_ <= Kh[s_]; ++j_) steps += (int64_t)(M - j_ + 1) * fs;
    for (int j_ = 1; j_ < Kh[s_]; ++j_) steps += (int64_t)std::max(0, M - 1 - j_) * cs;
  }
  if (steps_out) *steps_out = steps;
  return warn ? MQ_WARN_NOT_CONVERGED : MQ_OK;
}

// Parareal for n_samples samples in one persistent launch (para_build).
static int parareal_run_dev(mq_problem* p, const mq_parareal_desc* pd, int32_t n_samples, const double* xi,
                            double* q, int32_t* iters, double* final_state, mq_run_stats* st) {
  last_flags().clear();
  if (!p || !pd) return fail(MQ_ERR_INVALID_ARG, "null argument");
  if (!xi || !q || !iters) return fail(MQ_ERR_INVALID_ARG, "xi, q and iters are required");
  if (n_samples < 1) return fail(MQ_ERR_INVALID_ARG, "n_samples must be >= 1");
  int rc = para_validate(p, pd);
  if (rc) return rc;
  if (p->d.material == MQ_MAT_NONLINEAR) return fail(MQ_ERR_INVALID_ARG, "Parareal takes linear materials");
  const double t_start = now_ms();
  if (st) std::memset(st, 0, sizeof(*st));
  rc = check_finite(p, xi, (size_t)n_samples * p->n_xi);
  if (rc) return rc;
  TmpPtr<double> tables;
  rc = assemble(p, xi, n_samples, tables);
  if (rc) return rc;
  ParaRun pr;
  rc = para_build(p, pd, n_samples, tables.get(), pr);
  if (rc) return rc;
  RunOut ro;
  rc = run_instances(p, pr.insts, st, &ro, nullptr);
  if (rc) return rc;
  std::vector<int32_t> pflags;
  std::vector<int> Kh;
  int64_t steps = 0;
  const int rf = para_finish(p, pr, ro.flags.data(), q, iters, final_state, pflags, Kh, &steps);
  if (rf < 0) return rf;
  if (st) {
    st->sample_steps = steps;
    st->n_instances = (int64_t)pr.insts.size();
    st->total_ms = now_ms() - t_start;
  }
  last_flags() = pflags;
  if (rf == MQ_WARN_NOT_CONVERGED) {
    last_error() = "Parareal reached k_max above the tolerance (or a solver cap) for some samples";
    return MQ_WARN_NOT_CONVERGED;
  }
  return ro.status;
}

int mlmc_combined_run(mq_problem* p, int32_t n_levels, const mq_level_desc* lv, const int32_t* n_samples,
                      const double* const* xi, const mq_combined_desc* cd, double* const* q_fine,
                      double* const* q_coarse, int32_t* para_iters, mq_run_stats* st, mq_combined_stats* cs) {
  const FlagsClearedOnReturn no_flags;
  if (int rh = refuse_host(p)) return rh;
  if (!p || !lv || !n_samples || !xi || !cd || !q_fine || !q_coarse || !para_iters)
    return fail(MQ_ERR_INVALID_ARG, "null argument");
  if (n_levels < 2 || n_levels > 16) return fail(MQ_ERR_INVALID_ARG, "n_levels must be in [2, 16]");
  if (p->path == MQ_PATH_WIDE) return fail(MQ_ERR_INVALID_ARG, "the combined run uses the resident or streaming path");
  if (p->d.material == MQ_MAT_NONLINEAR) return fail(MQ_ERR_INVALID_ARG, "the combined run takes linear materials");
  const int L = n_levels - 1;
  for (int l = 0; l <= L; ++l) {
    if (n_samples[l] < 1 || !xi[l] || !q_fine[l] || (l > 0 && !q_coarse[l]))
      return fail(MQ_ERR_INVALID_ARG, "every level needs samples, xi and outputs");
    if (lv[l].steps_per_period < 1 || lv[l].n_periods < 1 || (l > 0 && lv[l].coarse_steps_per_period < 1))
      return fail(MQ_ERR_INVALID_ARG, "invalid level description");
  }
  const int nper = lv[L].n_periods;
  int cspp = cd->coarse_steps_per_period;
  if (cspp == 0) {
    if (L < 2) return fail(MQ_ERR_INVALID_ARG, "coarse_steps_per_period is required with fewer than 3 levels");
    cspp = lv[L - 2].steps_per_period;
  }
  if (cspp < 1 || cd->n_slices < 0 || cd->k_max < 0 || !(cd->tol >= 0))
    return fail(MQ_ERR_INVALID_ARG, "invalid combined-run description");
  // Eq. (25) with the device's persistent slots as cores
  const int n_c = (int)max_slots(p);
  const double CL = (double)lv[L].steps_per_period * nper;
  const double CL1 = (double)lv[L - 1].steps_per_period * lv[L - 1].n_periods;
  const int n_c_para = (int)std::floor(n_c / (n_samples[L] * (1.0 + CL1 / CL)));
  const int64_t fine_total = (int64_t)lv[L].steps_per_period * nper, coarse_total = (int64_t)cspp * nper;
  int M = cd->n_slices;
  if (M == 0)
    for (int m = 2; m <= std::max(2, n_c_para); m *= 2)
      if (fine_total % m == 0 && coarse_total % m == 0) M = m;
  if (M < 2 || fine_total % M || coarse_total % M)
    return fail(MQ_ERR_INVALID_ARG, "the slices (>= 2) must divide the fine and coarse step counts of level L");
  const int kmax = cd->k_max > 0 ? cd->k_max : M;
  const double t0 = now_ms();
  if (st) std::memset(st, 0, sizeof(*st));
  // batched part: levels 0..L-1 and the coupled coarse runs of level L
  std::vector<LevelBufs> lbs(n_levels);
  std::vector<std::pair<int64_t, Inst>> keyed;
  int group0 = 0;
  for (int l = 0; l <= L; ++l) {
    std::vector<Inst> f, c;
    int rc;
    if (l < L) {
      rc = prepare_level(p, &lv[l], n_samples[l], xi[l], q_fine[l], q_coarse[l], false, lbs[l], f, c, group0);
    } else {
      const mq_level_desc lc{lv[L].coarse_steps_per_period, 0, nper, 0};
      rc = prepare_level(p, &lc, n_samples[L], xi[L], q_coarse[L], nullptr, false, lbs[L], f, c, group0);
    }
    if (rc) return rc;
    group0 += n_samples[l];
    for (auto& i : f) keyed.push_back({i.n_steps, i});
    for (auto& i : c) keyed.push_back({i.n_steps, i});
  }
  std::stable_sort(keyed.begin(), keyed.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  // level L's fine values by Parareal (Section II-D), on the tables of its samples
  const mq_parareal_desc pd{nper, M, (int32_t)(fine_total / M), (int32_t)(coarse_total / M), kmax, 0, cd->tol};
  int rc = para_validate(p, &pd);
  if (rc) return rc;
  ParaRun pr;
  rc = para_build(p, &pd, n_samples[L], lbs[L].tables, pr);
  if (rc) return rc;
  // ONE persistent launch: the Parareal entries form the first work queue, the
  // level instances (longest first) the second.  Eq. (25) on the device: N_L * M
  // workgroups (at most half) start on the Parareal queue, the others on the
  // levels; a workgroup whose queue is empty moves to the other one.
  const int n_para = (int)pr.insts.size();
  std::vector<Inst> all = pr.insts;
  for (auto& k : keyed) all.push_back(k.second);
  const int level_slots = n_c - std::min(n_samples[L] * M, n_c / 2);
  RunOut ro;
  ro.queue0 = n_para;
  ro.grid0 = n_c - level_slots;
  rc = run_instances(p, all, st, &ro, nullptr);
  if (rc) return rc;
  std::vector<int32_t> pflags;
  std::vector<int> Kh;
  int64_t para_steps = 0;
  const int rcb = para_finish(p, pr, ro.flags.data(), q_fine[L], para_iters, nullptr, pflags, Kh, &para_steps);
  if (rcb < 0) return rcb;
  const std::vector<int>& K = Kh;
  // executed work: fine slices j..M in iteration j; coarse chains over M - j slices
  // before iteration j + 1 while the sample is still iterating (the first one is the
  // initial prediction)
  int64_t fsteps = 0, csteps = 0;
  int kmx = 0;
  double ksum = 0;
  for (int32_t k : K) {
    for (int j = 1; j <= k; ++j) {
      fsteps += (int64_t)(M - j + 1) * (fine_total / M);
      csteps += (int64_t)(M - j) * (coarse_total / M);
    }
    kmx = std::max(kmx, (int)k);
    ksum += k;
  }
  if (st) {
    // executed work: the level instances ran whole; the Parareal entries ran
    // the sequential algorithm's work for these K
    int64_t level_steps = 0;
    for (auto& k : keyed) level_steps += k.second.n_steps;
    st->sample_steps = level_steps + para_steps;
    st->total_ms = now_ms() - t0;
  }
  if (cs) {
    std::memset(cs, 0, sizeof(*cs));
    cs->n_slices = M;
    cs->coarse_steps_per_period = cspp;
    cs->n_cores = n_c;
    cs->n_c_para = n_c_para;
    cs->ms_levels = ro.done_ms[1];    // device time to the last level instance's end
    cs->ms_parareal = ro.done_ms[0];  // ... and to the last Parareal entry's end
    cs->ms_total = now_ms() - t0;
    cs->para_fine_steps = fsteps;
    cs->para_coarse_steps = csteps;
    cs->mean_k = ksum / K.size();
    cs->max_k = kmx;
    cs->level_slots = level_slots;
  }
  if (rcb == MQ_WARN_NOT_CONVERGED) last_error() = "Parareal reached k_max above the tolerance for some samples";
  return std::max(ro.status, rcb);
}

int mlmc_estimate(int32_t n_levels, const int32_t* n_per_level, const double* const* q_fine,
                  const double* const* q_coarse, double* out, void* stream) {
  if (n_levels < 1 || n_levels > 64 || !n_per_level || !q_fine || !out)
    return fail(MQ_ERR_INVALID_ARG, "invalid arguments");
  for (int l = 0; l < n_levels; ++l) {
    if (n_per_level[l] < 1) return fail(MQ_ERR_INVALID_ARG, "every level needs >= 1 sample");
    if (!q_fine[l]) return fail(MQ_ERR_INVALID_ARG, "null q_fine entry");
    if (l > 0 && (!q_coarse || !q_coarse[l])) return fail(MQ_ERR_INVALID_ARG, "null q_coarse entry for a level > 0");
  }
  hipStream_t st = (hipStream_t)stream;
  std::vector<const double*> qc(n_levels, nullptr);
  for (int l = 1; l < n_levels; ++l) qc[l] = q_coarse[l];
  TmpPtr<int> dn;
  TmpPtr<const double*> dqf, dqc;
  HIP_TRY(tmp_alloc(dn, n_levels, st));
  HIP_TRY(tmp_alloc(dqf, n_levels, st));
  HIP_TRY(tmp_alloc(dqc, n_levels, st));
  HIP_TRY(hipMemcpyAsync(dn.get(), n_per_level, n_levels * sizeof(int), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(dqf.get(), q_fine, n_levels * sizeof(double*), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(dqc.get(), qc.data(), n_levels * sizeof(double*), hipMemcpyHostToDevice, st));
  HIP_TRY(launch_level_stats(n_levels, dn.get(), dqf.get(), dqc.get(), out, st));
  HIP_TRY(hipStreamSynchronize(st));
  return MQ_OK;
}

int mq_plan_split(int32_t n, const int32_t* steps, int32_t slots, int32_t split_steps, int32_t cap,
                  int32_t* orig, int32_t* first, int32_t* len, int32_t* dep, double* makespan, int32_t* m_out) {
  if (n < 0 || (n > 0 && !steps) || slots < 1 || split_steps < -1 || cap < 0 || !m_out)
    return fail(MQ_ERR_INVALID_ARG, "invalid arguments");
  if (cap > 0 && (!orig || !first || !len || !dep)) return fail(MQ_ERR_INVALID_ARG, "null output array");
  std::vector<int> st(steps, steps + n);
  for (int v : st)
    if (v < 1) return fail(MQ_ERR_INVALID_ARG, "steps must be >= 1");
  const int S = split_steps == 0 ? 32 : (split_steps < 0 ? 0 : split_steps);
  const PiecePlan pl = plan_pieces(st, std::min<size_t>((size_t)n, (size_t)slots), S);
  const int m = (int)pl.orig.size();
  for (int e = 0; e < m && e < cap; ++e) {
    orig[e] = pl.orig[e];
    first[e] = pl.first[e];
    len[e] = pl.len[e];
    dep[e] = pl.dep[e];
  }
  if (makespan) {
    makespan[0] = pl.mk0;
    makespan[1] = pl.mk;
  }
  *m_out = m;
  return MQ_OK;
}

int mq_debug_apply(mq_problem* p, int32_t which, double dt, int32_t n, const double* xi,
                   const double* x, double* y) {
  if (int rh = refuse_host(p)) return rh;
  if (!p || !xi || !x || !y) return fail(MQ_ERR_INVALID_ARG, "null argument");
  if (which < 0 || which > 2 || n < 1 || !(dt > 0)) return fail(MQ_ERR_INVALID_ARG, "invalid arguments");
  int rc = check_finite(p, xi, (size_t)n * p->n_xi);
  if (rc) return rc;
  TmpPtr<double> tables;
  rc = assemble(p, xi, n, tables);
  if (rc) return rc;
  HIP_TRY(launch_apply(p->hm.g, which, dt, tables.get(), n, x, y, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return MQ_OK;
}

int mlmc_level_run_noalloc(mq_problem* p, const mq_level_desc* lv, int32_t n_samples, const double* xi,
                           double* q_fine, double* q_coarse, double* final_state, mq_run_stats* st) {
  last_flags().clear();
  if (int rh = refuse_host(p)) return rh;
  if (!p || !lv) return fail(MQ_ERR_INVALID_ARG, "null argument");
  if (p->path == MQ_PATH_WIDE) return fail(MQ_ERR_INVALID_ARG, "the wide path allocates its own workspace");
  if (!p->scratch) return fail(MQ_ERR_DEVICE, "the fixed workspace of this device was not found at set-up");
  if (n_samples < 1) return fail(MQ_ERR_INVALID_ARG, "n_samples must be >= 1");
  if (lv->steps_per_period < 1 || lv->n_periods < 1 || lv->coarse_steps_per_period < 0)
    return fail(MQ_ERR_INVALID_ARG, "steps_per_period, n_periods >= 1 and coarse_steps_per_period >= 0 required");
  const int64_t nf = (int64_t)lv->steps_per_period * lv->n_periods;
  const int64_t nc = (int64_t)lv->coarse_steps_per_period * lv->n_periods;
  if (nf > (1 << 24) || nc > (1 << 24)) return fail(MQ_ERR_INVALID_ARG, "too many steps");
  const size_t need = noalloc_need(p, n_samples, nf, nc, final_state != nullptr);
  if (need > (size_t)MQ_NOALLOC_WORKSPACE_BYTES)
    return fail(MQ_ERR_INVALID_ARG, "the run needs " + std::to_string(need) + " bytes of workspace, more than the " +
                                        std::to_string((size_t)MQ_NOALLOC_WORKSPACE_BYTES) +
                                        " of the allocation-free call (use mlmc_level_run or fewer samples)");
  return level_run_dev(p, lv, n_samples, xi, q_fine, q_coarse, final_state, st, p->scratch,
                       (size_t)MQ_NOALLOC_WORKSPACE_BYTES);
}

// ---- host-pointer forms (mem_kind = MQ_MEM_HOST): inputs copied to per-call
// device buffers, the device form run, outputs copied back; blocking ----

int mq_set_initial_state(mq_problem* p, const double* a0) {
  if (!host_mode(p) || !a0) return set_initial_state_dev(p, a0);
  const size_t nd = (size_t)p->hm.g.n * p->hm.g.n;
  TmpPtr<double> d;
  HIP_TRY(tmp_alloc(d, nd, p->stream));
  HIP_TRY(copy_sync(d.get(), a0, nd * sizeof(double), hipMemcpyHostToDevice, p->stream));
  return set_initial_state_dev(p, d.get());
}

int mlmc_level_run(mq_problem* p, const mq_level_desc* lv, int32_t n_samples, const double* xi,
                   double* q_fine, double* q_coarse, double* final_state, mq_run_stats* st) {
  if (!host_mode(p)) return level_run_dev(p, lv, n_samples, xi, q_fine, q_coarse, final_state, st);
  if (n_samples < 1) return fail(MQ_ERR_INVALID_ARG, "n_samples must be >= 1");
  if (!xi || !q_fine) return fail(MQ_ERR_INVALID_ARG, "xi and q_fine are required");
  const size_t n = (size_t)n_samples, nd = (size_t)p->hm.g.n * p->hm.g.n;
  TmpPtr<double> dxi, dqf, dqc, dfs;
  HIP_TRY(tmp_alloc(dxi, n * p->n_xi, p->stream));
  HIP_TRY(copy_sync(dxi.get(), xi, n * p->n_xi * sizeof(double), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(tmp_alloc(dqf, n, p->stream));
  if (q_coarse) HIP_TRY(tmp_alloc(dqc, n, p->stream));
  if (final_state) HIP_TRY(tmp_alloc(dfs, n * nd, p->stream));
  const int rc = level_run_dev(p, lv, n_samples, dxi.get(), dqf.get(), q_coarse ? dqc.get() : nullptr,
                               final_state ? dfs.get() : nullptr, st);
  if (rc < 0) return rc;
  HIP_TRY(hipMemcpyAsync(q_fine, dqf.get(), n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  if (q_coarse) HIP_TRY(hipMemcpyAsync(q_coarse, dqc.get(), n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  if (final_state)
    HIP_TRY(hipMemcpyAsync(final_state, dfs.get(), n * nd * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return rc;
}

int mlmc_multilevel_run(mq_problem* p, int32_t n_levels, const mq_level_desc* lv,
                        const int32_t* n_samples, const double* const* xi, double* const* q_fine,
                        double* const* q_coarse, mq_run_stats* st) {
  if (!host_mode(p)) return multilevel_run_dev(p, n_levels, lv, n_samples, xi, q_fine, q_coarse, st);
  if (!lv || !n_samples || !xi || !q_fine || !q_coarse) return fail(MQ_ERR_INVALID_ARG, "null argument");
  if (n_levels < 1 || n_levels > 64) return fail(MQ_ERR_INVALID_ARG, "n_levels must be in [1, 64]");
  std::vector<TmpPtr<double>> dxi(n_levels), dqf(n_levels), dqc(n_levels);
  std::vector<const double*> px(n_levels);
  std::vector<double*> pf(n_levels), pc(n_levels, nullptr);
  for (int l = 0; l < n_levels; ++l) {
    if (n_samples[l] < 1) return fail(MQ_ERR_INVALID_ARG, "n_samples must be >= 1");
    if (!xi[l] || !q_fine[l]) return fail(MQ_ERR_INVALID_ARG, "xi and q_fine are required");
    const size_t n = (size_t)n_samples[l];
    HIP_TRY(tmp_alloc(dxi[l], n * p->n_xi, p->stream));
    HIP_TRY(copy_sync(dxi[l].get(), xi[l], n * p->n_xi * sizeof(double), hipMemcpyHostToDevice, p->stream));
    HIP_TRY(tmp_alloc(dqf[l], n, p->stream));
    px[l] = dxi[l].get();
    pf[l] = dqf[l].get();
    if (q_coarse[l]) {
      HIP_TRY(tmp_alloc(dqc[l], n, p->stream));
      pc[l] = dqc[l].get();
    }
  }
  const int rc = multilevel_run_dev(p, n_levels, lv, n_samples, px.data(), pf.data(), pc.data(), st);
  if (rc < 0) return rc;
  for (int l = 0; l < n_levels; ++l) {
    const size_t b = (size_t)n_samples[l] * sizeof(double);
    HIP_TRY(hipMemcpyAsync(q_fine[l], pf[l], b, hipMemcpyDeviceToHost, p->stream));
    if (pc[l]) HIP_TRY(hipMemcpyAsync(q_coarse[l], pc[l], b, hipMemcpyDeviceToHost, p->stream));
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  return rc;
}

int parareal_run(mq_problem* p, const mq_parareal_desc* pd, int32_t n_samples, const double* xi,
                 double* q, int32_t* iters, double* final_state, mq_run_stats* st) {
  if (!host_mode(p)) return parareal_run_dev(p, pd, n_samples, xi, q, iters, final_state, st);
  if (n_samples < 1) return fail(MQ_ERR_INVALID_ARG, "n_samples must be >= 1");
  if (!xi || !q || !iters) return fail(MQ_ERR_INVALID_ARG, "xi, q and iters are required");
  const size_t n = (size_t)n_samples, nd = (size_t)p->hm.g.n * p->hm.g.n;
  TmpPtr<double> dxi, dq, dfs;
  TmpPtr<int32_t> dit;
  HIP_TRY(tmp_alloc(dxi, n * p->n_xi, p->stream));
  HIP_TRY(copy_sync(dxi.get(), xi, n * p->n_xi * sizeof(double), hipMemcpyHostToDevice, p->stream));
  HIP_TRY(tmp_alloc(dq, n, p->stream));
  HIP_TRY(tmp_alloc(dit, n, p->stream));
  if (final_state) HIP_TRY(tmp_alloc(dfs, n * nd, p->stream));
  const int rc = parareal_run_dev(p, pd, n_samples, dxi.get(), dq.get(), dit.get(),
                                  final_state ? dfs.get() : nullptr, st);
  if (rc < 0) return rc;
  HIP_TRY(hipMemcpyAsync(q, dq.get(), n * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipMemcpyAsync(iters, dit.get(), n * sizeof(int32_t), hipMemcpyDeviceToHost, p->stream));
  if (final_state)
    HIP_TRY(hipMemcpyAsync(final_state, dfs.get(), n * nd * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return rc;
}

}  // extern "C"
