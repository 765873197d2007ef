// Wide path: the instances of a call run one after the other, each spread
// over the whole device (every solver pass is a grid-wide kernel).  The inner
// multigrid-CG iterations are replayed in batches from a captured graph; the
// passes of an iteration return at once after convergence (a flag in device
// memory), so the host reads that flag once per batch.  For few large
// instances this trades throughput for latency.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "problem.h"

namespace mq {

namespace {

constexpr int WIDE_BATCH = 4;  // inner iterations per graph replay

struct GraphExec {
  hipGraph_t g = nullptr;
  hipGraphExec_t e = nullptr;
  ~GraphExec() {
    if (e) (void)hipGraphExecDestroy(e);
    if (g) (void)hipGraphDestroy(g);
  }
};

}  // namespace

int run_wide(mq_problem* p, std::vector<Inst>& insts, mq_run_stats* st, int* status, std::vector<int>* flags_out) {
  const Geom& g = p->hm.g;
  for (const Inst& in : insts)
    if (in.n_chain > 0 || in.carry) return fail(MQ_ERR_INVALID_ARG, "the wide path runs plain level instances only");
  HIP_TRY(hipStreamSynchronize(p->stream));
  int rc = ensure_work(p, 1);
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(p->stream));
  // the legacy default stream cannot be captured: a private stream then
  // (every stream takes a share of the process's hardware queues, so an
  // explicit stream is used as it is)
  struct OwnStream {
    hipStream_t s = nullptr;
    ~OwnStream() {
      if (s) (void)hipStreamDestroy(s);
    }
  } own;
  if (!p->stream) HIP_TRY(hipStreamCreateWithFlags(&own.s, hipStreamNonBlocking));
  const hipStream_t ws = p->stream ? p->stream : own.s;
  const size_t FS = (size_t)g.N * g.P, RHW = (size_t)g.RW * g.RH;
  const size_t vsz = p->d.precision == MQ_PREC_FP64 ? sizeof(double) : sizeof(float);
  WideCtx c{};
  c.g = g;
  c.mg = p->mg;
  c.sv = solver_of(p);
  c.air = 4.0 * g.nu_air;
  // coarse levels larger than one workgroup's comfortable size run grid-wide
  c.lt = 1;
  while (c.lt < c.mg.nlev && c.mg.lv[c.lt].n > 63) ++c.lt;
  c.sub = MGGeom{};
  c.sub.nlev = c.mg.nlev - c.lt + 1;
  c.sub.region_elems = c.mg.region_elems;
  c.sub.ctab_elems = c.mg.ctab_elems;
  c.sub.lv[0] = c.mg.lv[c.lt - 1];
  for (int l = 1; l <= c.sub.nlev; ++l) c.sub.lv[l] = c.mg.lv[c.lt - 1 + l];
  c.nblk = wide_blocks(g);
  // slot 0 of the work buffer in the streaming layout
  double* base = p->work.get();
  c.w.Av = base;
  c.w.Xv = base + FS;
  c.w.Bv = base + 2 * FS;
  c.w.Xp = base + 4 * FS;
  char* vb = reinterpret_cast<char*>(base + p->work_slots * ie_work_doubles(g));
  auto vec = [&](size_t k) { return (void*)(vb + k * vsz); };
  c.w.R = vec(0);
  c.w.Y = vec(FS);
  c.w.P = vec(2 * FS);
  c.w.Z = vec(3 * FS);
  c.w.T = vec(4 * FS);
  c.w.Q = vec(5 * FS);
  c.w.tE = vec(6 * FS);
  c.w.tN = vec(6 * FS + RHW);
  c.w.tNE = vec(6 * FS + 2 * RHW);
  c.w.tD = vec(6 * FS + 3 * RHW);
  c.w.tDi = vec(6 * FS + 4 * RHW);
  c.w.mgreg = vec(6 * FS + 5 * RHW);
  c.w.ctab = vec(6 * FS + 5 * RHW + c.mg.region_elems);
  c.w.S = p->dS.get();
  TmpPtr<double> part;
  TmpPtr<WideScal> sc;
  HIP_TRY(tmp_alloc(part, 2 * (size_t)c.nblk, ws));
  HIP_TRY(tmp_alloc(sc, 1, ws));
  c.w.part = part.get();
  c.w.sc = sc.get();

  // capture one batch of inner iterations (its kernels read everything that
  // changes from device memory, so one graph serves every instance).  Another
  // thread's operation on the legacy default stream can invalidate a capture;
  // the batch is then launched directly (the same kernels in the same order).
  GraphExec graph;
  bool use_graph = false;
  if (hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal) == hipSuccess) {
    hipError_t ce = hipSuccess;
    for (int b = 0; b < WIDE_BATCH && ce == hipSuccess; ++b) ce = wide_iteration(c, ws);
    const hipError_t ee = hipStreamEndCapture(ws, &graph.g);
    use_graph = ce == hipSuccess && ee == hipSuccess && graph.g &&
                hipGraphInstantiate(&graph.e, graph.g, nullptr, nullptr, 0) == hipSuccess;
  }
  if (!use_graph) {
    (void)hipGetLastError();
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(ws, &cs));
    if (cs != hipStreamCaptureStatusNone) return fail(MQ_ERR_DEVICE, "wide path: stream left in capture");
  }

  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, ws));
  const int max_batches = c.sv.max_iter / WIDE_BATCH + 2;
  WideScal h{};
  auto read_sc = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(&h, sc.get(), sizeof(WideScal), hipMemcpyDeviceToHost, ws);
    if (e == hipSuccess) e = hipStreamSynchronize(ws);
    return e;
  };
  for (Inst& in : insts) {
    c.w.tab = in.tab;
    const double inv_dt = 1.0 / in.dt;
    HIP_TRY(wide_setup(c, inv_dt, in.a_init, ws));
    int flags = 0, sweeps = 0;
    std::vector<double> src(in.n_steps);
    HIP_TRY(hipMemcpyAsync(src.data(), in.src + in.k0 + 1, in.n_steps * sizeof(double), hipMemcpyDeviceToHost,
                           ws));
    HIP_TRY(hipStreamSynchronize(ws));
    for (int step = 0; step < in.n_steps; ++step) {
      if (p->wide_yield) p->wide_yield();
      HIP_TRY(wide_rhs(c, src[step], ws));
      bool conv = false;
      for (int sweep = 0; sweep <= c.sv.max_sweeps; ++sweep) {
        HIP_TRY(wide_resid(c, inv_dt, ws));
        HIP_TRY(read_sc());
        if (h.flags & FLAG_FAILED) break;
        if (h.conv) {
          conv = true;
          break;
        }
        if (sweep == c.sv.max_sweeps) break;
        ++sweeps;
        for (int b = 0; b < max_batches; ++b) {
          if (use_graph) {
            HIP_TRY(hipGraphLaunch(graph.e, ws));
          } else {
            for (int i = 0; i < WIDE_BATCH; ++i) HIP_TRY(wide_iteration(c, ws));
          }
          HIP_TRY(read_sc());
          if (h.done) break;
        }
        HIP_TRY(wide_xupd(c, ws));
      }
      if (!conv) flags |= FLAG_NOT_CONVERGED;
      HIP_TRY(wide_end_step(c, inv_dt, ws));
    }
    HIP_TRY(wide_finish(c, in.q_scale, in.q_out, in.a_out, ws));
    HIP_TRY(read_sc());
    flags |= h.flags;
    if (flags_out) flags_out->push_back(flags);
    if (st) {
      st->n_instances += 1;
      st->sample_steps += in.n_steps;
      st->inner_iters += h.it_total;
      st->sweeps += sweeps;
      if (flags & FLAG_NOT_CONVERGED) st->n_not_converged++;
      if (flags & FLAG_FAILED) st->n_failed++;
    }
    if (flags & FLAG_WARN) *status = MQ_WARN_NOT_CONVERGED;
  }
  HIP_TRY(hipEventRecord(e1, ws));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) {
    st->kernel_ms += ms;
    st->path = MQ_PATH_WIDE;
    st->grid = c.nblk;
    st->block = 256;
  }
  return MQ_OK;
}

}  // namespace mq
