// Internal: the problem handle and the host helpers shared by the C ABI
// (abi.cpp) and the request server (serve.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "mq_internal.h"
#include "setup.h"

namespace mq {

// Message of the last non-zero status on the calling thread.
std::string& last_error();

inline int fail(int code, const std::string& msg) {
  last_error() = msg;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e__ = (expr);                                                       \
    if (e__ != hipSuccess)                                                         \
      return ::mq::fail(e__ == hipErrorOutOfMemory ? MQ_ERR_OUT_OF_MEMORY : MQ_ERR_DEVICE, \
                        std::string(#expr) + ": " + hipGetErrorString(e__));       \
  } while (0)

// Device allocation owned by a unique_ptr.
struct DevFree {
  void operator()(void* p) const {
    if (p) (void)hipFree(p);
  }
};
template <class T>
using DevPtr = std::unique_ptr<T, DevFree>;

template <class T>
hipError_t dev_alloc(DevPtr<T>& out, size_t count) {
  T* p = nullptr;
  hipError_t e = hipMalloc((void**)&p, (count > 0 ? count : 1) * sizeof(T));
  if (e == hipSuccess) out.reset(p);
  return e;
}

// Pinned host allocation owned by a unique_ptr.
struct PinnedFree {
  void operator()(void* p) const {
    if (p) (void)hipHostFree(p);
  }
};
template <class T>
using PinPtr = std::unique_ptr<T, PinnedFree>;

// Per-call device buffer, allocated and freed in the order of one stream
// (hipMallocAsync / hipFreeAsync): unlike hipFree, releasing it does not wait
// for the work of other streams, so calls on different streams overlap.
struct StreamFree {
  hipStream_t s = nullptr;
  void operator()(void* p) const {
    if (p) (void)hipFreeAsync(p, s);
  }
};
template <class T>
using TmpPtr = std::unique_ptr<T, StreamFree>;

template <class T>
hipError_t tmp_alloc(TmpPtr<T>& out, size_t count, hipStream_t s) {
  T* p = nullptr;
  hipError_t e = hipMallocAsync((void**)&p, (count > 0 ? count : 1) * sizeof(T), s);
  if (e == hipSuccess) out = TmpPtr<T>(p, StreamFree{s});
  return e;
}

// Per-call device memory: stream-ordered allocations that live as long as this
// object, or consecutive 256-byte-aligned slices of a fixed region (then
// nothing is allocated: the allocation-free entry point).
class CallMem {
 public:
  void use_stream(hipStream_t s) { s_ = s; }
  void use_region(char* base, size_t cap) {
    base_ = base;
    cap_ = cap;
    used_ = 0;
  }
  bool fixed() const { return base_ != nullptr; }
  size_t left() const { return cap_ - used_; }
  static size_t rounded(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
  template <class T>
  hipError_t get(T*& out, size_t count) {
    const size_t bytes = rounded((count > 0 ? count : 1) * sizeof(T));
    if (base_) {
      if (bytes > cap_ - used_) return hipErrorOutOfMemory;
      out = reinterpret_cast<T*>(base_ + used_);
      used_ += bytes;
      return hipSuccess;
    }
    TmpPtr<char> t;
    const hipError_t e = tmp_alloc(t, bytes, s_);
    if (e != hipSuccess) return e;
    out = reinterpret_cast<T*>(t.get());
    owned_.push_back(std::move(t));
    return hipSuccess;
  }

 private:
  hipStream_t s_ = nullptr;
  char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
  std::vector<TmpPtr<char>> owned_;
};

// Copy ordered on stream s, complete when it returns.
inline hipError_t copy_sync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

}  // namespace mq

struct mq_problem {
  mq_problem_desc d;
  mq::HostMesh hm;
  int device = 0;
  hipStream_t stream = nullptr;
  int num_cu = 0;
  int lds_limit = 0;
  int n_xi = 0;
  double wall_khz = 100000.0;
  int resident_ok = 0;
  int lds_bytes = 0;
  int path = MQ_PATH_STREAMING;
  int precond = MQ_PRECOND_JACOBI;
  int tile = 1;
  mq::MGGeom mg{};
  double mat[10];
  mq::DevPtr<double> dS;
  mq::DevPtr<uint8_t> dcond;
  mq::DevPtr<double> dkl;
  mq::DevPtr<int> dcounter;
  mq::DevPtr<int> dflag;
  // per-slot work buffers (grown on demand, zeroed when allocated)
  mq::DevPtr<double> work;
  size_t work_slots = 0;
  // wide path: called on the host between time steps (may block to let other
  // work have the device); empty: none
  std::function<void()> wide_yield;
  // start state a_0 of later runs on the full grid (zero boundary ring), set by
  // mq_set_initial_state; empty: a_0 = 0
  mq::DevPtr<double> a0;
  // completion records of the last launch's entries (coherent pinned host
  // memory, grown on demand; see HostDone)
  mq::PinPtr<mq::HostDone> done_rec;
  size_t done_cap = 0;
  // this device's fixed workspace of the allocation-free entry point
  // (MQ_NOALLOC_WORKSPACE_BYTES, shared by every handle on the device)
  char* scratch = nullptr;
};

namespace mq {

Solver solver_of(const mq_problem* p);
// Persistent-kernel slots the device holds at once for this problem.
size_t max_slots(const mq_problem* p);
// Grow the work buffer to `slots` slots (allocation; call while the stream is idle).
int ensure_work(mq_problem* p, size_t slots);
// Device bytes of `slots` work slots.
size_t work_bytes(const mq_problem* p, size_t slots);
// J(t_k) = J0 sin(2 pi f k dt), k = 0..n_total (FP64 on the host).
std::vector<double> source_table(const mq_problem_desc& d, double dt, int n_total);
// Launch one persistent time-stepping kernel over the device instance table
// `dinst` on p->stream without waiting.  The work buffer must already hold
// min(n, max_slots(p)) slots.
// work (nullable): use these work_slots slots instead of the handle's work buffer.
// n_first >= 0: entries [0, n_first) form a second work queue that workgroups
// below grid_first take first (see the kernels' queue_next).
// para: the entries include one-launch Parareal entries.
int launch_persistent(mq_problem* p, const Inst* dinst, int n, int* grid, int* block, double* work = nullptr,
                      size_t work_slots = 0, int n_first = -1, int grid_first = -1, bool para = false);
// Wide path (wide.cpp): run the instances one after the other over the whole device.
// flags (nullable): receives one entry of FLAG_* bits per instance, in insts order
int run_wide(mq_problem* p, std::vector<Inst>& insts, mq_run_stats* st, int* status, std::vector<int>* flags);

}  // namespace mq
