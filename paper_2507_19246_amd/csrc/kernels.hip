// HIP kernels for gfx950 (CDNA4, wave64).
//
//  k_assemble      per-sample materials (Eq. (1) coefficients sigma, nu per
//                  element) and the P1 stencils of M_sigma and K_nu (Eq. (4))
//                  on the sample-dependent box, FP64.
//  k_ie_resident   persistent implicit Euler (Eqs. (6)-(7), increment form)
//                  with FP64 iterative refinement around a Jacobi-scaled CG in
//                  VT (float or double); one workgroup owns one instance and
//                  keeps the CG vectors in registers and LDS; the Joule-loss
//                  sum of Eq. (26) is accumulated in FP64.
//  k_ie_stream     same algorithm with the CG vectors in global memory, for
//                  meshes whose state does not fit one compute unit.
//  small kernels   debug operator apply, layout copies, level statistics of
//                  Eq. (9), Parareal interface jumps (Eq. (12) stopping test).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "mq_internal.h"

namespace mq {

// ---------------------------------------------------------------------------
// materials + assembly
// ---------------------------------------------------------------------------
struct MatParams {
  double sigma0, nu_cond, nu_air, s_sigma, s_nu, s_kl, k1, k2, k3, s_k;
};

__device__ inline void elem_material(int material, const MatParams& mp, const uint8_t* cond,
                                     const double* kl, int n_modes, int e, const double* xi,
                                     double* sig, double* nu) {
  if (!cond[e]) {
    *sig = 0.0;
    *nu = mp.nu_air;
    return;
  }
  if (material == MQ_MAT_LOGNORMAL_SCALAR) {
    *sig = mp.sigma0 * exp(mp.s_sigma * xi[0]);
    *nu = mp.nu_cond * exp(mp.s_nu * xi[1]);
  } else if (material == MQ_MAT_KL) {
    double gsum = 0.0;
    for (int k = 0; k < n_modes; ++k) gsum = fma(kl[(size_t)e * n_modes + k], xi[k], gsum);
    *sig = exp(log(mp.sigma0) + mp.s_kl * gsum);
    *nu = mp.nu_cond;
  } else {  // nonlinear iron: nu at B = 0 here, updated by the Picard loop
    *sig = mp.sigma0;
    *nu = mp.k1 * exp(mp.s_k * xi[0]) + mp.k3 * exp(mp.s_k * xi[2]);
  }
}

// One thread per (table node, sample).  Box nodes get the six-triangle P1
// stencil; other table nodes the air constants (M = 0, K = nu_air * [4, -1]).
//   K_C = nu(a0)/2 + nu(a1)/2 + nu(b0) + nu(c1) + nu(d0)/2 + nu(d1)/2
//   K_E = -(nu(a0) + nu(c1))/2          K_N = -(nu(a1) + nu(b0))/2
//   M_C = h^2/12 * (sum of the six sigmas)
//   M_E = h^2/24 (s(a0) + s(c1))  M_N = h^2/24 (s(a1) + s(b0))  M_NE = h^2/24 (s(a0) + s(a1))
// with a = cell (I, J), b = cell (I-1, J), c = cell (I, J-1), d = cell (I-1, J-1)
// of full-grid node (I, J); t0 = {(I,J),(I+1,J),(I+1,J+1)}, t1 = {(I,J),(I+1,J+1),(I,J+1)}.
__global__ void k_assemble(Geom g, CellRegion cr, const uint8_t* __restrict__ cond,
                           const double* __restrict__ kl, int n_modes, int material, MatParams mp,
                           const double* __restrict__ xi, int n_xi, int n_samples,
                           double* __restrict__ tables) {
  const int RHW = g.RW * g.RH;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int smp = blockIdx.y;
  if (t >= RHW || smp >= n_samples) return;
  double* T = tables + (size_t)smp * tab_stride(g);
  if (t == 0) {
    const double* x0 = xi + (size_t)smp * n_xi;
    double* kp = T + T_NPLANES * RHW;
    const bool nl = material == MQ_MAT_NONLINEAR;
    kp[0] = nl ? mp.k1 * exp(mp.s_k * x0[0]) : 0.0;
    kp[1] = nl ? mp.k2 * exp(mp.s_k * x0[1]) : 0.0;
    kp[2] = nl ? mp.k3 * exp(mp.s_k * x0[2]) : 0.0;
    kp[3] = 0.0;
  }
  const int i = g.bx0 - 1 + t % g.RW;
  const int j = g.by0 - 1 + t / g.RW;
  const bool inbox = i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1;
  if (!inbox) {
    T[T_MC * RHW + t] = 0.0;
    T[T_ME * RHW + t] = 0.0;
    T[T_MN * RHW + t] = 0.0;
    T[T_MNE * RHW + t] = 0.0;
    T[T_KC * RHW + t] = 4.0 * g.nu_air;
    T[T_KE * RHW + t] = -g.nu_air;
    T[T_KN * RHW + t] = -g.nu_air;
    return;
  }
  const double* x = xi + (size_t)smp * n_xi;
  const int I = i + 1, J = j + 1;  // full-grid node
  auto eidx = [&](int ci, int cj, int tt) { return ((cj - cr.cy0) * cr.cw + (ci - cr.cx0)) * 2 + tt; };
  double sa0, na0, sa1, na1, sb0, nb0, sc1, nc1, sd0, nd0, sd1, nd1;
  elem_material(material, mp, cond, kl, n_modes, eidx(I, J, 0), x, &sa0, &na0);
  elem_material(material, mp, cond, kl, n_modes, eidx(I, J, 1), x, &sa1, &na1);
  elem_material(material, mp, cond, kl, n_modes, eidx(I - 1, J, 0), x, &sb0, &nb0);
  elem_material(material, mp, cond, kl, n_modes, eidx(I, J - 1, 1), x, &sc1, &nc1);
  elem_material(material, mp, cond, kl, n_modes, eidx(I - 1, J - 1, 0), x, &sd0, &nd0);
  elem_material(material, mp, cond, kl, n_modes, eidx(I - 1, J - 1, 1), x, &sd1, &nd1);
  const double h12 = g.h2 / 12.0, h24 = g.h2 / 24.0;
  T[T_MC * RHW + t] = h12 * (sa0 + sa1 + sb0 + sc1 + sd0 + sd1);
  T[T_ME * RHW + t] = h24 * (sa0 + sc1);
  T[T_MN * RHW + t] = h24 * (sa1 + sb0);
  T[T_MNE * RHW + t] = h24 * (sa0 + sa1);
  T[T_KC * RHW + t] = 0.5 * (na0 + na1 + nd0 + nd1) + nb0 + nc1;
  T[T_KE * RHW + t] = -0.5 * (na0 + nc1);
  T[T_KN * RHW + t] = -0.5 * (na1 + nb0);
}

hipError_t launch_assemble(const Geom& g, const CellRegion& cr, const uint8_t* cond,
                           const double* kltab, int n_modes, int material, const double* xi,
                           int n_xi, int n_samples, const double* mat_params, double* tables,
                           hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  MatParams mp;
  mp.sigma0 = mat_params[0];
  mp.nu_cond = mat_params[1];
  mp.nu_air = mat_params[2];
  mp.s_sigma = mat_params[3];
  mp.s_nu = mat_params[4];
  mp.s_kl = mat_params[5];
  mp.k1 = mat_params[6];
  mp.k2 = mat_params[7];
  mp.k3 = mat_params[8];
  mp.s_k = mat_params[9];
  const int RHW = g.RW * g.RH;
  dim3 grid((RHW + 255) / 256, n_samples);
  hipLaunchKernelGGL(k_assemble, grid, dim3(256), 0, st, g, cr, cond, kltab, n_modes, material,
                     mp, xi, n_xi, n_samples, tables);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 stencil helpers on full-grid vectors (pitch P, zero boundary ring)
// ---------------------------------------------------------------------------
struct NodeRef {
  int gi;     // full-grid index
  int t;      // table index (valid when inL)
  bool inL;   // node reads its couplings from the tables
};

__device__ inline NodeRef node_ref(const Geom& g, int i, int j) {
  NodeRef r;
  r.gi = (j + 1) * g.P + (i + 1);
  r.inL = i >= g.bx0 && i < g.lx1 && j >= g.by0 && j < g.ly1;
  r.t = (j - g.by0 + 1) * g.RW + (i - g.bx0 + 1);
  return r;
}

// (K v)_node
__device__ inline double K_apply(const Geom& g, const double* __restrict__ tab, const double* v,
                                 const NodeRef& nr) {
  const int P = g.P;
  const double c = v[nr.gi], e = v[nr.gi + 1], w = v[nr.gi - 1], n = v[nr.gi + P], s = v[nr.gi - P];
  if (!nr.inL) return g.nu_air * (4.0 * c - (e + w) - (n + s));
  const int RHW = g.RW * g.RH, t = nr.t;
  const double* KC = tab + T_KC * RHW;
  const double* KE = tab + T_KE * RHW;
  const double* KN = tab + T_KN * RHW;
  return KC[t] * c + KE[t] * e + KE[t - 1] * w + KN[t] * n + KN[t - g.RW] * s;
}

// (M v)_node (zero outside the lookup region)
__device__ inline double M_apply(const Geom& g, const double* __restrict__ tab, const double* v,
                                 const NodeRef& nr) {
  if (!nr.inL) return 0.0;
  const int P = g.P, RHW = g.RW * g.RH, t = nr.t;
  const double* MC = tab + T_MC * RHW;
  const double* ME = tab + T_ME * RHW;
  const double* MN = tab + T_MN * RHW;
  const double* MNE = tab + T_MNE * RHW;
  const int gi = nr.gi;
  return MC[t] * v[gi] + ME[t] * v[gi + 1] + ME[t - 1] * v[gi - 1] + MN[t] * v[gi + P] +
         MN[t - g.RW] * v[gi - P] + MNE[t] * v[gi + P + 1] + MNE[t - g.RW - 1] * v[gi - P - 1];
}

// ((M/dt + K) v)_node
__device__ inline double A_apply(const Geom& g, const double* __restrict__ tab, const double* v,
                                 const NodeRef& nr, double inv_dt) {
  if (!nr.inL) return K_apply(g, tab, v, nr);
  return M_apply(g, tab, v, nr) * inv_dt + K_apply(g, tab, v, nr);
}

// A_apply, M_apply and K_apply with the table loads grouped: a node inside
// the lookup region issues all its table loads before any use, and a wave
// with no such node issues none.  Same expression per node as A_apply,
// M_apply and K_apply.
struct Tab7 {
  double kc, ke, kw, kn, ks, mc, me, mw, mn, ms, mne, msw;
};
__device__ inline Tab7 tab_load(const Geom& g, const double* __restrict__ tab, const NodeRef& nr, bool want_m,
                                bool want_k) {
  Tab7 T{};
  if (nr.inL) {
    const int RW = g.RW, RHW = g.RW * g.RH, t = nr.t;
    if (want_k) {
      T.kc = tab[T_KC * RHW + t];
      T.ke = tab[T_KE * RHW + t];
      T.kw = tab[T_KE * RHW + t - 1];
      T.kn = tab[T_KN * RHW + t];
      T.ks = tab[T_KN * RHW + t - RW];
    }
    if (want_m) {
      T.mc = tab[T_MC * RHW + t];
      T.me = tab[T_ME * RHW + t];
      T.mw = tab[T_ME * RHW + t - 1];
      T.mn = tab[T_MN * RHW + t];
      T.ms = tab[T_MN * RHW + t - RW];
      T.mne = tab[T_MNE * RHW + t];
      T.msw = tab[T_MNE * RHW + t - RW - 1];
    }
  }
  return T;
}
__device__ inline double A_apply_u(const Geom& g, const double* __restrict__ tab, const double* v,
                                   const NodeRef& nr, double inv_dt) {
  const int P = g.P, gi = nr.gi;
  const double c = v[gi], e = v[gi + 1], w = v[gi - 1], n = v[gi + P], s = v[gi - P], ne = v[gi + P + 1],
               sw = v[gi - P - 1];
  const Tab7 T = tab_load(g, tab, nr, true, true);
  const double air = g.nu_air * (4.0 * c - (e + w) - (n + s));
  const double m = T.mc * c + T.me * e + T.mw * w + T.mn * n + T.ms * s + T.mne * ne + T.msw * sw;
  const double k = T.kc * c + T.ke * e + T.kw * w + T.kn * n + T.ks * s;
  return nr.inL ? m * inv_dt + k : air;
}
__device__ inline double K_apply_u(const Geom& g, const double* __restrict__ tab, const double* v,
                                   const NodeRef& nr) {
  const int P = g.P, gi = nr.gi;
  const double c = v[gi], e = v[gi + 1], w = v[gi - 1], n = v[gi + P], s = v[gi - P];
  const Tab7 T = tab_load(g, tab, nr, false, true);
  const double air = g.nu_air * (4.0 * c - (e + w) - (n + s));
  return nr.inL ? T.kc * c + T.ke * e + T.kw * w + T.kn * n + T.ks * s : air;
}
// (M v)_node inside the lookup region (callers add it only there)
__device__ inline double M_apply_u(const Geom& g, const double* __restrict__ tab, const double* v,
                                   const NodeRef& nr) {
  const int P = g.P, gi = nr.gi;
  const double c = v[gi], e = v[gi + 1], w = v[gi - 1], n = v[gi + P], s = v[gi - P], ne = v[gi + P + 1],
               sw = v[gi - P - 1];
  const Tab7 T = tab_load(g, tab, nr, true, false);
  return T.mc * c + T.me * e + T.mw * w + T.mn * n + T.ms * s + T.mne * ne + T.msw * sw;
}

// ---------------------------------------------------------------------------
// deterministic reductions (wave64 butterfly, then waves in order)
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Reduce NV values over the workgroup; every thread gets the same sums.
// `red` holds 2 slots of [NWAVES][4] doubles; `slot` alternates between calls
// so that one barrier per reduction suffices.
template <int NV, int NWAVES>
__device__ inline void block_sum(double (&v)[NV], double* red, int& slot) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  double* base = red + slot * NWAVES * 4;
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) base[wv * 4 + q] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int k = 0; k < NWAVES; ++k) s += base[k * 4 + q];
    v[q] = s;
  }
  slot ^= 1;
}

// ---------------------------------------------------------------------------
// Persistent work queue: two queues in one launch
// ---------------------------------------------------------------------------
// counter[0], counter[1]: next position in queue 0 (entries [0, counter[2]))
// and queue 1 (entries [counter[2], n_inst)); workgroups below counter[3]
// start on queue 0, the others on queue 1, and each moves to the other queue
// once its own is empty.  Called by thread 0; returns n_inst when both queues
// are empty.  Within a queue, entries are handed out in order.
__device__ inline int queue_next(int* counter, int n_inst, int& q, int& moved) {
  const int n0 = counter[2];
  for (;;) {
    const int base = q == 0 ? 0 : n0, end = q == 0 ? n0 : n_inst;
    if (base < end) {
      const int k = atomicAdd(counter + q, 1);
      if (base + k < end) return base + k;
    }
    if (moved) return n_inst;
    moved = 1;
    q ^= 1;
  }
}

__global__ void k_queue_init(int* counter, int n_first, int grid_first) {
  if (threadIdx.x == 0) {
    counter[0] = 0;
    counter[1] = 0;
    counter[2] = n_first;
    counter[3] = grid_first;
  }
}

hipError_t launch_queue_init(int* counter, int n_first, int grid_first, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  hipLaunchKernelGGL(k_queue_init, dim3(1), dim3(64), 0, st, counter, n_first, grid_first);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Parareal in one persistent launch: flags between queue entries
// ---------------------------------------------------------------------------
// Wait (thread 0, bounded) until *f is set, then make the writer's data visible
// to the whole workgroup (the writer may have run on another XCD).  Returns
// false after the time limit.
// abort (nullable): a launch-wide flag; a wait that times out sets it, and every
// wait that sees it gives up at once, so a missing flag costs one time limit
// per launch, not one per entry.
template <int NT>
__device__ inline bool para_wait(const int* f, unsigned long long limit, int* s_ok, int* abort = nullptr) {
  if (threadIdx.x == 0) {
    const unsigned long long t0 = wall_clock64();
    int ok = 1;
    while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      if (wall_clock64() - t0 > limit ||
          (abort && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
        ok = 0;
        if (abort) __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(8);
    }
    *s_ok = ok;
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  const bool ok = *s_ok != 0;
  __syncthreads();
  return ok;
}

// Publish everything the workgroup wrote, then set *f.
__device__ inline void para_set(int* f) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(f, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Entry prologue of a queue entry (false at once for entries that are not part
// of a one-launch Parareal run).  Returns true when a Parareal entry has
// nothing to run: its sample stopped at an earlier iteration, or (coarse chain
// of iteration j >= 1) the jumps of iteration j stop it now, or no correction
// segment is left.  Such an entry sets every flag it owns.  A chain j >= 1
// that continues has computed the jumps of Section II-C's stopping test
// (largest ||F_n - U_n|| / ||F_n|| over n = j..M-1), written U_j = F_j and set
// first_done; *flags gets FLAG_FAILED after a timed-out wait.
template <int NT, int NWAVES>
__device__ bool para_prologue(const Geom& g, const Inst& in, double* red, int& slot, int* s_ok, int* flags) {
  // every branch below is taken by the workgroup as a whole (wave-uniform values)
  if (__builtin_amdgcn_readfirstlane(in.para != nullptr ? 1 : 0) == 0) return false;  // not a Parareal entry
  const ParaCtl* pc = in.para;
  const int s = __builtin_amdgcn_readfirstlane(in.sample);
  const int j = __builtin_amdgcn_readfirstlane(in.para_iter);
  const int n_jump = __builtin_amdgcn_readfirstlane(in.n_jump);
  const int n_chain = __builtin_amdgcn_readfirstlane(in.n_chain);
  const bool chain = __builtin_amdgcn_readfirstlane(in.para_chain) != 0;
  const int n = g.n, nd = n * n;
  __shared__ int s_skip;
  if (threadIdx.x == 0) {
    const int K = __hip_atomic_load(pc->K + s, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    s_skip = (K != 0 && K < j) ? 1 : 0;
  }
  __syncthreads();
  int skip = __builtin_amdgcn_readfirstlane(s_skip);
  __syncthreads();
  if (!skip && chain && j >= 1) {
    double Jmax = 0.0;
    for (int k = 0; k < n_jump; ++k) {
      if (!para_wait<NT>(in.jump_wait[k], PARA_WAIT_TICKS, s_ok, pc->abort)) *flags |= FLAG_FAILED;
      const double* F = in.jump_f[k];
      const double* U = in.jump_u[k];
      double v[2] = {0.0, 0.0};
      for (int idx = threadIdx.x; idx < nd; idx += NT) {
        const int gi = (idx / n + 1) * g.P + idx % n + 1;
        const double d = F[gi] - U[gi];
        v[0] += d * d;
        v[1] += F[gi] * F[gi];
      }
      block_sum<2, NWAVES>(v, red, slot);
      Jmax = fmax(Jmax, v[1] > 0.0 ? sqrt(v[0] / v[1]) : sqrt(v[0]));
    }
    // the last slice's fine run has read U_{M-1}^(j-1) before the chain overwrites it
    if (!para_wait<NT>(in.jump_wait[n_jump], PARA_WAIT_TICKS, s_ok, pc->abort)) *flags |= FLAG_FAILED;
    const int stop = __builtin_amdgcn_readfirstlane(((pc->fixed_k == 0 && Jmax <= pc->tol) || j >= pc->kcap) ? 1 : 0);
    if (threadIdx.x == 0) {
      pc->J[(size_t)s * pc->kcap + (j - 1)] = Jmax;
      if (stop) {
        if (pc->fixed_k == 0 && Jmax > pc->tol) atomicOr(pc->flags + s, FLAG_PARAREAL_KMAX);
        __hip_atomic_store(pc->K + s, j, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (stop) {
      skip = 1;
    } else {
      for (int idx = threadIdx.x; idx < nd; idx += NT) {
        const int gi = (idx / n + 1) * g.P + idx % n + 1;
        in.u_first[gi] = in.f_first[gi];
      }
      para_set(in.first_done);
      // no segment left (j = M - 1): nothing to run; done flag set by the caller
      if (n_chain == 0) return true;
    }
  }
  if (skip) {
    if (in.first_done) para_set(in.first_done);
    if (in.seg_done)
      for (int k = 0; k < n_chain; ++k) para_set(in.seg_done[k]);
  }
  return skip != 0;
}

// ---------------------------------------------------------------------------
// resident time-stepping kernel
// ---------------------------------------------------------------------------
// Workgroup = CW * NS threads; thread (c, s) owns interior column i = c and
// rows [s*SH, s*SH + SH) (rows >= n idle).  CG vectors y, r, p, s, w of the
// thread's SH nodes stay in registers; r is mirrored into an LDS grid with a
// zero halo for the stencil; the scaled coupling tables of the box sit in LDS.
//
// Solver per step (increment form of Eq. (7)):
//   b = J(t_{k+1}) S - K a;   x = previous increment (warm start)
//   repeat: r64 = b - (M/dt + K) x in FP64; stop if ||r64|| <= tol ||b||;
//           g = D^{-1/2} r64 (VT); CG on D^{-1/2} A D^{-1/2} y = g from y = 0
//           (Jacobi preconditioning as a symmetric scaling) to ||r|| <=
//           inner_rtol ||g||; x += D^{-1/2} y
//   q += x^T M x / dt;  a += x
// CG uses the single-reduction recurrences of Chronopoulos and Gear (J. Comput.
// Appl. Math. 25 (1989)): s = A p and w = A r are carried so each iteration
// needs one stencil apply and one fused reduction of (r.r, w.r).
// Completion record of a launch entry in coherent pinned host memory: the
// value and flags first, then done with a system-scope release store, so a host
// thread that sees done (acquire) also sees q.
__device__ inline void publish_done(HostDone* hd, double q, int flags) {
  if (!hd) return;
  hd->q = q;
  hd->flags = flags;
  __hip_atomic_store(&hd->done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <typename VT>
__device__ inline VT vt(double x) { return (VT)x; }

// ---------------------------------------------------------------------------
// multigrid helpers (resident path)
// ---------------------------------------------------------------------------
// Coarse level l in LDS: vectors R, Z, T with a zero halo ((n+2)^2 each) and
// Galerkin tables C, E, N, NE and the inverse diagonal ID over the box +- 1
// ring (pitch RW).  Threads map to nodes as a TX x TY grid (TX = 2^txs >= n),
// so no integer division appears in the level loops.
// Outside its table region a level's operator is the air stencil
// air * [1, -1/4, -1/4, -1/4, -1/4] (air = 1 for a hierarchy of the scaled
// system, 4 nu_air for one of the unscaled operator).
template <typename VT>
struct CLev {
  int n, np, bx0, by0, lx1, ly1, RW, txs;
  VT air, air_id;
  VT *R, *Z, *T;
  const VT *C, *E, *N, *NE, *ID;
};

template <typename VT>
__device__ inline CLev<VT> clev(const MGGeom& mg, int l, VT* region, const VT* ctab, int nthr,
                                VT air = VT(1)) {
  const MGLevel& M = mg.lv[l];
  CLev<VT> L;
  L.air = air;
  L.air_id = VT(1) / air;
  L.n = M.n;
  L.np = M.n + 2;
  L.bx0 = M.bx0;
  L.by0 = M.by0;
  L.lx1 = M.lx1;
  L.ly1 = M.ly1;
  L.RW = M.RW;
  int s = 0;
  while ((1 << s) < M.n && (2 << s) <= nthr) ++s;
  L.txs = s;
  const int sz = L.np * L.np;
  L.R = region + M.vec_off;
  L.Z = L.R + sz;
  L.T = L.Z + sz;
  const int pl = M.RW * M.RH;
  L.C = ctab + M.tab_off;
  L.E = L.C + pl;
  L.N = L.E + pl;
  L.NE = L.N + pl;
  L.ID = L.NE + pl;
  return L;
}

template <typename VT>
__device__ inline bool clev_inL(const CLev<VT>& L, int i, int j) {
  return i >= L.bx0 && i < L.lx1 && j >= L.by0 && j < L.ly1;
}

// (A v)(i, j) and the inverse diagonal at a coarse node (v halo'd, pitch np)
template <typename VT>
__device__ inline VT capp(const CLev<VT>& L, const VT* v, int i, int j, VT* idg) {
  const int np = L.np, p = (j + 1) * np + i + 1;
  const VT c = v[p], e = v[p + 1], w = v[p - 1], nn = v[p + np], s = v[p - np];
  if (clev_inL(L, i, j)) {
    const int t = (j - L.by0 + 1) * L.RW + (i - L.bx0 + 1);
    *idg = L.ID[t];
    return L.C[t] * c + L.E[t] * e + L.E[t - 1] * w + L.N[t] * nn + L.N[t - L.RW] * s +
           L.NE[t] * v[p + np + 1] + L.NE[t - L.RW - 1] * v[p - np - 1];
  }
  *idg = L.air_id;
  return L.air * (c - VT(0.25) * ((e + w) + (nn + s)));
}

// A lane's value from the lane to its left / right in the wave (DPP wave
// shifts; 0 in lane 0 / lane 63).  Callers read them only where that lane is
// active.
__device__ inline float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ inline float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

// The same for levels in global memory: a node inside the table region
// issues all its table loads together before any use (a wave with no such
// node issues none), so the loads of a pass are not serialised behind the
// region test.  Same expression per node as capp.
template <typename VT>
__device__ inline VT capp_gm(const CLev<VT>& L, const VT* v, int i, int j, VT* idg) {
  const int np = L.np, p = (j + 1) * np + i + 1;
  const VT c = v[p], e = v[p + 1], w = v[p - 1], nn = v[p + np], s = v[p - np], ne = v[p + np + 1],
           sw = v[p - np - 1];
  const bool in = clev_inL(L, i, j);
  VT tc = VT(0), te = VT(0), tw = VT(0), tn = VT(0), ts = VT(0), tne = VT(0), tsw = VT(0), ti = VT(0);
  if (in) {
    const int t = (j - L.by0 + 1) * L.RW + (i - L.bx0 + 1);
    tc = L.C[t];
    te = L.E[t];
    tw = L.E[t - 1];
    tn = L.N[t];
    ts = L.N[t - L.RW];
    tne = L.NE[t];
    tsw = L.NE[t - L.RW - 1];
    ti = L.ID[t];
  }
  *idg = in ? ti : L.air_id;
  return in ? tc * c + te * e + tw * w + tn * nn + ts * s + tne * ne + tsw * sw
            : L.air * (c - VT(0.25) * ((e + w) + (nn + s)));
}

template <typename VT>
__device__ inline VT clev_id(const CLev<VT>& L, int i, int j) {
  return clev_inL(L, i, j) ? L.ID[(j - L.by0 + 1) * L.RW + (i - L.bx0 + 1)] : L.air_id;
}

// Restriction P^T t at coarse node (ic, jc): coarse c <-> fine 2c+1, weights 1
// and 1/2 on the six "/"-mesh neighbours; t halo'd with pitch fp.
template <typename VT>
__device__ inline VT restrict_at(const VT* t, int fp, int ic, int jc) {
  const int p = (2 * jc + 2) * fp + 2 * ic + 2;
  return t[p] + VT(0.5) * ((t[p + 1] + t[p - 1]) + (t[p + fp] + t[p - fp]) + (t[p + fp + 1] + t[p - fp - 1]));
}

// Prolongation (P z_c)(i, j): P1 interpolation on the coarse "/" triangulation;
// zc halo'd with pitch cp (its zero ring is the Dirichlet boundary).
template <typename VT>
__device__ inline VT prolong_at(const VT* zc, int cp, int i, int j) {
  const int ic = i >> 1, jc = j >> 1;  // i odd: coarse (i-1)/2 = ic; i even: coarse ic-1 and ic
  auto Zc = [&](int a, int b) { return zc[(b + 1) * cp + a + 1]; };
  const bool io = i & 1, jo = j & 1;
  if (io && jo) return Zc(ic, jc);
  if (!io && jo) return VT(0.5) * (Zc(ic - 1, jc) + Zc(ic, jc));
  if (io && !jo) return VT(0.5) * (Zc(ic, jc - 1) + Zc(ic, jc));
  return VT(0.5) * (Zc(ic - 1, jc - 1) + Zc(ic, jc));
}

// Synchronisation of wave 0 alone (coarse levels it handles by itself): its
// LDS operations are complete and ordered once they have been waited for.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Level passes; (me, nthr) are the participating threads.  GM: the level
// lives in global memory; the stencil passes then take two rows per step,
// both rows' loads ahead of either row's store (no node of a pass reads what
// another node of it writes), to double the loads in flight.
template <typename VT, bool GM = false>
__device__ inline void c_resid(const CLev<VT>& L, int me, int nthr) {  // T = R - A Z
  const int tx = me & ((1 << L.txs) - 1), ty = nthr >> L.txs;
  if (tx >= L.n) return;
  if constexpr (GM) {
    for (int j = me >> L.txs; j < L.n; j += 2 * ty) {
      const int j2 = j + ty < L.n ? j + ty : j;
      VT d;
      const int p = (j + 1) * L.np + tx + 1, p2 = (j2 + 1) * L.np + tx + 1;
      const VT a = L.R[p] - capp_gm(L, L.Z, tx, j, &d);
      const VT b = L.R[p2] - capp_gm(L, L.Z, tx, j2, &d);
      L.T[p] = a;
      if (j + ty < L.n) L.T[p2] = b;
    }
    return;
  }
  for (int j = me >> L.txs; j < L.n; j += ty) {
    VT d;
    const int p = (j + 1) * L.np + tx + 1;
    L.T[p] = L.R[p] - capp(L, L.Z, tx, j, &d);
  }
}
template <typename VT, bool GM = false>
__device__ inline void c_restrict(const CLev<VT>& F, const CLev<VT>& Cc, VT om, bool exact, int me,
                                  int nthr) {  // Cc.R = P^T F.T, Cc.Z = om ID R (ID R at the coarsest)
  const int tx = me & ((1 << Cc.txs) - 1), ty = nthr >> Cc.txs;
  if (tx >= Cc.n) return;
  if constexpr (GM) {
    const VT f = exact ? VT(1) : om;
    for (int j = me >> Cc.txs; j < Cc.n; j += 2 * ty) {
      const int j2 = j + ty < Cc.n ? j + ty : j;
      const VT r = restrict_at(F.T, F.np, tx, j), r2 = restrict_at(F.T, F.np, tx, j2);
      const VT d = clev_id(Cc, tx, j), d2 = clev_id(Cc, tx, j2);
      const int p = (j + 1) * Cc.np + tx + 1, p2 = (j2 + 1) * Cc.np + tx + 1;
      Cc.R[p] = r;
      Cc.Z[p] = f * d * r;
      if (j + ty < Cc.n) {
        Cc.R[p2] = r2;
        Cc.Z[p2] = f * d2 * r2;
      }
    }
    return;
  }
  for (int j = me >> Cc.txs; j < Cc.n; j += ty) {
    const VT r = restrict_at(F.T, F.np, tx, j);
    const int p = (j + 1) * Cc.np + tx + 1;
    Cc.R[p] = r;
    Cc.Z[p] = (exact ? VT(1) : om) * clev_id(Cc, tx, j) * r;
  }
}
template <typename VT, bool GM = false>
__device__ inline void c_prolong(const CLev<VT>& L, const VT* zc, int cp, int me, int nthr) {
  const int tx = me & ((1 << L.txs) - 1), ty = nthr >> L.txs;
  if (tx >= L.n) return;
  if constexpr (GM) {
    for (int j = me >> L.txs; j < L.n; j += 2 * ty) {
      const int j2 = j + ty < L.n ? j + ty : j;
      const int p = (j + 1) * L.np + tx + 1, p2 = (j2 + 1) * L.np + tx + 1;
      const VT a = L.Z[p] + prolong_at(zc, cp, tx, j), b = L.Z[p2] + prolong_at(zc, cp, tx, j2);
      L.Z[p] = a;
      if (j + ty < L.n) L.Z[p2] = b;
    }
    return;
  }
  for (int j = me >> L.txs; j < L.n; j += ty) L.Z[(j + 1) * L.np + tx + 1] += prolong_at(zc, cp, tx, j);
}
template <typename VT, bool GM = false>
__device__ inline void c_post(const CLev<VT>& L, VT om, int me, int nthr) {  // T = Z + om ID (R - A Z)
  const int tx = me & ((1 << L.txs) - 1), ty = nthr >> L.txs;
  if (tx >= L.n) return;
  if constexpr (GM) {
    for (int j = me >> L.txs; j < L.n; j += 2 * ty) {
      const int j2 = j + ty < L.n ? j + ty : j;
      VT id, id2;
      const int p = (j + 1) * L.np + tx + 1, p2 = (j2 + 1) * L.np + tx + 1;
      const VT az = capp_gm(L, L.Z, tx, j, &id), az2 = capp_gm(L, L.Z, tx, j2, &id2);
      const VT a = L.Z[p] + om * id * (L.R[p] - az), b = L.Z[p2] + om * id2 * (L.R[p2] - az2);
      L.T[p] = a;
      if (j + ty < L.n) L.T[p2] = b;
    }
    return;
  }
  for (int j = me >> L.txs; j < L.n; j += ty) {
    VT id;
    const int p = (j + 1) * L.np + tx + 1;
    const VT az = capp(L, L.Z, tx, j, &id);
    L.T[p] = L.Z[p] + om * id * (L.R[p] - az);
  }
}
template <typename VT>
__device__ inline void c_zero_halo(const CLev<VT>& L, int me, int nthr) {
  const int np = L.np, m = 4 * (L.n + 1);
  for (int q = me; q < m; q += nthr) {
    int p;
    if (q < np) p = q;                                   // row 0
    else if (q < 2 * np) p = (L.n + 1) * np + (q - np);  // row n+1
    else if (q < 2 * np + L.n) p = (q - 2 * np + 1) * np;          // column 0
    else p = (q - 2 * np - L.n + 1) * np + L.n + 1;                // column n+1
    L.R[p] = VT(0);
    L.Z[p] = VT(0);
    L.T[p] = VT(0);
  }
}

// Damped-Jacobi sweeps Z <- Z + om ID (R - A Z) at the coarsest level in
// use; returns the vector that holds the result (Z and T alternate).
template <typename VT, bool GM, class SYNC>
__device__ __attribute__((always_inline)) inline const VT* c_coarsest(CLev<VT> C, VT om, int sweeps, int me, int nthr, SYNC sync) {
  for (int s = 0; s < sweeps; ++s) {
    c_post<VT, GM>(C, om, me, nthr);
    sync();
    VT* t = C.Z;
    C.Z = C.T;
    C.T = t;
  }
  return C.Z;
}

// Coarse part of the V(1,1) cycle over levels 1..L (L = min(nlev, lmax) when
// lmax > 0), R_1 and Z_1 = om ID R_1 (ID R_1 if L = 1) already in place.  At
// level L, Z_L = ID R_L followed by `csweeps` damped-Jacobi sweeps (exact when
// level L is the single-node level).  Levels with n >= block_min use the whole
// workgroup, smaller ones run on wave 0 alone.  Returns level 1's corrected
// vector.
template <typename VT, int NT, bool GM = false>
__device__ __attribute__((always_inline)) inline const VT* coarse_cycle(const MGGeom& mg, VT* region, const VT* ctab, VT om, int tid,
                                         VT air = VT(1), int lmax = 0, int csweeps = 0, int block_min = 15,
                                         int l0 = 1) {
  const int L = (lmax > 0 && lmax < mg.nlev) ? lmax : mg.nlev;
  auto is_block = [&](int l) { return NT == 64 || mg.lv[l].n >= block_min; };
  auto bsync = [] { __syncthreads(); };
  int lb = l0 - 1;  // last block level
  while (lb + 1 <= L && is_block(lb + 1)) ++lb;
  const VT* zL = nullptr;
  // block levels: descent
  for (int l = l0; l <= lb && l < L; ++l) {
    const CLev<VT> F = clev<VT>(mg, l, region, ctab, NT, air);
    const CLev<VT> Cc = clev<VT>(mg, l + 1, region, ctab, NT, air);
    c_resid<VT, GM>(F, tid, NT);
    __syncthreads();
    c_restrict<VT, GM>(F, Cc, om, l + 1 == L, tid, NT);
    __syncthreads();
  }
  if (lb == L) zL = c_coarsest<VT, GM>(clev<VT>(mg, L, region, ctab, NT, air), om, csweeps, tid, NT, bsync);
  // wave levels
  if (lb < L) {
    if (tid < 64) {
      for (int l = lb + 1; l < L; ++l) {
        const CLev<VT> F = clev<VT>(mg, l, region, ctab, 64, air);
        const CLev<VT> Cc = clev<VT>(mg, l + 1, region, ctab, 64, air);
        c_resid<VT, GM>(F, tid, 64);
        wave_sync();
        c_restrict<VT, GM>(F, Cc, om, l + 1 == L, tid, 64);
        wave_sync();
      }
      zL = c_coarsest<VT, GM>(clev<VT>(mg, L, region, ctab, 64, air), om, csweeps, tid, 64, wave_sync);
      for (int l = L - 1; l > lb; --l) {
        const CLev<VT> F = clev<VT>(mg, l, region, ctab, 64, air);
        const CLev<VT> Cc = clev<VT>(mg, l + 1, region, ctab, 64, air);
        c_prolong<VT, GM>(F, l + 1 == L ? zL : Cc.T, Cc.np, tid, 64);
        wave_sync();
        c_post<VT, GM>(F, om, tid, 64);
        wave_sync();
      }
    } else {
      // the other waves only need the pointer: the same alternation as wave 0
      CLev<VT> C = clev<VT>(mg, L, region, ctab, 64, air);
      zL = (csweeps & 1) ? C.T : C.Z;
    }
    __syncthreads();
  }
  // block levels: ascent
  for (int l = (lb < L ? lb : L - 1); l >= l0; --l) {
    const CLev<VT> F = clev<VT>(mg, l, region, ctab, NT, air);
    const CLev<VT> Cc = clev<VT>(mg, l + 1, region, ctab, NT, air);
    c_prolong<VT, GM>(F, l + 1 == L ? zL : Cc.T, Cc.np, tid, NT);
    __syncthreads();
    c_post<VT, GM>(F, om, tid, NT);
    __syncthreads();
  }
  return L == l0 ? zL : clev<VT>(mg, l0, region, ctab, NT, air).T;
}

// The same cycle with levels lds_lev..L in LDS (lds_reg: their vectors,
// lds_tab: their tables, in the global layout's order) and levels
// 1..lds_lev-1 in global memory (whole-workgroup levels); returns level 1's
// corrected vector.  Same arithmetic as coarse_cycle.
template <typename VT, int NT>
__device__ __attribute__((always_inline)) inline const VT* coarse_cycle_lds(const MGGeom& mg, VT* region, const VT* ctab,
                                                                          VT* lds_reg, const VT* lds_tab, int lds_lev,
                                                                          VT om, int tid, VT air, int lmax, int csweeps,
                                                                          int block_min) {
  const int L = (lmax > 0 && lmax < mg.nlev) ? lmax : mg.nlev;
  VT* const lreg = lds_reg - mg.lv[lds_lev].vec_off;  // level l's vectors at lreg + vec_off(l)
  const VT* const ltab = lds_tab - mg.lv[lds_lev].tab_off;
  for (int l = 1; l < lds_lev; ++l) {
    const CLev<VT> F = clev<VT>(mg, l, region, ctab, NT, air);
    c_resid<VT, true>(F, tid, NT);
    __syncthreads();
    if (l + 1 < lds_lev) c_restrict<VT, true>(F, clev<VT>(mg, l + 1, region, ctab, NT, air), om, l + 1 == L, tid, NT);
    else c_restrict<VT, true>(F, clev<VT>(mg, l + 1, lreg, ltab, NT, air), om, l + 1 == L, tid, NT);
    __syncthreads();
  }
  const VT* zl = coarse_cycle<VT, NT, false>(mg, lreg, ltab, om, tid, air, lmax, csweeps, block_min, lds_lev);
  __syncthreads();
  for (int l = lds_lev - 1; l >= 1; --l) {
    const CLev<VT> F = clev<VT>(mg, l, region, ctab, NT, air);
    const int cp = mg.lv[l + 1].n + 2;
    if (l + 1 == lds_lev) c_prolong<VT, true>(F, zl, cp, tid, NT);
    else c_prolong<VT, true>(F, clev<VT>(mg, l + 1, region, ctab, NT, air).T, cp, tid, NT);
    __syncthreads();
    c_post<VT, true>(F, om, tid, NT);
    __syncthreads();
  }
  return clev<VT>(mg, 1, region, ctab, NT, air).T;
}

// Galerkin coarse entries A_c(c, c + D) = (P e_c)^T A_f (P e_{c+D}) for
// D in {0, E, N, NE}; `cf(i, j, d)` returns the fine coupling of node (i, j)
// in direction d (0 C, 1 E, 2 W, 3 N, 4 S, 5 NE, 6 SW).
template <class CF>
__device__ inline void galerkin_entries(CF cf, int nf, int nc, int ic, int jc, double out[4]) {
  const int OX[7] = {0, 1, -1, 0, 0, 1, -1};
  const int OY[7] = {0, 0, 0, 1, -1, 1, -1};
  const double PW[7] = {1.0, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5};
  const int DX[4] = {0, 1, 0, 1}, DY[4] = {0, 0, 1, 1};
  for (int q = 0; q < 4; ++q) {
    const int cx = ic + DX[q], cy = jc + DY[q];
    double s = 0.0;
    if (cx < nc && cy < nc) {
      for (int a = 0; a < 7; ++a) {
        const int fi = 2 * ic + 1 + OX[a], fj = 2 * jc + 1 + OY[a];
        if (fi < 0 || fj < 0 || fi >= nf || fj >= nf) continue;
        for (int d = 0; d < 7; ++d) {
          const int gi = fi + OX[d], gj = fj + OY[d];
          if (gi < 0 || gj < 0 || gi >= nf || gj >= nf) continue;
          const int ox = gi - (2 * cx + 1), oy = gj - (2 * cy + 1);
          double w2 = 0.0;
          if (ox == 0 && oy == 0) w2 = 1.0;
          else if ((ox == 1 && oy == 0) || (ox == -1 && oy == 0) || (ox == 0 && oy == 1) ||
                   (ox == 0 && oy == -1) || (ox == 1 && oy == 1) || (ox == -1 && oy == -1))
            w2 = 0.5;
          if (w2 != 0.0) s += PW[a] * cf(fi, fj, d) * w2;
        }
      }
    }
    out[q] = s;
  }
}


// Galerkin coarse operators for levels 1..nlev into ctab (5 planes per level:
// C, E, N, NE, 1/C).  The fine level's couplings are those of the scaled
// system D^{-1/2} A D^{-1/2} (fE, fN, fNE, pitch fpitch, unit diagonal).
// With `unscaled`, level 1 is P^T A P of the unscaled A (fine couplings
// divided by d_i d_j, d = D^{-1/2} from dn(i, j)), i.e. the interpolation from
// level 1 to the scaled fine level is D^{1/2} P: the coarse space then holds
// the smooth functions of A rather than of the scaled system, whose scaling
// jumps across the conductor boundary.  Otherwise it is P^T Ahat P.
template <typename VT, class DN>
__device__ void build_galerkin(const MGGeom& mg, VT* ctab, const VT* tE, const VT* tN, const VT* tNE,
                               DN dn, bool unscaled, double d_air, int fpitch, int tid, int nthr) {
  const double air = unscaled ? 1.0 / (d_air * d_air) : 1.0;  // air diagonal of the coarse levels
  for (int l = 1; l <= mg.nlev; ++l) {
    const MGLevel& M = mg.lv[l];
    const MGLevel& F = mg.lv[l - 1];
    const int pl = M.RW * M.RH;
    VT* C = ctab + M.tab_off;
    VT* E = C + pl;
    VT* Nn = E + pl;
    VT* NE = Nn + pl;
    VT* ID = NE + pl;
    const int fp = l == 1 ? fpitch : F.RW;
    const VT* fC = l == 1 ? nullptr : ctab + F.tab_off;
    const VT* fE = l == 1 ? tE : fC + F.RW * F.RH;
    const VT* fN = l == 1 ? tN : fE + F.RW * F.RH;
    const VT* fNE = l == 1 ? tNE : fN + F.RW * F.RH;
    const double air_below = l == 1 ? 1.0 : air;
    auto cs = [&](int fi, int fj, int d) -> double {  // coupling of the level below
      if (!(fi >= F.bx0 && fi < F.lx1 && fj >= F.by0 && fj < F.ly1)) {
        if (d == 0) return air_below;
        return d <= 4 ? -0.25 * air_below : 0.0;
      }
      const int t = (fj - F.by0 + 1) * fp + (fi - F.bx0 + 1);
      switch (d) {
        case 0: return fC ? (double)fC[t] : 1.0;
        case 1: return (double)fE[t];
        case 2: return (double)fE[t - 1];
        case 3: return (double)fN[t];
        case 4: return (double)fN[t - fp];
        case 5: return (double)fNE[t];
        default: return (double)fNE[t - fp - 1];
      }
    };
    const bool unscale = l == 1 && unscaled;
    auto cf = [&](int fi, int fj, int d) -> double {
      const double c = cs(fi, fj, d);
      if (!unscale) return c;
      const int OXd[7] = {0, 1, -1, 0, 0, 1, -1}, OYd[7] = {0, 0, 0, 1, -1, 1, -1};
      return c / (dn(fi, fj) * dn(fi + OXd[d], fj + OYd[d]));
    };
    for (int t = tid; t < pl; t += nthr) {
      const int i = M.bx0 - 1 + t % M.RW, j = M.by0 - 1 + t / M.RW;
      const bool box = i >= M.bx0 && i < M.bx1 && j >= M.by0 && j < M.by1;
      double o[4] = {air, -0.25 * air, -0.25 * air, 0.0};
      if (box) galerkin_entries(cf, F.n, M.n, i, j, o);
      C[t] = vt<VT>(o[0]);
      E[t] = vt<VT>(o[1]);
      Nn[t] = vt<VT>(o[2]);
      NE[t] = vt<VT>(o[3]);
      ID[t] = vt<VT>(1.0 / o[0]);
    }
    __syncthreads();
  }
}

// LDS pitches are compile-time constants (LP = CW + 2 for the grid, TP for
// the tables) so that every per-node LDS offset folds into the instruction's
// immediate offset instead of occupying a register.
template <typename VT, int CW, int SH, int NS, int TP, bool MG, bool NL, bool PARA>
__global__ __launch_bounds__(CW* NS) void k_ie_resident(Geom g, MGGeom mg, Solver sv,
                                                        const Inst* __restrict__ insts, int n_inst,
                                                        int* counter, double* work,
                                                        const double* __restrict__ S,
                                                        const uint8_t* __restrict__ cond, CellRegion cr) {
  constexpr int NT = CW * NS;
  constexpr int NWAVES = NT / 64;
  constexpr int LP = CW + 2;
  constexpr int CR = SH / 4;  // first-coarse-level rows per thread in the restriction
  extern __shared__ double smem_d[];
  const int n = g.n, RHW = g.RW * g.RH, TRH = g.RH * TP;
  double* red = smem_d;                                  // 2 * NWAVES * 4 doubles
  VT* rl = reinterpret_cast<VT*>(red + 2 * NWAVES * 4);  // (n+2) x LP grid with zero halo
  const int region = MG ? mg.region_elems : (n + 2) * LP; // multigrid: shared with coarse vectors
  VT* tE = rl + region;                                  // scaled tables, RH x TP each
  VT* tN = tE + TRH;
  VT* tNE = tN + TRH;
  VT* ctab = tNE + TRH;                                  // coarse Galerkin tables (multigrid)
  __shared__ int s_inst;
  __shared__ int s_depok;
  __shared__ int s_dmin;  // bits of min_i D_ii^{-1/2} (positive float: int order = float order)

  const int tid = threadIdx.x;
  const int ci = tid % CW;
  // a wave lies in one row slice when CW is a multiple of 64: the slice index is
  // then wave-uniform, and so is every per-row test below (scalar branches)
  const int slice = CW % 64 == 0 ? __builtin_amdgcn_readfirstlane(tid / CW) : tid / CW;
  int j0 = slice * SH;
  const bool colok = ci < n;
  const bool strip_ok = colok && j0 < n;
  const size_t FS = (size_t)g.N * g.P;
  double* Av = work + (size_t)blockIdx.x * ie_work_doubles(g);
  double* Xv = Av + FS;
  double* Bv = Xv + FS;
  const size_t PS = res_plane_doubles(g);   // thread-private planes hold SH * NT <= PS elements
  VT* Yv = reinterpret_cast<VT*>(Bv + FS);   // multigrid CG iterate, thread-private [k][tid] layout
  double* Pv = Bv + FS + PS;                 // previous increment (extrapolated start)
  double* Qv = Pv + FS;                      // Picard: increment of the last fixed-point iterate
  VT* Dv = reinterpret_cast<VT*>(Qv + FS);   // per-node D^{-1/2}, thread-private [k][tid] layout
  double* Tslot = Qv + FS + PS;              // Picard: this instance's FP64 tables (K re-assembled)
  const double d_air = 1.0 / sqrt(4.0 * g.nu_air);
  int slot = 0;

  // node k of this thread is row j0 + k of column ci; indices are affine in k
  const int gi0 = (j0 + 1) * g.P + ci + 1;
  const int t0 = (j0 - g.by0 + 1) * g.RW + (ci - g.bx0 + 1);  // FP64 tables (pitch RW)
  int s0 = (j0 - g.by0 + 1) * TP + (ci - g.bx0 + 1);    // LDS tables (pitch TP)
  int l0 = (j0 + 1) * LP + ci + 1;
  // Called at the top of each inner iteration: the row index and the LDS bases
  // become opaque there, so the per-row tests and offsets derived from them are
  // recomputed in the iteration (a few scalar operations) instead of being kept
  // live across the whole loop, which exhausts the scalar register file.
  auto refresh = [&]() __attribute__((always_inline)) {
    // opaque to the optimiser, and back to a scalar register where the slice
    // is wave-uniform (readfirstlane rather than an "s" asm constraint, which
    // the backend cannot honour once the Parareal entry prologue is present,
    // and which spills more here)
    asm volatile("" : "+v"(j0));
    if constexpr (CW % 64 == 0) j0 = __builtin_amdgcn_readfirstlane(j0);
    asm volatile("" : "+v"(l0), "+v"(s0));
  };
  const bool col_L = ci >= g.bx0 && ci < g.lx1;
  const bool col_box = ci >= g.bx0 && ci < g.bx1;
  auto ACT = [&](int k) { return colok && (j0 + k) < n; };
  auto NREF = [&](int k) {
    NodeRef r;
    const int j = j0 + k;
    r.gi = gi0 + k * g.P;
    r.t = t0 + k * g.RW;
    r.inL = col_L && j >= g.by0 && j < g.ly1;
    return r;
  };
  auto INBOX = [&](int k) {
    const int j = j0 + k;
    return col_box && j >= g.by0 && j < g.by1;
  };

  int q_cur = (int)blockIdx.x < counter[3] ? 0 : 1, q_moved = 0;  // work queue of this workgroup (thread 0)
  for (;;) {
    if (tid == 0) s_inst = queue_next(counter, n_inst, q_cur, q_moved);
    __syncthreads();
    const int id = s_inst;
    __syncthreads();
    if (id >= n_inst) break;
    const Inst in = insts[id];
    const double* tab = in.tab;
    const double inv_dt = 1.0 / in.dt;
    const unsigned long long t_begin = wall_clock64();
    if constexpr (NL) {
      // private copy of the sample's tables; K planes are re-assembled per Picard iteration
      for (int t = tid; t < T_NPLANES * RHW + 3; t += NT) Tslot[t] = in.tab[t];
      __syncthreads();
      tab = Tslot;
    }
    double dmin = 0.0, floor_fac = 0.0;

    // scaled couplings D^{-1/2} A D^{-1/2} over the table region, FP64 -> VT
    auto dscale = [&](int i, int j) -> double {
      if (i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1) {
        const int t = (j - g.by0 + 1) * g.RW + (i - g.bx0 + 1);
        return 1.0 / sqrt(tab[T_MC * RHW + t] * inv_dt + tab[T_KC * RHW + t]);
      }
      return d_air;
    };
    auto build_tables = [&]() {
    if (tid == 0) s_dmin = __float_as_int((float)d_air);
    __syncthreads();
    for (int t = tid; t < RHW; t += NT) {
      const int i = g.bx0 - 1 + t % g.RW, j = g.by0 - 1 + t / g.RW;
      const bool box = i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1;
      const double di = dscale(i, j);
      if (box) atomicMin(&s_dmin, __float_as_int((float)di));
      double e = -0.25, nn = -0.25, ne = 0.0;
      if (box) {
        e = (tab[T_ME * RHW + t] * inv_dt + tab[T_KE * RHW + t]) * di * dscale(i + 1, j);
        nn = (tab[T_MN * RHW + t] * inv_dt + tab[T_KN * RHW + t]) * di * dscale(i, j + 1);
        ne = tab[T_MNE * RHW + t] * inv_dt * di * dscale(i + 1, j + 1);
      }
      const int ts = (t / g.RW) * TP + t % g.RW;
      tE[ts] = vt<VT>(e);
      tN[ts] = vt<VT>(nn);
      tNE[ts] = vt<VT>(ne);
    }
    __syncthreads();
    // inner solves stop once the scaled residual guarantees the outer test:
    // ||b - A x|| <= D_max^{1/2} ||r_scaled|| (half the outer tolerance)
    // (mixed precision only: FP64 inner solves run to inner_rtol, which keeps the
    // FP64 path well below its outer tolerance)
    dmin = (double)__int_as_float(s_dmin) * 0.999;
    floor_fac = sizeof(VT) == 4 ? 0.25 * sv.tol * sv.tol * dmin * dmin : 0.0;
    if constexpr (MG) {
      // Galerkin hierarchy of the scaled system: the D^{1/2} P transfers of the
      // streaming path need D per node inside the V-cycle, which costs more
      // here (registers, global loads) than the ~5% of iterations it saves
      auto dnf = [&](int i, int j) -> double { return (double)vt<VT>(dscale(i, j)); };
      build_galerkin<VT>(mg, ctab, tE, tN, tNE, dnf, false, d_air, TP, tid, NT);
    }
    };
    // a later piece of an instance: wait (bounded) until the previous piece has
    // published its state; the work queue hands out a piece only after its
    // predecessor, so the wait ends
    int dep_flags = 0;
    if (in.dep_wait) {
      if (tid == 0) {
        const unsigned long long tw = wall_clock64();
        int ok = 1;
        const unsigned long long lim = PARA ? PARA_WAIT_TICKS : DEP_WAIT_TICKS;
        int* abort = nullptr;
        if constexpr (PARA) abort = in.para ? in.para->abort : nullptr;
        while (__hip_atomic_load(in.dep_wait, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
          if (wall_clock64() - tw > lim ||
              (abort && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            ok = 0;
            if (abort) __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(8);
        }
        s_depok = ok;
      }
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (!s_depok) dep_flags = FLAG_FAILED;
      __syncthreads();
    }
    // Parareal entry of a one-launch run: skip (sample stopped, or stopped by
    // this chain's jumps) or run; a continuing chain has written U_j
    // (the branch is made wave-uniform: it leaves the entry as a whole)
    if constexpr (PARA) {
      if (__builtin_amdgcn_readfirstlane(para_prologue<NT, NWAVES>(g, in, red, slot, &s_depok, &dep_flags) ? 1 : 0)) {
        if (tid == 0 && in.stat) {
          in.stat[3] = dep_flags;
          in.stat[4] = in.stat[6] = (int)(t_begin & 0xffffffffull);
          in.stat[5] = in.stat[7] = (int)(t_begin >> 32);
        }
        if (in.dep_done) para_set(in.dep_done);
        __syncthreads();
        continue;
      }
    }
    for (int t = tid; t < (n + 2) * LP; t += NT) rl[t] = VT(0);
#pragma unroll 1
    for (int k = 0; k < SH; ++k) {
      if (ACT(k)) {
        const int gi = gi0 + k * g.P;
        Av[gi] = in.a_init ? in.a_init[gi] : 0.0;
        Xv[gi] = in.carry_in ? in.carry[gi] : 0.0;
        Pv[gi] = in.carry_in ? in.carry[FS + gi] : 0.0;
        Qv[gi] = 0.0;
      }
    }
    __syncthreads();
    // Picard: K(nu(|grad a|^2)) on the box from the state a_k + Q (FP64)
    auto assemble_K = [&]() {
      const double* kp = in.tab + T_NPLANES * RHW;  // k1', k2', k3' of the sample
      const double k1 = kp[0], k2 = kp[1], k3 = kp[2], hinv2 = 1.0 / g.h2;
      auto st_at = [&](int I, int J) -> double {  // full-grid node value of a_k + Q
        const int q = J * g.P + I;
        return Av[q] + Qv[q];
      };
      auto nu_el = [&](int ci_, int cj_, int tt) -> double {
        const int e = ((cj_ - cr.cy0) * cr.cw + (ci_ - cr.cx0)) * 2 + tt;
        if (!cond[e]) return g.nu_air;
        double gx, gy;
        if (tt == 0) {
          gx = st_at(ci_ + 1, cj_) - st_at(ci_, cj_);
          gy = st_at(ci_ + 1, cj_ + 1) - st_at(ci_ + 1, cj_);
        } else {
          gx = st_at(ci_ + 1, cj_ + 1) - st_at(ci_, cj_ + 1);
          gy = st_at(ci_, cj_ + 1) - st_at(ci_, cj_);
        }
        return k1 * exp(k2 * (gx * gx + gy * gy) * hinv2) + k3;
      };
      double* T = Tslot;
      for (int t = tid; t < RHW; t += NT) {
        const int i = g.bx0 - 1 + t % g.RW, j = g.by0 - 1 + t / g.RW;
        if (!(i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1)) continue;
        const int I = i + 1, J = j + 1;
        const double na0 = nu_el(I, J, 0), na1 = nu_el(I, J, 1), nb0 = nu_el(I - 1, J, 0);
        const double nc1 = nu_el(I, J - 1, 1), nd0 = nu_el(I - 1, J - 1, 0), nd1 = nu_el(I - 1, J - 1, 1);
        T[T_KC * RHW + t] = 0.5 * (na0 + na1 + nd0 + nd1) + nb0 + nc1;
        T[T_KE * RHW + t] = -0.5 * (na0 + nc1);
        T[T_KN * RHW + t] = -0.5 * (na1 + nb0);
      }
      __syncthreads();
    };
    // per-node D^{-1/2} (box: from the FP64 tables; elsewhere the air value),
    // rounded to VT like the scaled system it multiplies; computed once per
    // table build into the thread's own entries of Dv
    auto fill_dn = [&]() {
#pragma unroll 1
      for (int k = 0; k < SH; ++k) {
        if (!ACT(k)) continue;
        VT d = vt<VT>(d_air);
        if (INBOX(k)) {
          const int t = t0 + k * g.RW;
          d = vt<VT>(1.0 / sqrt(tab[T_MC * RHW + t] * inv_dt + tab[T_KC * RHW + t]));
        }
        Dv[k * NT + tid] = d;
      }
    };
    if constexpr (!NL) {
      build_tables();
      fill_dn();
    }
    auto DN = [&](int k) -> double { return (double)Dv[k * NT + tid]; };

    double qsum = in.carry_in ? in.carry[2 * FS] : 0.0;
    int it_total = 0, sw_total = 0, it_max_step = 0, flags = dep_flags, pic_total = 0;
    // per-phase device wall-clock ticks (thread 0): fine V-cycle descent,
    // coarse levels, fine ascent, CG apply + reductions; right-hand side,
    // refinement residuals, increment updates, QoI + state update
    unsigned long long ph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    unsigned long long tmark = 0;
    auto tick = [&](int q) __attribute__((always_inline)) {
      if (tid == 0) {
        const unsigned long long t = wall_clock64();
        if (q >= 0) ph[q] += t - tmark;
        tmark = t;
      }
    };
    const int n_seg = in.n_chain > 0 ? in.n_chain : 1;
    for (int seg = 0; seg < n_seg; ++seg) {
      const int kseg0 = in.k0 + seg * in.n_steps;
      for (int step = 0; step < in.n_steps; ++step) {
        const double Jt = in.src[kseg0 + step + 1];
        int pic_it = 0;
        for (;;) {  // Picard iterations (a single pass for linear materials)
        tick(-1);
        if constexpr (NL) {
          assemble_K();
          build_tables();
          fill_dn();
        }
        // b = J(t_{k+1}) S - K a and ||b||^2
        double part[1] = {0.0};
#pragma unroll 1
        for (int k = 0; k < SH; ++k) {
          if (ACT(k)) {
            const NodeRef nr = NREF(k);
            const double b = Jt * S[nr.gi] - K_apply_u(g, tab, Av, nr);
            Bv[nr.gi] = b;
            part[0] += b * b;
          }
        }
        block_sum<1, NWAVES>(part, red, slot);
        tick(4);
        const double bb = part[0];
        int it_step = 0;
        if (bb == 0.0) {
#pragma unroll 1
          for (int k = 0; k < SH; ++k)
            if (ACT(k)) Xv[gi0 + k * g.P] = 0.0;
          __syncthreads();
        } else {
          bool conv = false;
          for (int sweep = 0; sweep <= sv.max_sweeps; ++sweep) {
            // FP64 residual of the current increment; its scaled copy goes to LDS
            tick(-1);
            double rr[1] = {0.0};
#pragma unroll 1
            for (int k = 0; k < SH; ++k) {
              if (ACT(k)) {
                const NodeRef nr = NREF(k);
                const double res = Bv[nr.gi] - A_apply_u(g, tab, Xv, nr, inv_dt);
                rr[0] += res * res;
                rl[l0 + k * LP] = vt<VT>(res * DN(k));
              }
            }
            block_sum<1, NWAVES>(rr, red, slot);  // barrier: LDS residual complete
            tick(5);
            if (!(rr[0] == rr[0]) || isinf(rr[0])) {
              flags |= FLAG_FAILED;
              break;
            }
            if (rr[0] <= sv.tol * sv.tol * bb) {
              conv = true;
              break;
            }
            if (sweep == sv.max_sweeps) break;
            sw_total++;
            if constexpr (MG) {
              // ---- CG preconditioned by a geometric multigrid V(1,1)-cycle ----
              // (standard PCG ordering; registers y, r, p and one of q / t / z)
              const VT om = vt<VT>(sv.mg_omega);
              auto publish = [&](const VT(&v)[SH]) __attribute__((always_inline)) {
#pragma unroll
                for (int k = 0; k < SH; ++k)
                  if (ACT(k)) rl[l0 + k * LP] = v[k];
              };
              // w = A v on the fine level (v published in the LDS grid)
              auto fine_apply = [&](const VT(&v)[SH], VT(&w)[SH]) __attribute__((always_inline)) {
                if (!strip_ok) {
#pragma unroll
                  for (int k = 0; k < SH; ++k) w[k] = VT(0);
                  return;
                }
                VT lprev = rl[l0 - LP - 1];
                VT rcur = rl[l0 + 1];
                const VT below = rl[l0 - LP];
#pragma unroll
                for (int k = 0; k < SH; ++k) {
                  const int j = j0 + k;
                  if (j < n) {
                    const VT lcur = rl[l0 + k * LP - 1];
                    const VT rnxt = rl[l0 + (k + 1) * LP + 1];
                    const VT up = (k + 1 < SH) ? v[(k + 1 < SH) ? k + 1 : k] : rl[l0 + (k + 1) * LP];
                    const VT dnv = (k > 0) ? v[(k > 0) ? k - 1 : 0] : below;
                    if (col_L && j >= g.by0 && j < g.ly1) {
                      const int t = s0 + k * TP;
                      w[k] = v[k] + tE[t] * rcur + tE[t - 1] * lcur + tN[t] * up + tN[t - TP] * dnv +
                             tNE[t] * rnxt + tNE[t - TP - 1] * lprev;
                    } else {
                      w[k] = v[k] - VT(0.25) * ((rcur + lcur) + (up + dnv));
                    }
                    lprev = lcur;
                    rcur = rnxt;
                  } else {
                    w[k] = VT(0);
                  }
                  __builtin_amdgcn_sched_barrier(0);
                }
              };
              // post-smoothing z <- z + om (r - A z) in place (old z kept for the stencil)
              auto fine_smooth = [&](VT(&v)[SH], const VT(&rr_)[SH]) __attribute__((always_inline)) {
                if (!strip_ok) return;
                VT lprev = rl[l0 - LP - 1];
                VT rcur = rl[l0 + 1];
                VT dnv = rl[l0 - LP];
#pragma unroll
                for (int k = 0; k < SH; ++k) {
                  const int j = j0 + k;
                  if (j < n) {
                    const VT lcur = rl[l0 + k * LP - 1];
                    const VT rnxt = rl[l0 + (k + 1) * LP + 1];
                    const VT up = (k + 1 < SH) ? v[(k + 1 < SH) ? k + 1 : k] : rl[l0 + (k + 1) * LP];
                    const VT c = v[k];
                    VT w;
                    if (col_L && j >= g.by0 && j < g.ly1) {
                      const int t = s0 + k * TP;
                      w = c + tE[t] * rcur + tE[t - 1] * lcur + tN[t] * up + tN[t - TP] * dnv +
                          tNE[t] * rnxt + tNE[t - TP - 1] * lprev;
                    } else {
                      w = c - VT(0.25) * ((rcur + lcur) + (up + dnv));
                    }
                    v[k] = c + om * (rr_[k] - w);
                    dnv = c;
                    lprev = lcur;
                    rcur = rnxt;
                  }
                  __builtin_amdgcn_sched_barrier(0);
                }
              };
              // z = B r (symmetric V(1,1) cycle)
              auto vcycle = [&](const VT(&rv)[SH], VT(&zv)[SH]) __attribute__((always_inline)) {
                tick(-1);
                publish(rv);
                __syncthreads();
                fine_apply(rv, zv);  // zv used as scratch: A r
#pragma unroll
                for (int k = 0; k < SH; ++k) zv[k] = rv[k] - om * zv[k];  // t = r - A (om r)
                __syncthreads();
                publish(zv);
                __syncthreads();
                // restriction to level 1 (registers), then R_1, Z_1 into the shared region
                const CLev<VT> L1 = clev<VT>(mg, 1, rl, ctab, NT);
                const int n1 = L1.n;
                const int tx1 = tid & ((1 << L1.txs) - 1), ty1 = NT >> L1.txs, jb1 = tid >> L1.txs;
                VT rc[CR];
#pragma unroll
                for (int m = 0; m < CR; ++m) {
                  const int j = jb1 + m * ty1;
                  rc[m] = (tx1 < n1 && j < n1) ? restrict_at(rl, LP, tx1, j) : VT(0);
                  __builtin_amdgcn_sched_barrier(0);
                }
                __syncthreads();
                for (int l = 1; l <= mg.nlev; ++l) c_zero_halo(clev<VT>(mg, l, rl, ctab, NT), tid, NT);
                const bool exact1 = mg.nlev == 1 || sv.mg_levels == 1;
#pragma unroll
                for (int m = 0; m < CR; ++m) {
                  const int j = jb1 + m * ty1;
                  if (tx1 < n1 && j < n1) {
                    const int q = (j + 1) * L1.np + tx1 + 1;
                    L1.R[q] = rc[m];
                    L1.Z[q] = (exact1 ? VT(1) : om) * clev_id(L1, tx1, j) * rc[m];
                  }
                }
                __syncthreads();
                tick(0);
                const VT* z1 = coarse_cycle<VT, NT>(mg, rl, ctab, om, tid, VT(1), sv.mg_levels, sv.mg_coarse_sweeps,
                                                    sv.mg_block_min);
                tick(1);
#pragma unroll
                for (int k = 0; k < SH; ++k) {
                  zv[k] = ACT(k) ? om * rv[k] + prolong_at(z1, L1.np, ci, j0 + k) : VT(0);
                  __builtin_amdgcn_sched_barrier(0);
                }
                __syncthreads();
                publish(zv);
                // restore the zero halo of the fine grid (the region held coarse data)
                for (int q = tid; q < 2 * LP + 2 * n; q += NT) {
                  int idx;
                  if (q < LP) idx = q;
                  else if (q < 2 * LP) idx = (n + 1) * LP + (q - LP);
                  else if (q < 2 * LP + n) idx = (q - 2 * LP + 1) * LP;
                  else idx = (q - 2 * LP - n + 1) * LP + n + 1;
                  rl[idx] = VT(0);
                }
                __syncthreads();
                fine_smooth(zv, rv);
                tick(2);
              };

              // the iterate y is accumulated in the slot's global VT buffer
              // (owner-thread access only) to keep three vectors in registers
              VT r[SH], p[SH], z[SH];
#pragma unroll
              for (int k = 0; k < SH; ++k) {
                r[k] = ACT(k) ? rl[l0 + k * LP] : VT(0);
                p[k] = VT(0);
                if (ACT(k)) Yv[k * NT + tid] = VT(0);
              }
              double rho = 1.0, stop = 0.0;
              int it = 0;
              for (;;) {
                refresh();
                vcycle(r, z);
                double rz[2];
                {
                  VT a = VT(0), b = VT(0);
#pragma unroll
                  for (int k = 0; k < SH; ++k) {
                    a += r[k] * z[k];
                    b += r[k] * r[k];
                  }
                  rz[0] = (double)a;
                  rz[1] = (double)b;
                }
                block_sum<2, NWAVES>(rz, red, slot);
                double beta = 0.0;
                if (it == 0) {
                  stop = fmax(sv.inner_rtol * sv.inner_rtol * rz[1], floor_fac * bb);
                  if (!(rz[1] > 0.0) || !(rz[0] > 0.0)) break;
                } else {
                  if (rz[1] <= stop || !(rz[1] == rz[1])) break;
                  beta = rz[0] / rho;
                }
                rho = rz[0];
                const VT b_ = vt<VT>(beta);
#pragma unroll
                for (int k = 0; k < SH; ++k) p[k] = z[k] + b_ * p[k];
                if (it == sv.max_iter) break;
                ++it;
                tick(-1);
                publish(p);
                __syncthreads();
                fine_apply(p, z);  // z holds q = A p here
                double pq[1];
                {
                  VT a = VT(0);
#pragma unroll
                  for (int k = 0; k < SH; ++k) a += p[k] * z[k];
                  pq[0] = (double)a;
                }
                block_sum<1, NWAVES>(pq, red, slot);
                const VT a_ = vt<VT>(rho / pq[0]);
#pragma unroll
                for (int k = 0; k < SH; ++k) {
                  if (ACT(k)) Yv[k * NT + tid] += a_ * p[k];
                  r[k] = r[k] - a_ * z[k];
                }
                tick(3);
              }
              it_step += it;
#pragma unroll
              for (int k = 0; k < SH; ++k)
                if (ACT(k)) rl[l0 + k * LP] = Yv[k * NT + tid];
            } else {
            // ---- inner CG on the scaled system, y0 = 0, r0 = g ----
            // Chronopoulos-Gear ordering: the reduction of r.r shares its
            // barrier with the LDS publication of r, the stencil result w is
            // folded into p, s and r.w at once, so y, r, p, s are the only
            // per-node registers and each iteration has two barriers.
            VT y[SH], r[SH], p[SH], s[SH];
#pragma unroll
            for (int k = 0; k < SH; ++k) {
              r[k] = ACT(k) ? rl[l0 + k * LP] : VT(0);
              y[k] = VT(0);
              p[k] = VT(0);
              s[k] = VT(0);
            }
            double gam_prev = 1.0, alpha = 1.0, stop = 0.0;
            int it = 0;
            for (;; ++it) {
              refresh();
              double gv[1];
              {
                VT pg = VT(0);
#pragma unroll
                for (int k = 0; k < SH; ++k) {
                  if (ACT(k)) rl[l0 + k * LP] = r[k];
                  pg += r[k] * r[k];
                }
                gv[0] = (double)pg;
              }
              block_sum<1, NWAVES>(gv, red, slot);  // also publishes r in LDS
              const double gam = gv[0];
              if (it == 0) {
                stop = fmax(sv.inner_rtol * sv.inner_rtol * gam, floor_fac * bb);
                if (!(gam > 0.0)) break;
              } else if (gam <= stop || !(gam == gam)) {
                break;
              }
              if (it == sv.max_iter) break;
              const double beta = it == 0 ? 0.0 : gam / gam_prev;
              const VT b_ = vt<VT>(beta);
              VT pd = VT(0);
              if (strip_ok) {
                VT lprev = rl[l0 - LP - 1];    // (i-1, j0-1)
                VT rcur = rl[l0 + 1];          // (i+1, j0)
                const VT below = rl[l0 - LP];  // (i, j0-1)
#pragma unroll
                for (int k = 0; k < SH; ++k) {
                  const int j = j0 + k;
                  if (j < n) {
                    const VT lcur = rl[l0 + k * LP - 1];        // (i-1, j)
                    const VT rnxt = rl[l0 + (k + 1) * LP + 1];  // (i+1, j+1)
                    const VT up = (k + 1 < SH) ? r[(k + 1 < SH) ? k + 1 : k] : rl[l0 + (k + 1) * LP];
                    const VT dnv = (k > 0) ? r[(k > 0) ? k - 1 : 0] : below;
                    VT w;
                    if (col_L && j >= g.by0 && j < g.ly1) {
                      const int t = s0 + k * TP;
                      w = r[k] + tE[t] * rcur + tE[t - 1] * lcur + tN[t] * up + tN[t - TP] * dnv +
                          tNE[t] * rnxt + tNE[t - TP - 1] * lprev;
                    } else {
                      w = r[k] - VT(0.25) * ((rcur + lcur) + (up + dnv));
                    }
                    p[k] = r[k] + b_ * p[k];
                    s[k] = w + b_ * s[k];
                    pd += w * r[k];
                    lprev = lcur;
                    rcur = rnxt;
                  }
                  // keep the scheduler from hoisting every node's LDS loads
                  // to the top (register pressure at 1024 threads)
                  __builtin_amdgcn_sched_barrier(0);
                }
              }
              double dv[1] = {(double)pd};
              block_sum<1, NWAVES>(dv, red, slot);
              alpha = it == 0 ? gam / dv[0] : gam / (dv[0] - beta * gam / alpha);
              gam_prev = gam;
              const VT a_ = vt<VT>(alpha);
#pragma unroll
              for (int k = 0; k < SH; ++k) {
                y[k] = y[k] + a_ * p[k];
                r[k] = r[k] - a_ * s[k];
              }
            }
            it_step += it;
            // stage y in the thread's own LDS cells (read back by the same
            // thread only), then x += D^{-1/2} y in FP64
#pragma unroll
            for (int k = 0; k < SH; ++k)
              if (ACT(k)) rl[l0 + k * LP] = y[k];
            }
            tick(-1);
#pragma unroll 1
            for (int k = 0; k < SH; ++k)
              if (ACT(k)) Xv[gi0 + k * g.P] += DN(k) * (double)rl[l0 + k * LP];
            __syncthreads();
            tick(6);
          }
          if (!conv) flags |= FLAG_NOT_CONVERGED;
        }
        it_total += it_step;
        it_max_step = it_step > it_max_step ? it_step : it_max_step;
        if constexpr (!NL) break;
        // fixed-point test ||a^(i+1) - a^(i)|| <= tol ||a^(i+1)|| with a^(i) = a_k + Q
        double dn2[2] = {0.0, 0.0};
#pragma unroll 1
        for (int k = 0; k < SH; ++k) {
          if (ACT(k)) {
            const int gi = gi0 + k * g.P;
            const double x = Xv[gi], dq = x - Qv[gi], an = Av[gi] + x;
            dn2[0] += dq * dq;
            dn2[1] += an * an;
            Qv[gi] = x;
          }
        }
        block_sum<2, NWAVES>(dn2, red, slot);
        ++pic_it;
        if (dn2[0] <= sv.picard_tol * sv.picard_tol * dn2[1]) break;
        if (pic_it >= sv.picard_max) {
          flags |= FLAG_PICARD_CAP;
          break;
        }
        }
        pic_total += pic_it;
        // Joule-loss term d^T M d / dt and the state update a += d
        tick(-1);
        double qq[1] = {0.0};
#pragma unroll 1
        for (int k = 0; k < SH; ++k) {
          const NodeRef nr = NREF(k);
          if (ACT(k) && nr.inL) qq[0] += Xv[nr.gi] * M_apply_u(g, tab, Xv, nr);
        }
        block_sum<1, NWAVES>(qq, red, slot);
        qsum += qq[0] * inv_dt;
#pragma unroll 4
        for (int k = 0; k < SH; ++k) {
          if (ACT(k)) {
            // a += d; next start 2 d_k - d_{k-1} (linear extrapolation)
            const int gi = gi0 + k * g.P;
            const double d = Xv[gi];
            Av[gi] += d;
            Xv[gi] = 2.0 * d - Pv[gi];
            Pv[gi] = d;
            if constexpr (NL) Qv[gi] = 0.0;  // (linear: never written, zero from the start)
          }
        }
        __syncthreads();
        tick(7);
      }
      if (in.n_chain > 0) {
        // Parareal coarse chain: A holds C(U_{n-1}); U_n = F_n + (C_new - C_old_n)
        const double* Fn = in.chain_f[seg];
        double* Cn = in.chain_c[seg];
        double* Un = in.chain_u[seg];
#pragma unroll 1
        for (int k = 0; k < SH; ++k) {
          if (ACT(k)) {
            const int gi = gi0 + k * g.P;
            const double cn = Av[gi];
            const double u = Fn ? Fn[gi] + (cn - Cn[gi]) : cn;
            Cn[gi] = cn;
            Un[gi] = u;
            Av[gi] = u;
          }
        }
        __syncthreads();
        if constexpr (PARA)
          if (in.seg_done) para_set(in.seg_done[seg]);
      }
    }
    if (in.a_out) {
#pragma unroll 1
      for (int k = 0; k < SH; ++k)
        if (ACT(k)) in.a_out[gi0 + k * g.P] = Av[gi0 + k * g.P];
    }
    if (in.carry) {
#pragma unroll 1
      for (int k = 0; k < SH; ++k) {
        if (ACT(k)) {
          const int gi = gi0 + k * g.P;
          in.carry[gi] = Xv[gi];
          in.carry[FS + gi] = Pv[gi];
        }
      }
      if (tid == 0) in.carry[2 * FS] = qsum;
    }
    if (in.dep_done) {
      // publish a_out and carry to the next piece (it may run on another XCD)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (tid == 0) __hip_atomic_store(in.dep_done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == 0) {
      if (in.q_out) *in.q_out = qsum * in.q_scale;
      if (in.stat) {
        const unsigned long long t_end = wall_clock64();
        in.stat[0] = it_total;
        in.stat[1] = sw_total;
        in.stat[2] = it_max_step;
        in.stat[3] = flags;
        in.stat[4] = (int)(t_begin & 0xffffffffull);
        in.stat[5] = (int)(t_begin >> 32);
        in.stat[6] = (int)(t_end & 0xffffffffull);
        in.stat[7] = (int)(t_end >> 32);
        for (int q = 0; q < 8; ++q) in.stat[8 + q] = (int)(ph[q] >> 4);  // units of 16 ticks
        in.stat[16] = pic_total;
      }
      publish_done(in.host_done, qsum * in.q_scale, flags);
    }
    __syncthreads();
  }
}

template <typename VT>
static size_t resident_lds(const Geom& g, const ResCfg& c, const MGGeom* mg) {
  const int nw = c.cw * c.ns / 64;
  size_t region = (size_t)(g.n + 2) * (c.cw + 2), ctab = 0;
  if (mg && mg->nlev > 0) {
    region = mg->region_elems;
    ctab = mg->ctab_elems;
  }
  return 2 * nw * 4 * sizeof(double) + (region + 3 * (size_t)g.RH * c.tp + ctab) * sizeof(VT);
}

// Resident tile: CW columns (one per thread of a slice), NS slices of SH rows.
// tile 1: 16 rows per thread; tile 2 (meshes of 64..127 interior nodes per
// side): 32 rows per thread in 512-thread workgroups, which leaves 256
// registers per lane instead of 128.

int stream_threads(int tile);

int ie_block_threads(const Geom& g, int path, int tile) {
  if (path == MQ_PATH_WIDE) return 256;
  ResCfg c;
  if (path == MQ_PATH_RESIDENT && pick_resident(g, tile, &c)) return c.cw * c.ns;
  return stream_threads(tile);
}

int resident_lp(const Geom& g, int tile) {
  ResCfg c;
  if (!pick_resident(g, tile, &c)) return 0;
  return c.cw + 2;
}

int resident_supported(const Geom& g, const MGGeom* mg, int precision, int lds_limit, int* lds_bytes, int tile) {
  ResCfg c;
  if (!pick_resident(g, tile, &c)) return 0;
  // 1024-thread FP64 workgroups would need more than 128 VGPRs per lane
  if (precision == MQ_PREC_FP64 && c.cw * c.ns > 256) return 0;
  // the restriction to the first coarse level keeps SH/4 coarse rows per thread
  if (mg && mg->nlev > 0) {
    int tx = 1;
    while (tx < mg->lv[1].n && 2 * tx <= c.cw * c.ns) tx *= 2;
    const int ty = c.cw * c.ns / tx;
    if ((mg->lv[1].n + ty - 1) / ty > c.sh / 4) return 0;
  }
  size_t b = precision == MQ_PREC_FP64 ? resident_lds<double>(g, c, mg) : resident_lds<float>(g, c, mg);
  if (lds_bytes) *lds_bytes = (int)b;
  return b <= (size_t)lds_limit ? 1 : 0;
}

template <typename VT, int CW, int SH, int NS, int TP, bool MG, bool NL, bool PARA>
static hipError_t launch_res(const Geom& g, const MGGeom& mg, const Solver& sv, const Inst* insts,
                             int n_inst, int* counter, double* work, int max_grid, const double* S,
                             const uint8_t* cond, const CellRegion& cr,
                             int* grid_out, int* block_out, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  constexpr int NT = CW * NS;
  // the thread-private [row][thread] planes of the work slot must hold SH * NT elements
  if ((size_t)SH * NT > res_plane_doubles(g)) return hipErrorInvalidValue;
  const size_t lds = resident_lds<VT>(g, ResCfg{CW, SH, NS, TP}, MG ? &mg : nullptr);
  auto kern = k_ie_resident<VT, CW, SH, NS, TP, MG, NL, PARA>;
  hipError_t e0 = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e0 != hipSuccess) return e0;
  const int grid = max_grid < n_inst ? max_grid : n_inst;
  if (grid_out) *grid_out = grid;
  if (block_out) *block_out = NT;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), lds, st, g, mg, sv, insts, n_inst, counter, work, S,
                     cond, cr);
  return hipGetLastError();
}

template <typename VT, bool MG, bool NL>
static hipError_t dispatch_res(const Geom& g, const MGGeom& mg, const Solver& sv, const Inst* insts,
                               int n_inst, int* counter, double* work, int max_grid, const double* S,
                               const uint8_t* cond, const CellRegion& cr,
                               int* grid_out, int* block_out, hipStream_t st) {
  ResCfg c;
  if (!pick_resident(g, sv.tile, &c)) return hipErrorInvalidValue;
  if (sv.para) {  // Parareal entries (linear materials only)
    if constexpr (NL) {
      return hipErrorInvalidValue;
    } else {
#define MQ_RES(CW_, SH_, NS_, TP_) \
  launch_res<VT, CW_, SH_, NS_, TP_, MG, NL, true>(g, mg, sv, insts, n_inst, counter, work, max_grid, S, cond, cr, grid_out, block_out, st)
      if (c.cw == 32) return MQ_RES(32, 16, 2, 32);
      if (c.cw == 64) return MQ_RES(64, 16, 4, 64);
      if (c.sh == 32) return MQ_RES(128, 32, 4, 64);
      return MQ_RES(128, 16, 8, 64);
#undef MQ_RES
    }
  }
  if (c.cw == 32) return launch_res<VT, 32, 16, 2, 32, MG, NL, false>(g, mg, sv, insts, n_inst, counter, work, max_grid, S, cond, cr, grid_out, block_out, st);
  if (c.cw == 64) return launch_res<VT, 64, 16, 4, 64, MG, NL, false>(g, mg, sv, insts, n_inst, counter, work, max_grid, S, cond, cr, grid_out, block_out, st);
  if (c.sh == 32) return launch_res<VT, 128, 32, 4, 64, MG, NL, false>(g, mg, sv, insts, n_inst, counter, work, max_grid, S, cond, cr, grid_out, block_out, st);
  return launch_res<VT, 128, 16, 8, 64, MG, NL, false>(g, mg, sv, insts, n_inst, counter, work, max_grid, S, cond, cr, grid_out, block_out, st);
}

template <typename VT, bool MG>
static int occupancy_res(const Geom& g, const MGGeom* mg, const ResCfg& c) {
  int nb = 0;
  const int nt = c.cw * c.ns;
  const size_t lds = resident_lds<VT>(g, c, MG ? mg : nullptr);
  hipError_t e;
  if (c.cw == 32) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ie_resident<VT, 32, 16, 2, 32, MG, false, false>, nt, lds);
  else if (c.cw == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ie_resident<VT, 64, 16, 4, 64, MG, false, false>, nt, lds);
  else if (c.sh == 32) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ie_resident<VT, 128, 32, 4, 64, MG, false, false>, nt, lds);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ie_resident<VT, 128, 16, 8, 64, MG, false, false>, nt, lds);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

int ie_slots_per_cu(const Geom& g, const MGGeom* mg, int path, int precision, int tile) {
  ResCfg c;
  if (path == MQ_PATH_RESIDENT && pick_resident(g, tile, &c)) {
    const bool usemg = mg && mg->nlev > 0;
    if (precision == MQ_PREC_FP64)
      return usemg ? occupancy_res<double, true>(g, mg, c) : occupancy_res<double, false>(g, mg, c);
    return usemg ? occupancy_res<float, true>(g, mg, c) : occupancy_res<float, false>(g, mg, c);
  }
  return tile == 2 ? 2 : 1;  // streaming: one 1024-thread or two 512-thread workgroups per CU
}

hipError_t launch_ie_stream(const Geom& g, const MGGeom& mg, const Solver& sv, const Inst* insts, int n_inst,
                            int* counter, double* work, int n_slots, int max_grid, const double* S,
                            int* grid_out, int* block_out, hipStream_t st);

// n_slots: slots the work buffer was laid out for; max_grid (<= n_slots):
// workgroups to launch.  The multigrid variant runs when mg.nlev > 0 and
// sv.precond == 1.
hipError_t launch_ie(const Geom& g, const MGGeom& mg, const Solver& sv, const Inst* insts, int n_inst,
                     int* counter, double* work, int n_slots, int max_grid, const double* S, int path,
                     int precision, const CellRegion& cr, const uint8_t* cond, const double* nl_params,
                     int* grid_out, int* block_out, hipStream_t st) {
  (void)nl_params;
  if (max_grid > n_slots) max_grid = n_slots;
  if (path == MQ_PATH_RESIDENT) {
    const bool usemg = sv.precond == 1 && mg.nlev > 0;
    const bool nl = sv.nonlinear != 0;
#define MQ_DISPATCH(VT_, MG_, NL_) \
  dispatch_res<VT_, MG_, NL_>(g, mg, sv, insts, n_inst, counter, work, max_grid, S, cond, cr, grid_out, block_out, st)
    if (precision == MQ_PREC_FP64) {
      if (nl) return usemg ? MQ_DISPATCH(double, true, true) : MQ_DISPATCH(double, false, true);
      return usemg ? MQ_DISPATCH(double, true, false) : MQ_DISPATCH(double, false, false);
    }
    if (nl) return usemg ? MQ_DISPATCH(float, true, true) : MQ_DISPATCH(float, false, true);
    return usemg ? MQ_DISPATCH(float, true, false) : MQ_DISPATCH(float, false, false);
#undef MQ_DISPATCH
  }
  return launch_ie_stream(g, mg, sv, insts, n_inst, counter, work, n_slots, max_grid, S, grid_out, block_out, st);
}

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------
__global__ void k_apply(Geom g, int which, double inv_dt, const double* __restrict__ tables, int nsmp,
                        const double* __restrict__ x, double* __restrict__ y, double* scratch) {
  // scratch: full-grid copy of x per sample, boundary zero
  const int nd = g.n * g.n;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int smp = blockIdx.y;
  if (idx >= nd || smp >= nsmp) return;
  const size_t FS = (size_t)g.N * g.P;
  const double* v = scratch + smp * FS;
  const double* tab = tables + (size_t)smp * tab_stride(g);
  const int i = idx % g.n, j = idx / g.n;
  const NodeRef nr = node_ref(g, i, j);
  double out;
  if (which == MQ_APPLY_M) out = M_apply(g, tab, v, nr);
  else if (which == MQ_APPLY_K) out = K_apply(g, tab, v, nr);
  else out = A_apply(g, tab, v, nr, inv_dt);
  y[(size_t)smp * nd + idx] = out;
}

__global__ void k_scatter_full(Geom g, int nsmp, const double* __restrict__ in, double* out) {
  const int nd = g.n * g.n;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int smp = blockIdx.y;
  if (idx >= nd || smp >= nsmp) return;
  const int i = idx % g.n, j = idx / g.n;
  out[(size_t)smp * g.N * g.P + (j + 1) * g.P + i + 1] = in[(size_t)smp * nd + idx];
}

__global__ void k_zero(double* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}
__global__ void k_zero_i(int* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

hipError_t launch_fill_zero(double* p, size_t n, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  if (n == 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}
hipError_t launch_fill_zero_i(int* p, size_t n, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  if (n == 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero_i, dim3(blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_apply(const Geom& g, int which, double dt, const double* tables, int n,
                        const double* x, double* y, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  // x: [n][nd] interior order; builds full-grid copies in y's scratch? Use a temporary.
  const size_t FS = (size_t)g.N * g.P;
  double* scratch = nullptr;
  hipError_t e = hipMallocAsync((void**)&scratch, FS * n * sizeof(double), st);
  if (e != hipSuccess) return e;
  e = launch_fill_zero(scratch, FS * n, st);
  if (e != hipSuccess) return e;
  const int nd = g.n * g.n;
  dim3 grid((nd + 255) / 256, n);
  hipLaunchKernelGGL(k_scatter_full, grid, dim3(256), 0, st, g, n, x, scratch);
  hipLaunchKernelGGL(k_apply, grid, dim3(256), 0, st, g, which, 1.0 / dt, tables, n, x, y, scratch);
  e = hipGetLastError();
  hipError_t e2 = hipFreeAsync(scratch, st);
  return e != hipSuccess ? e : e2;
}

__global__ void k_gather_interior(Geom g, const double* const* full, double* out) {
  const int nd = g.n * g.n;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int smp = blockIdx.y;
  if (idx >= nd) return;
  const int i = idx % g.n, j = idx / g.n;
  out[(size_t)smp * nd + idx] = full[smp][(j + 1) * g.P + i + 1];
}

hipError_t launch_to_interior(const Geom& g, int n, const double* const* full, double* out,
                              hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  const int nd = g.n * g.n;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_interior, dim3((nd + 255) / 256, n), dim3(256), 0, st, g, full, out);
  return hipGetLastError();
}

__global__ void k_scatter_interior(Geom g, const double* in, double* const* full) {
  const int nd = g.n * g.n;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int smp = blockIdx.y;
  if (idx >= nd) return;
  const int i = idx % g.n, j = idx / g.n;
  full[smp][(j + 1) * g.P + i + 1] = in[(size_t)smp * nd + idx];
}

hipError_t launch_to_full(const Geom& g, int n, const double* in, double* const* full, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  const int nd = g.n * g.n;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter_interior, dim3((nd + 255) / 256, n), dim3(256), 0, st, g, in, full);
  return hipGetLastError();
}

// Level statistics of Eq. (9): one workgroup (256 threads) per level; each
// thread sums a contiguous chunk in sample order, chunks are combined by a
// fixed binary tree.  out = {E, Y_0..Y_L, V_0..V_L}; E is summed over levels
// in order by the last block to finish (a second tiny kernel).
__global__ void k_level_stats(const int* nper, const double* const* qf, const double* const* qc,
                              double* out, int n_levels) {
  const int l = blockIdx.x;
  const int N = nper[l];
  const double* f = qf[l];
  const double* c = (l > 0) ? qc[l] : nullptr;
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  const int chunk = (N + 255) / 256;
  const int b = tid * chunk, e = min(N, b + chunk);
  double s = 0.0;
  for (int k = b; k < e; ++k) s += c ? f[k] - c[k] : f[k];
  sh[tid] = s;
  __syncthreads();
  for (int m = 128; m >= 1; m >>= 1) {
    if (tid < m) sh[tid] = sh[tid] + sh[tid + m];
    __syncthreads();
  }
  const double mean = sh[0] / N;
  __syncthreads();
  double v = 0.0;
  for (int k = b; k < e; ++k) {
    const double d = (c ? f[k] - c[k] : f[k]) - mean;
    v += d * d;
  }
  sh[tid] = v;
  __syncthreads();
  for (int m = 128; m >= 1; m >>= 1) {
    if (tid < m) sh[tid] = sh[tid] + sh[tid + m];
    __syncthreads();
  }
  if (tid == 0) {
    out[1 + l] = mean;
    out[1 + n_levels + l] = N > 1 ? sh[0] / (N - 1) : 0.0;
  }
}

__global__ void k_level_total(double* out, int n_levels) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double e = 0.0;
    for (int l = 0; l < n_levels; ++l) e += out[1 + l];
    out[0] = e;
  }
}

hipError_t launch_level_stats(int n_levels, const int* n_per_level, const double* const* qf,
                              const double* const* qc, double* out, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  hipLaunchKernelGGL(k_level_stats, dim3(n_levels), dim3(256), 0, st, n_per_level, qf, qc, out, n_levels);
  hipLaunchKernelGGL(k_level_total, dim3(1), dim3(64), 0, st, out, n_levels);
  return hipGetLastError();
}

// Interface jumps: for pair p, out2[2p] = ||F - U||^2, out2[2p+1] = ||F||^2 over interior nodes.
// Parareal QoI per sample (one-launch run): Q = (sum_n q_n) / T over the M
// slices in slice order, q_n from the slice's latest fine run, iteration
// min(n, K) (FP64).  q: [S][kcap][M].
__global__ void k_para_qoi(const double* __restrict__ qb, const int* __restrict__ K, int kcap, int M, int n_samples,
                           double T, double* __restrict__ q) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_samples) return;
  const int Ks = K[s];
  double acc = 0.0;
  for (int n = 1; n <= M; ++n) {
    const int jj = n < Ks ? n : Ks;
    acc += qb[((size_t)s * kcap + (jj - 1)) * M + (n - 1)];
  }
  q[s] = acc / T;
}

hipError_t launch_para_qoi(const double* qb, const int* K, int kcap, int M, int n_samples, double T, double* q,
                           hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  if (n_samples == 0) return hipSuccess;
  hipLaunchKernelGGL(k_para_qoi, dim3((n_samples + 255) / 256), dim3(256), 0, st, qb, K, kcap, M, n_samples, T, q);
  return hipGetLastError();
}

__global__ void k_check_finite(const double* x, size_t n, int* bad) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(x[i])) atomicOr(bad, 1);
}

hipError_t launch_check_finite(const double* x, size_t n, int* bad, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  if (n == 0) return hipSuccess;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_check_finite, dim3(blocks), dim3(256), 0, st, x, n, bad);
  return hipGetLastError();
}

}  // namespace mq

namespace mq {

// ---------------------------------------------------------------------------
// streaming time-stepping kernel (CG vectors in global memory)
// ---------------------------------------------------------------------------
// Same instance loop and solver as k_ie_resident; each thread walks interior
// nodes idx = tid, tid + NT, ... (row-major, coalesced).  Per slot the VT
// workspace holds R (full grid, zero ring), Y, P, S, W and the scaled tables.
template <typename VT>
__device__ inline VT stencil_scaled(const Geom& g, const VT* __restrict__ R, const VT* tE,
                                    const VT* tN, const VT* tNE, const NodeRef& nr) {
  const int gi = nr.gi, P = g.P;
  const VT c = R[gi], e = R[gi + 1], w = R[gi - 1], nn = R[gi + P], s = R[gi - P];
  if (!nr.inL) return c - VT(0.25) * ((e + w) + (nn + s));
  const int t = nr.t;
  return c + tE[t] * e + tE[t - 1] * w + tN[t] * nn + tN[t - g.RW] * s + tNE[t] * R[gi + P + 1] +
         tNE[t - g.RW - 1] * R[gi - P - 1];
}

// Per-slot VT workspace of the streaming kernel: six full-grid vectors, the
// four quad-table planes, the five table planes over the box region (scaled
// E, N, NE, D^{-1/2}, D^{1/2}) and, with multigrid, the coarse-level vectors
// and Galerkin tables.  (Rounded up to 64 elements: every slot, every
// full-grid vector and every quad plane in it starts 16-byte aligned.)
__host__ __device__ inline size_t stream_slot_elems(const Geom& g, const MGGeom& mg, bool use_mg) {
  const QTab q = qtab_geom(g);
  size_t e = 6 * (size_t)g.N * g.P + 4 * (size_t)q.rows * q.qw + 5 * (size_t)g.RW * g.RH;
  if (use_mg) e += (size_t)mg.region_elems + (size_t)mg.ctab_elems;
  return (e + 63) & ~(size_t)63;
}

// Four consecutive nodes of one row (float4 form of the streaming kernel's
// fine passes, mixed precision).  The full-grid FP32 vectors are addressed 3
// elements past their plane's start there, so that node (i, j) with i = 0 mod
// 4 sits at a 16-byte boundary (needs a pitch P = N + 3, i.e. N = 1 mod 4; the
// last accessed element, the top-right ring node, then stays inside the plane).
typedef float f4v __attribute__((ext_vector_type(4)));
struct F4x2 {
  f4v a, b;
};
__device__ inline f4v ld4(const float* p) { return *reinterpret_cast<const f4v*>(p); }
// store the first nv (1..4) components
__device__ inline void st4(float* p, const f4v& v, int nv) {
  if (nv == 4) {
    *reinterpret_cast<f4v*>(p) = v;
  } else {
    p[0] = v[0];
    if (nv > 1) p[1] = v[1];
    if (nv > 2) p[2] = v[2];
  }
}
// Where a quad's left and right neighbour quads are: quads of one row sit in
// consecutive lanes, so the nodes just across a quad's edges are the
// neighbouring lanes' values, except at the row's ends (the zero boundary
// ring on the left; on the right only the boundary node, never stored, reads
// past it) and where a row continues in the next wave (then loaded).
struct QLane {
  bool lzero, lload, rload;
};
__device__ inline QLane qlane(int qtx, int nq) {
  const int lane = threadIdx.x & 63;
  return QLane{qtx == 0, lane == 0 && qtx > 0, lane == 63 && qtx + 1 < nq};
}
// scaled 7-point stencil of four nodes (i0..i0+3, j) from their rows c (row
// j), up (j + 1), dn (j - 1) and the four values across the quad's edges (w =
// (i0-1, j), e = (i0+4, j), ne = (i0+4, j+1), sw = (i0-1, j-1)): the
// coefficients from the quad tables inside the lookup region (air values
// elsewhere), the W and SW coefficients at the quad's left edge from the
// adjacent lane.  Same expression per node as stencil_scaled inside the
// lookup region.
__device__ inline f4v stencil4_rows(const Geom& g, const QTab& q, const QLane& ql, const f4v& c, const f4v& up,
                                    const f4v& dn, float w, float e, float ne, float sw, const float* qE,
                                    const float* qN, const float* qNE, int i0, int j) {
  const int b = qbase(g, q, i0, j);
  f4v E, N, Nb, NE, NEb;
  if (b >= 0) {
    E = ld4(qE + b);
    N = ld4(qN + b);
    Nb = ld4(qN + b - q.qw);
    NE = ld4(qNE + b);
    NEb = ld4(qNE + b - q.qw);
  } else {
    E = N = Nb = f4v{-0.25f, -0.25f, -0.25f, -0.25f};
    NE = NEb = f4v{0.0f, 0.0f, 0.0f, 0.0f};
  }
  float Ew = from_left(E[3]), NEbw = from_left(NEb[3]);
  if (ql.lzero) {
    NEbw = 0.0f;
    Ew = -0.25f;
  }
  if (ql.lload) {
    Ew = b >= 0 ? qE[b - 1] : -0.25f;
    NEbw = b >= 0 ? qNE[b - q.qw - 1] : 0.0f;
  }
  f4v out;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float ek = k < 3 ? c[k < 3 ? k + 1 : 0] : e, wk = k > 0 ? c[k > 0 ? k - 1 : 0] : w;
    const float nek = k < 3 ? up[k < 3 ? k + 1 : 0] : ne, swk = k > 0 ? dn[k > 0 ? k - 1 : 0] : sw;
    const float cw = k > 0 ? E[k > 0 ? k - 1 : 0] : Ew, csw = k > 0 ? NEb[k > 0 ? k - 1 : 0] : NEbw;
    out[k] = c[k] + E[k] * ek + cw * wk + N[k] * up[k] + Nb[k] * dn[k] + NE[k] * nek + csw * swk;
  }
  return out;
}
// The same stencil of the vector V (gi = index of (i0, j)): three row loads,
// the values across the quad's edges from the adjacent lanes (the zero ring
// at a row's ends; loaded where a row continues in the next wave).
__device__ inline f4v stencil4(const Geom& g, const QTab& q, const QLane& ql, const float* __restrict__ V,
                               const float* qE, const float* qN, const float* qNE, int i0, int j, int gi) {
  const int P = g.P;
  const f4v c = ld4(V + gi), up = ld4(V + gi + P), dn = ld4(V + gi - P);
  float w = from_left(c[3]), sw = from_left(dn[3]), e = from_right(c[0]), ne = from_right(up[0]);
  if (ql.lzero) w = sw = 0.0f;
  if (ql.lload) {
    w = V[gi - 1];
    sw = V[gi - P - 1];
  }
  if (ql.rload) {
    e = V[gi + 4];
    ne = V[gi + P + 4];
  }
  return stencil4_rows(g, q, ql, c, up, dn, w, e, ne, sw, qE, qN, qNE, i0, j);
}

// LC: coarse levels sv.lds_lev.. in LDS (launched with their bytes of dynamic
// LDS); otherwise every coarse level in global memory.
template <typename VT, int NT, bool MG, bool PARA, bool LC = false>
__global__ __launch_bounds__(NT, 4) void k_ie_stream(Geom g, MGGeom mg, Solver sv, const Inst* __restrict__ insts,
                                                  int n_inst, int* counter, double* work,
                                                  const double* __restrict__ S, VT* vwork) {
  constexpr int NWAVES = NT / 64;
  __shared__ double red[2 * NWAVES * 4];
  __shared__ int s_inst;
  __shared__ int s_dmin;
  __shared__ int s_depok;
  __shared__ unsigned long long s_ph[9];  // thread 0's phase clocks, then its last mark
  extern __shared__ double smem_d[];      // multigrid: coarse levels lds_lev.. (vectors, then tables)
  const int tid = threadIdx.x;
  const int n = g.n, nd = n * n, RHW = g.RW * g.RH;
  const size_t FS = (size_t)g.N * g.P;
  double* Av = work + (size_t)blockIdx.x * ie_work_doubles(g);
  double* Xv = Av + FS;
  double* Bv = Xv + FS;
  double* Xprev = Bv + 2 * FS;
  VT* const vslot = vwork + (size_t)blockIdx.x * stream_slot_elems(g, mg, MG);
  // float4 form of the fine multigrid-CG passes (mixed precision, pitch N + 3):
  // the six full-grid vectors are addressed 3 elements into their planes
  constexpr bool QV = sizeof(VT) == 4 && MG;
  const bool quad = QV && g.P == g.N + 3;
  const int voff = quad ? 3 : 0;
  VT* Rv = vslot + voff;
  VT* Yv = vslot + FS + voff;
  VT* Pv = vslot + 2 * FS + voff;
  VT* Sv = vslot + 3 * FS + voff;
  VT* Wv = vslot + 4 * FS + voff;
  VT* Vv = vslot + 5 * FS + voff;  // multigrid: q = A p
  const QTab qg = qtab_geom(g);
  const int QE = qg.rows * qg.qw;
  float* const qE = (float*)(vslot + 6 * FS);  // quad tables (float form only)
  float* const qN = qE + QE;
  float* const qNE = qN + QE;
  float* const qDi = qNE + QE;
  VT* tE = vslot + 6 * FS + 4 * (size_t)QE;
  VT* tN = tE + RHW;
  VT* tNE = tN + RHW;
  VT* tD = tNE + RHW;
  VT* tDi = tD + RHW;                // D^{1/2}
  VT* mgreg = tDi + RHW;             // multigrid: coarse vectors (zero halo)
  VT* ctab = mgreg + mg.region_elems;  // multigrid: Galerkin tables
  // fine-level thread grid: 2^fs columns x (NT >> fs) rows, no divisions
  int fs = 0;
  while ((1 << fs) < n && (2 << fs) <= NT) ++fs;
  const int ftx = tid & ((1 << fs) - 1), fty = NT >> fs, fj0 = tid >> fs;
  // quad grid: 2^qs threads per row of n + 1 = 4 nq columns (the last quad holds
  // the boundary column n, never stored)
  const int nq = (n + 1) >> 2;
  int qs = 0;
  while ((1 << qs) < nq && (2 << qs) <= NT) ++qs;
  const int qtx = tid & ((1 << qs) - 1), qty = NT >> qs, qj0 = tid >> qs;
  const double d_air = 1.0 / sqrt(4.0 * g.nu_air);
  const int lw = g.lx1 - g.bx0, lh = g.ly1 - g.by0;
  int slot = 0;

  int q_cur = (int)blockIdx.x < counter[3] ? 0 : 1, q_moved = 0;  // work queue of this workgroup (thread 0)
  for (;;) {
    if (tid == 0) s_inst = queue_next(counter, n_inst, q_cur, q_moved);
    __syncthreads();
    const int id = s_inst;
    __syncthreads();
    if (id >= n_inst) break;
    const Inst in = insts[id];
    const double* tab = in.tab;
    const double inv_dt = 1.0 / in.dt;
    const unsigned long long t_begin = wall_clock64();
    // an entry of a one-launch Parareal run: wait (bounded) for its input, then
    // skip (sample stopped, or stopped by this chain's jumps) or run
    int dep_flags = 0;
    if constexpr (PARA) {
      if (in.dep_wait && !para_wait<NT>(in.dep_wait, PARA_WAIT_TICKS, &s_depok, in.para ? in.para->abort : nullptr))
        dep_flags = FLAG_FAILED;
      // (the branch is made wave-uniform: it leaves the entry as a whole)
      if (__builtin_amdgcn_readfirstlane(para_prologue<NT, NWAVES>(g, in, red, slot, &s_depok, &dep_flags) ? 1 : 0)) {
        if (tid == 0 && in.stat) {
          in.stat[3] = dep_flags;
          in.stat[4] = in.stat[6] = (int)(t_begin & 0xffffffffull);
          in.stat[5] = in.stat[7] = (int)(t_begin >> 32);
        }
        if (in.dep_done) para_set(in.dep_done);
        __syncthreads();
        continue;
      }
    }
    auto dscale = [&](int i, int j) -> double {
      if (i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1) {
        const int t = (j - g.by0 + 1) * g.RW + (i - g.bx0 + 1);
        return 1.0 / sqrt(tab[T_MC * RHW + t] * inv_dt + tab[T_KC * RHW + t]);
      }
      return d_air;
    };
    if (tid == 0) s_dmin = __float_as_int((float)d_air);
    __syncthreads();
    for (int t = tid; t < RHW; t += NT) {
      const int i = g.bx0 - 1 + t % g.RW, j = g.by0 - 1 + t / g.RW;
      const bool box = i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1;
      const double di = dscale(i, j);
      if (box) atomicMin(&s_dmin, __float_as_int((float)di));
      double e = -0.25, nn = -0.25, ne = 0.0;
      if (box) {
        e = (tab[T_ME * RHW + t] * inv_dt + tab[T_KE * RHW + t]) * di * dscale(i + 1, j);
        nn = (tab[T_MN * RHW + t] * inv_dt + tab[T_KN * RHW + t]) * di * dscale(i, j + 1);
        ne = tab[T_MNE * RHW + t] * inv_dt * di * dscale(i + 1, j + 1);
      }
      tE[t] = (VT)e;
      tN[t] = (VT)nn;
      tNE[t] = (VT)ne;
      tD[t] = (VT)di;
      tDi[t] = (VT)(1.0 / di);
    }
    for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
      const int gi = (j + 1) * g.P + i + 1;
      Av[gi] = in.a_init ? in.a_init[gi] : 0.0;
      Xv[gi] = in.carry_in ? in.carry[gi] : 0.0;
      Xprev[gi] = in.carry_in ? in.carry[FS + gi] : 0.0;
      if (quad) {
        Pv[gi] = VT(0);
        Vv[gi] = VT(0);
      }
    }
    __syncthreads();
    const double dmin = (double)__int_as_float(s_dmin) * 0.999;
    const double floor_fac = sizeof(VT) == 4 ? 0.25 * sv.tol * sv.tol * dmin * dmin : 0.0;
    if constexpr (MG) {
      auto dn = [&](int i, int j) -> double {  // fine D^{-1/2} (table region, else air)
        if (i >= g.bx0 - 1 && i <= g.bx1 && j >= g.by0 - 1 && j <= g.by1)
          return (double)tD[(j - g.by0 + 1) * g.RW + (i - g.bx0 + 1)];
        return d_air;
      };
      build_galerkin<VT>(mg, ctab, tE, tN, tNE, dn, true, d_air, g.RW, tid, NT);
      for (int l = 1; l <= mg.nlev; ++l) c_zero_halo(clev<VT>(mg, l, mgreg, ctab, NT), tid, NT);
      if constexpr (QV) {
        if (quad) {
          for (int p = tid; p < QE; p += NT) {
            const int i = qg.qx0 + p % qg.qw, j = g.by0 - 2 + p / qg.qw;
            const int ci = i - g.bx0 + 1, cj = j - g.by0 + 1;
            const bool in = ci >= 0 && ci < g.RW && cj >= 0 && cj < g.RH;
            const bool box = i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1;
            const int t = in ? cj * g.RW + ci : 0;
            qE[p] = in ? (float)tE[t] : -0.25f;
            qN[p] = in ? (float)tN[t] : -0.25f;
            qNE[p] = in ? (float)tNE[t] : 0.0f;
            qDi[p] = box ? (float)tDi[t] : (float)(1.0 / d_air);
          }
        }
      }
      __syncthreads();
      if constexpr (LC) {  // coarse levels lds_lev..: tables into LDS, zero halos
        const int la = sv.lds_lev, lz = stream_levels_used(mg, sv);
        const int nvec = lds_vec_elems(mg, la, lz), ntab = lds_tab_elems(mg, la, lz);
        VT* const lreg = reinterpret_cast<VT*>(smem_d);
        VT* const ltab = lreg + nvec;
        for (int q = tid; q < ntab; q += NT) ltab[q] = ctab[mg.lv[la].tab_off + q];
        for (int l = la; l <= lz; ++l)
          c_zero_halo(clev<VT>(mg, l, lreg - mg.lv[la].vec_off, ltab - mg.lv[la].tab_off, NT), tid, NT);
        __syncthreads();
      }
    }
    auto dnode = [&](int i, int j, const NodeRef& nr) -> VT {  // (load issued unconditionally)
      const bool box = i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1;
      const VT d = tD[box ? nr.t : g.RW + 1];
      return box ? d : (VT)d_air;
    };
    auto dnode_inv = [&](int i, int j, const NodeRef& nr) -> VT {  // D^{1/2}
      const bool box = i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1;
      return box ? tDi[nr.t] : (VT)(1.0 / d_air);
    };

    double qsum = in.carry_in ? in.carry[2 * FS] : 0.0;
    int it_total = 0, sw_total = 0, it_max_step = 0, flags = dep_flags;
    // phase clocks of thread 0 in LDS (same phase indices as the resident
    // kernel; kept out of the registers)
    if (tid == 0) {
      for (int q = 0; q < 8; ++q) s_ph[q] = 0;
      s_ph[8] = wall_clock64();
    }
    auto tick = [&](int q) __attribute__((always_inline)) {
      if (tid == 0) {
        const unsigned long long t = wall_clock64();
        if (q >= 0) s_ph[q] += t - s_ph[8];
        s_ph[8] = t;
      }
    };
    const int n_seg = in.n_chain > 0 ? in.n_chain : 1;
    for (int seg = 0; seg < n_seg; ++seg) {
      const int kseg0 = in.k0 + seg * in.n_steps;
      for (int step = 0; step < in.n_steps; ++step) {
        const double Jt = in.src[kseg0 + step + 1];
        tick(-1);
        double part[1] = {0.0};
        for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
          const NodeRef nr = node_ref(g, i, j);
          const double b = Jt * S[nr.gi] - K_apply_u(g, tab, Av, nr);
          Bv[nr.gi] = b;
          part[0] += b * b;
        }
        block_sum<1, NWAVES>(part, red, slot);
        tick(4);
        const double bb = part[0];
        int it_step = 0;
        if (bb == 0.0) {
          for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) Xv[(j + 1) * g.P + i + 1] = 0.0;
          __syncthreads();
        } else {
          bool conv = false;
          for (int sweep = 0; sweep <= sv.max_sweeps; ++sweep) {
            tick(-1);
            double rr[1] = {0.0};
            for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
              const NodeRef nr = node_ref(g, i, j);
              const double res = Bv[nr.gi] - A_apply_u(g, tab, Xv, nr, inv_dt);
              rr[0] += res * res;
              Rv[nr.gi] = (VT)(res * (double)dnode(i, j, nr));
              Yv[nr.gi] = VT(0);
              // (the float4 passes write S before reading it and read P and V
              // only times beta = 0 in the first iteration: finite from the
              // instance's start on, so they need no clearing per sweep)
              if (!quad) {
                Pv[nr.gi] = VT(0);
                Sv[nr.gi] = VT(0);
                if constexpr (MG) Vv[nr.gi] = VT(0);
              }
            }
            block_sum<1, NWAVES>(rr, red, slot);
            tick(5);
            if (!(rr[0] == rr[0]) || isinf(rr[0])) {
              flags |= FLAG_FAILED;
              break;
            }
            if (rr[0] <= sv.tol * sv.tol * bb) {
              conv = true;
              break;
            }
            if (sweep == sv.max_sweeps) break;
            sw_total++;
            int it = 0;
            if constexpr (MG) {
              // ---- CG preconditioned by a geometric multigrid V(1,1)-cycle ----
              // (the resident kernel's cycle with every level in global memory)
              const VT om = vt<VT>(sv.mg_omega);
              auto nodes = [&](auto&& f) __attribute__((always_inline)) {
                for (int j = fj0; j < n; j += fty)
                  for (int i = ftx; i < n; i += (1 << fs)) f(i, j, node_ref(g, i, j));
              };
              // The same nodes two rows at a time, split into a pure load/compute
              // part `ld` and a store/accumulate part `st`: both nodes' loads are
              // issued before either node's stores, which doubles the loads in
              // flight (no node of a pass reads what another node of the same pass
              // writes).  Stores and sums keep the order of `nodes` whenever a row
              // holds one node per thread (meshes up to 513 x 513).
              struct V2 {
                VT x, y;
              };
              auto nodes2 = [&](auto&& ld, auto&& st) __attribute__((always_inline)) {
                for (int j = fj0; j < n; j += 2 * fty) {
                  const int j2 = j + fty;
                  const int jb = j2 < n ? j2 : j;  // past the last row: reload row j, store nothing
                  for (int i = ftx; i < n; i += (1 << fs)) {
                    const NodeRef a = node_ref(g, i, j), b = node_ref(g, i, jb);
                    const V2 va = ld(i, j, a), vb = ld(i, jb, b);
                    st(a, va);
                    if (j2 < n) st(b, vb);
                  }
                }
              };
              // Four consecutive nodes per thread, one row at a time (float4 loads
              // and stores).  (Two rows per step, loads first, measured no faster:
              // the passes are bound by memory instructions issued, not by loads
              // in flight.)
              auto quads2 = [&](auto&& ld, auto&& st) __attribute__((always_inline)) {
                if (qtx >= nq) return;
                const int i0 = qtx << 2;
                const int nv = i0 + 4 <= n ? 4 : n - i0;
                for (int j = qj0; j < n; j += qty) {
                  const int ga = (j + 1) * g.P + i0 + 1;
                  const F4x2 va = ld(i0, j, ga);
                  st(ga, nv, va);
                }
              };
              const float di_air = (float)(1.0 / d_air);
              auto dinv4 = [&](int i0, int j) __attribute__((always_inline)) {  // D^{1/2} of four nodes
                const int b = qbase(g, qg, i0, j);
                return b >= 0 ? ld4(qDi + b) : f4v{di_air, di_air, di_air, di_air};
              };
              const QLane ql = qlane(qtx, nq);
              VT* Zm = Sv;  // preconditioned residual
              VT* Tm = Wv;  // fine residual t / smoothing output (swapped with Zm)
              // coarse levels hold the unscaled operators: level 1 <-> scaled fine
              // level through D^{1/2} P (air diagonal 4 nu_air = 1 / d_air^2)
              const VT air = vt<VT>(1.0 / (d_air * d_air));
              const CLev<VT> L1 = clev<VT>(mg, 1, mgreg, ctab, NT, air);
              const bool exact1 = mg.nlev == 1 || sv.mg_levels == 1;
              double rho = 1.0, stop = 0.0;
              for (;;) {
                tick(-1);
                // z = B r: pre-smoothing from zero (z = om r) and t = r - A z
                if constexpr (QV) {
                  if (quad) {
                    const float* R4 = (const float*)Rv;
                    quads2(
                        [&](int i0, int j, int gi) {
                          const f4v r = ld4(R4 + gi);
                          const f4v ar = stencil4(g, qg, ql, R4, qE, qN, qNE, i0, j, gi);
                          return F4x2{(float)om * r, (r - (float)om * ar) * dinv4(i0, j)};
                        },
                        [&](int gi, int nv, const F4x2& v) {
                          st4((float*)Zm + gi, v.a, nv);
                          st4((float*)Tm + gi, v.b, nv);
                        });
                  }
                }
                if (!quad)
                nodes2(
                    [&](int i, int j, const NodeRef& nr) {
                      const VT r = Rv[nr.gi];
                      return V2{om * r, (r - om * stencil_scaled<VT>(g, Rv, tE, tN, tNE, nr)) * dnode_inv(i, j, nr)};
                    },
                    [&](const NodeRef& nr, const V2& v) {
                      Zm[nr.gi] = v.x;
                      Tm[nr.gi] = v.y;
                    });
                __syncthreads();
                tick(0);
                {  // restriction to level 1 (two rows per step, loads first)
                  const int tx = tid & ((1 << L1.txs) - 1), ty = NT >> L1.txs;
                  const VT f1 = exact1 ? VT(1) : om;
                  if (tx < L1.n) {
                    for (int j = tid >> L1.txs; j < L1.n; j += 2 * ty) {
                      const int j2 = j + ty < L1.n ? j + ty : j;
                      const VT rc = restrict_at(Tm, g.P, tx, j), rc2 = restrict_at(Tm, g.P, tx, j2);
                      const VT d = clev_id(L1, tx, j), d2 = clev_id(L1, tx, j2);
                      const int q = (j + 1) * L1.np + tx + 1, q2 = (j2 + 1) * L1.np + tx + 1;
                      L1.R[q] = rc;
                      L1.Z[q] = f1 * d * rc;
                      if (j + ty < L1.n) {
                        L1.R[q2] = rc2;
                        L1.Z[q2] = f1 * d2 * rc2;
                      }
                    }
                  }
                }
                __syncthreads();
                const VT* z1;
                if constexpr (LC)
                  z1 = coarse_cycle_lds<VT, NT>(mg, mgreg, ctab, reinterpret_cast<VT*>(smem_d),
                                                reinterpret_cast<VT*>(smem_d) +
                                                    lds_vec_elems(mg, sv.lds_lev, stream_levels_used(mg, sv)),
                                                sv.lds_lev, om, tid, air, sv.mg_levels, sv.mg_coarse_sweeps,
                                                sv.mg_block_min);
                else
                  z1 = coarse_cycle<VT, NT, true>(mg, mgreg, ctab, om, tid, air, sv.mg_levels, sv.mg_coarse_sweeps,
                                                  sv.mg_block_min);
                __syncthreads();
                tick(1);
                // prolongation z <- z + P z_1 D^{1/2} and post-smoothing z <- z + om (r - A z);
                // r.z and r.r of the new z
                double rz[2] = {0.0, 0.0};
                if constexpr (QV) {
                  if (quad) {
                    // One pass: each quad forms the prolonged z of its four nodes on
                    // rows j - 1, j, j + 1 (the coarse values it needs: columns 2q - 1
                    // .. 2q + 1 of coarse rows m - 1 .. m + 1, m = j / 2, the left one
                    // from the adjacent lane) and takes the values across its edges
                    // from the adjacent lanes; the same values, computed in the same
                    // way, that a separate prolongation pass would store.
                    const float* Z4 = (const float*)Zm;
                    const float* zc1 = (const float*)z1;
                    const int cp = L1.np, nc = L1.n;
                    struct CRow {
                      float c0, c1, cm;  // coarse columns 2q, 2q + 1, 2q - 1 of one coarse row
                    };
                    auto crow = [&](int i0, int mr) __attribute__((always_inline)) {
                      const float* b = zc1 + (mr + 1) * cp + (i0 >> 1) + 1;
                      CRow r{b[0], b[1], 0.0f};
                      r.cm = from_left(r.c1);
                      if (ql.lzero) r.cm = 0.0f;
                      if (ql.lload) r.cm = b[-1];
                      return r;
                    };
                    // P z_1 on a fine row: odd rows from coarse row jr / 2 (a), even rows
                    // from coarse rows jr / 2 (a) and jr / 2 - 1 (b)
                    auto p_odd = [](const CRow& a) __attribute__((always_inline)) {
                      return f4v{0.5f * (a.cm + a.c0), a.c0, 0.5f * (a.c0 + a.c1), a.c1};
                    };
                    auto p_even = [](const CRow& a, const CRow& b) __attribute__((always_inline)) {
                      return f4v{0.5f * (b.cm + a.c0), 0.5f * (b.c0 + a.c0), 0.5f * (b.c0 + a.c1),
                                 0.5f * (b.c1 + a.c1)};
                    };
                    auto zrow = [&](int i0, int jr, int gr, const f4v& pv) __attribute__((always_inline)) {
                      if (jr < 0 || jr >= n) return f4v{0.0f, 0.0f, 0.0f, 0.0f};  // boundary ring
                      f4v z = ld4(Z4 + gr);
                      const f4v di = dinv4(i0, jr);
#pragma unroll
                      for (int k = 0; k < 4; ++k)
                        if (i0 + k < n) z[k] = z[k] + pv[k] * di[k];
                      return z;
                    };
                    // one node's prolonged z (the lanes at a wave's ends of rows that
                    // continue in the next wave)
                    auto zone = [&](int i, int jr) -> float {
                      if (i < 0 || i >= n || jr < 0 || jr >= n) return 0.0f;
                      const NodeRef nr = node_ref(g, i, jr);
                      return Z4[nr.gi] + (float)prolong_at(z1, cp, i, jr) * (float)dnode_inv(i, jr, nr);
                    };
                    quads2(
                        [&](int i0, int j, int gi) {
                          const int m = j >> 1;
                          const CRow a = crow(i0, m), b = crow(i0, m - 1), c = crow(i0, m + 1 <= nc ? m + 1 : nc);
                          const bool odd = j & 1;
                          const f4v zc = zrow(i0, j, gi, odd ? p_odd(a) : p_even(a, b));
                          const f4v zu = zrow(i0, j + 1, gi + g.P, odd ? p_even(c, a) : p_odd(a));
                          const f4v zd = zrow(i0, j - 1, gi - g.P, odd ? p_even(a, b) : p_odd(b));
                          float w = from_left(zc[3]), sw = from_left(zd[3]), e = from_right(zc[0]),
                                ne = from_right(zu[0]);
                          if (ql.lzero) w = sw = 0.0f;
                          if (ql.lload) {
                            w = zone(i0 - 1, j);
                            sw = zone(i0 - 1, j - 1);
                          }
                          if (ql.rload) {
                            e = zone(i0 + 4, j);
                            ne = zone(i0 + 4, j + 1);
                          }
                          const f4v az = stencil4_rows(g, qg, ql, zc, zu, zd, w, e, ne, sw, qE, qN, qNE, i0, j);
                          const f4v r = ld4((const float*)Rv + gi);
                          return F4x2{zc + (float)om * (r - az), r};
                        },
                        [&](int gi, int nv, const F4x2& v) {
                          st4((float*)Tm + gi, v.a, nv);
#pragma unroll
                          for (int k = 0; k < 4; ++k) {
                            if (k < nv) {
                              rz[0] += (double)(v.b[k] * v.a[k]);
                              rz[1] += (double)(v.b[k] * v.b[k]);
                            }
                          }
                        });
                  }
                }
                if (!quad) {
                  nodes2(
                      [&](int i, int j, const NodeRef& nr) {
                        return V2{Zm[nr.gi] + prolong_at(z1, L1.np, i, j) * dnode_inv(i, j, nr), VT(0)};
                      },
                      [&](const NodeRef& nr, const V2& v) { Zm[nr.gi] = v.x; });
                  __syncthreads();
                  nodes2(
                      [&](int, int, const NodeRef& nr) {
                        const VT r = Rv[nr.gi], z = Zm[nr.gi];
                        return V2{z + om * (r - stencil_scaled<VT>(g, Zm, tE, tN, tNE, nr)), r};
                      },
                      [&](const NodeRef& nr, const V2& v) {
                        Tm[nr.gi] = v.x;
                        rz[0] += (double)(v.y * v.x);
                        rz[1] += (double)(v.y * v.y);
                      });
                }
                block_sum<2, NWAVES>(rz, red, slot);
                tick(2);
                { VT* t_ = Zm; Zm = Tm; Tm = t_; }
                double beta = 0.0;
                if (it == 0) {
                  stop = fmax(sv.inner_rtol * sv.inner_rtol * rz[1], floor_fac * bb);
                  if (!(rz[1] > 0.0) || !(rz[0] > 0.0)) break;
                } else {
                  if (rz[1] <= stop || !(rz[1] == rz[1])) break;
                  beta = rz[0] / rho;
                }
                rho = rz[0];
                if (it == sv.max_iter) break;
                ++it;
                // p = z + beta p and q = A p = A z + beta q (one pass)
                const VT b_ = vt<VT>(beta);
                double pq[1] = {0.0};
                if constexpr (QV) {
                  if (quad) {
                    const float* Z4 = (const float*)Zm;
                    quads2(
                        [&](int i0, int j, int gi) {
                          const f4v az = stencil4(g, qg, ql, Z4, qE, qN, qNE, i0, j, gi);
                          return F4x2{ld4(Z4 + gi) + (float)b_ * ld4((const float*)Pv + gi),
                                      az + (float)b_ * ld4((const float*)Vv + gi)};
                        },
                        [&](int gi, int nv, const F4x2& v) {
                          st4((float*)Pv + gi, v.a, nv);
                          st4((float*)Vv + gi, v.b, nv);
#pragma unroll
                          for (int k = 0; k < 4; ++k)
                            if (k < nv) pq[0] += (double)(v.a[k] * v.b[k]);
                        });
                  }
                }
                if (!quad)
                nodes2(
                    [&](int, int, const NodeRef& nr) {
                      return V2{Zm[nr.gi] + b_ * Pv[nr.gi], stencil_scaled<VT>(g, Zm, tE, tN, tNE, nr) + b_ * Vv[nr.gi]};
                    },
                    [&](const NodeRef& nr, const V2& v) {
                      Pv[nr.gi] = v.x;
                      Vv[nr.gi] = v.y;
                      pq[0] += (double)(v.x * v.y);
                    });
                block_sum<1, NWAVES>(pq, red, slot);
                const VT a_ = vt<VT>(rho / pq[0]);
                if constexpr (QV) {
                  if (quad) {
                    quads2(
                        [&](int, int, int gi) {
                          return F4x2{ld4((const float*)Yv + gi) + (float)a_ * ld4((const float*)Pv + gi),
                                      ld4((const float*)Rv + gi) - (float)a_ * ld4((const float*)Vv + gi)};
                        },
                        [&](int gi, int nv, const F4x2& v) {
                          st4((float*)Yv + gi, v.a, nv);
                          st4((float*)Rv + gi, v.b, nv);
                        });
                  }
                }
                if (!quad)
                nodes2(
                    [&](int, int, const NodeRef& nr) {
                      return V2{Yv[nr.gi] + a_ * Pv[nr.gi], Rv[nr.gi] - a_ * Vv[nr.gi]};
                    },
                    [&](const NodeRef& nr, const V2& v) {
                      Yv[nr.gi] = v.x;
                      Rv[nr.gi] = v.y;
                    });
                __syncthreads();
                tick(3);
              }
            } else {
            double gd[2] = {0.0, 0.0};
            for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
              const NodeRef nr = node_ref(g, i, j);
              const VT w = stencil_scaled<VT>(g, Rv, tE, tN, tNE, nr);
              const VT r = Rv[nr.gi];
              Wv[nr.gi] = w;
              gd[0] += (double)(r * r);
              gd[1] += (double)(w * r);
            }
            block_sum<2, NWAVES>(gd, red, slot);
            const double g0 = gd[0];
            double gam = gd[0], alpha = gd[0] / gd[1], beta = 0.0;
            const double stop = fmax(sv.inner_rtol * sv.inner_rtol * g0, floor_fac * bb);
            if (g0 > 0.0) {
              for (it = 1; it <= sv.max_iter; ++it) {
                const VT a_ = (VT)alpha, b_ = (VT)beta;
                for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
                  const int gi = (j + 1) * g.P + i + 1;
                  const VT p = Rv[gi] + b_ * Pv[gi];
                  const VT s = Wv[gi] + b_ * Sv[gi];
                  Pv[gi] = p;
                  Sv[gi] = s;
                  Yv[gi] = Yv[gi] + a_ * p;
                  Rv[gi] = Rv[gi] - a_ * s;
                }
                __syncthreads();
                gd[0] = 0.0;
                gd[1] = 0.0;
                for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
                  const NodeRef nr = node_ref(g, i, j);
                  const VT w = stencil_scaled<VT>(g, Rv, tE, tN, tNE, nr);
                  const VT r = Rv[nr.gi];
                  Wv[nr.gi] = w;
                  gd[0] += (double)(r * r);
                  gd[1] += (double)(w * r);
                }
                block_sum<2, NWAVES>(gd, red, slot);
                if (gd[0] <= stop || !(gd[0] == gd[0])) break;
                const double bn = gd[0] / gam;
                alpha = gd[0] / (gd[1] - bn * gd[0] / alpha);
                beta = bn;
                gam = gd[0];
              }
              if (it > sv.max_iter) it = sv.max_iter;
            }
            }
            it_step += it;
            tick(-1);
            for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
              const NodeRef nr = node_ref(g, i, j);
              Xv[nr.gi] += (double)dnode(i, j, nr) * (double)Yv[nr.gi];
            }
            __syncthreads();
            tick(6);
          }
          if (!conv) flags |= FLAG_NOT_CONVERGED;
        }
        it_total += it_step;
        it_max_step = it_step > it_max_step ? it_step : it_max_step;
        tick(-1);
        double qq[1] = {0.0};
        for (int idx = tid; idx < lw * lh; idx += NT) {
          const NodeRef nr = node_ref(g, g.bx0 + idx % lw, g.by0 + idx / lw);
          qq[0] += Xv[nr.gi] * M_apply(g, tab, Xv, nr);
        }
        block_sum<1, NWAVES>(qq, red, slot);
        qsum += qq[0] * inv_dt;
        for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
          const int gi = (j + 1) * g.P + i + 1;
          const double d = Xv[gi];
          Av[gi] += d;
          Xv[gi] = 2.0 * d - Xprev[gi];
          Xprev[gi] = d;
        }
        __syncthreads();
        tick(7);
      }
      if (in.n_chain > 0) {
        const double* Fn = in.chain_f[seg];
        double* Cn = in.chain_c[seg];
        double* Un = in.chain_u[seg];
        for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
          const int gi = (j + 1) * g.P + i + 1;
          const double cn = Av[gi];
          const double u = Fn ? Fn[gi] + (cn - Cn[gi]) : cn;
          Cn[gi] = cn;
          Un[gi] = u;
          Av[gi] = u;
        }
        __syncthreads();
        if constexpr (PARA)
          if (in.seg_done) para_set(in.seg_done[seg]);
      }
    }
    if (in.a_out) {
      for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
        const int gi = (j + 1) * g.P + i + 1;
        in.a_out[gi] = Av[gi];
      }
    }
    if (in.carry) {
      for (int j = fj0; j < n; j += fty) for (int i = ftx; i < n; i += (1 << fs)) {
        const int gi = (j + 1) * g.P + i + 1;
        in.carry[gi] = Xv[gi];
        in.carry[FS + gi] = Xprev[gi];
      }
      if (tid == 0) in.carry[2 * FS] = qsum;
    }
    if constexpr (PARA)
      if (in.dep_done) para_set(in.dep_done);  // publishes a_out (and carry) first
    if (tid == 0) {
      if (in.q_out) *in.q_out = qsum * in.q_scale;
      if (in.stat) {
        const unsigned long long t_end = wall_clock64();
        in.stat[0] = it_total;
        in.stat[1] = sw_total;
        in.stat[2] = it_max_step;
        in.stat[3] = flags;
        in.stat[4] = (int)(t_begin & 0xffffffffull);
        in.stat[5] = (int)(t_begin >> 32);
        in.stat[6] = (int)(t_end & 0xffffffffull);
        in.stat[7] = (int)(t_end >> 32);
        for (int q = 0; q < 8; ++q) in.stat[8 + q] = (int)(s_ph[q] >> 4);  // units of 16 ticks
      }
      publish_done(in.host_done, qsum * in.q_scale, flags);
    }
    __syncthreads();
  }
}

constexpr int STREAM_NT = 1024;

size_t stream_vwork_elems(const Geom& g, const MGGeom* mg) {
  return stream_slot_elems(g, mg ? *mg : MGGeom{}, mg && mg->nlev > 0);
}

template <int NT, bool PARA>
static hipError_t launch_stream_nt(const Geom& g, const MGGeom& mg, const Solver& sv0, const Inst* insts, int n_inst,
                                  int* counter, double* work, int n_slots, int grid, const double* S, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  double* vbase = work + (size_t)n_slots * ie_work_doubles(g);
  const bool usemg = sv0.precond == 1 && mg.nlev > 0;
  Solver sv = sv0;
  size_t lds = 0;
  sv.lds_lev = 0;
  if (usemg && sv.precision != MQ_PREC_FP64) {
    // the kernel's own LDS takes under 2 KB; two 512-thread workgroups share a compute unit
    const size_t cap = (size_t)(NT == 512 ? sv.lds_limit / 2 : sv.lds_limit);
    if (cap > 4096) sv.lds_lev = stream_lds_level(mg, sv, sizeof(float), cap - 4096, &lds);
  }
  auto setup = [&](const void* kern) -> hipError_t {
    if (lds == 0) return hipSuccess;
    return hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  };
  if (sv.precision == MQ_PREC_FP64) {
    if (usemg)
      hipLaunchKernelGGL((k_ie_stream<double, NT, true, PARA>), dim3(grid), dim3(NT), lds, st, g, mg, sv, insts, n_inst,
                         counter, work, S, vbase);
    else
      hipLaunchKernelGGL((k_ie_stream<double, NT, false, PARA>), dim3(grid), dim3(NT), lds, st, g, mg, sv, insts,
                         n_inst, counter, work, S, vbase);
  } else {
    float* fb = reinterpret_cast<float*>(vbase);
    if (usemg && sv.lds_lev > 0) {
      const hipError_t e = setup((const void*)k_ie_stream<float, NT, true, PARA, true>);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_ie_stream<float, NT, true, PARA, true>), dim3(grid), dim3(NT), lds, st, g, mg, sv, insts,
                         n_inst, counter, work, S, fb);
    } else if (usemg)
      hipLaunchKernelGGL((k_ie_stream<float, NT, true, PARA>), dim3(grid), dim3(NT), lds, st, g, mg, sv, insts, n_inst,
                         counter, work, S, fb);
    else
      hipLaunchKernelGGL((k_ie_stream<float, NT, false, PARA>), dim3(grid), dim3(NT), lds, st, g, mg, sv, insts, n_inst,
                         counter, work, S, fb);
  }
  return hipGetLastError();
}

// Streaming workgroup size: 1024 threads (tile 1) or 512 threads (tile 2,
// two workgroups per compute unit).
int stream_threads(int tile) { return tile == 2 ? 512 : STREAM_NT; }

hipError_t launch_ie_stream(const Geom& g, const MGGeom& mg, const Solver& sv, const Inst* insts, int n_inst,
                            int* counter, double* work, int n_slots, int max_grid, const double* S,
                            int* grid_out, int* block_out, hipStream_t st) {
  // the VT workspace follows the FP64 work buffers of all n_slots slots
  const int grid = max_grid < n_inst ? max_grid : n_inst;
  const int nt = stream_threads(sv.tile);
  if (grid_out) *grid_out = grid;
  if (block_out) *block_out = nt;
  // Parareal entries take the instantiation with the entry prologue
  if (sv.para) {
    if (nt == 512) return launch_stream_nt<512, true>(g, mg, sv, insts, n_inst, counter, work, n_slots, grid, S, st);
    return launch_stream_nt<STREAM_NT, true>(g, mg, sv, insts, n_inst, counter, work, n_slots, grid, S, st);
  }
  if (nt == 512) return launch_stream_nt<512, false>(g, mg, sv, insts, n_inst, counter, work, n_slots, grid, S, st);
  return launch_stream_nt<STREAM_NT, false>(g, mg, sv, insts, n_inst, counter, work, n_slots, grid, S, st);
}

}  // namespace mq

// ---------------------------------------------------------------------------
// wide path: one instance spread over the whole device
// ---------------------------------------------------------------------------
// Every pass of the streaming solver becomes a grid-wide kernel (2-D grid:
// blockIdx.y = row, blockIdx.x * 256 + tid = column); reductions leave one
// partial per block and a one-block kernel sums them in a fixed order and
// takes the solver's scalar decisions into WideScal.  Passes of the inner CG
// return at once when WideScal::done is set, so the host can replay a fixed
// batch of iterations (a captured graph) and read one flag per batch.
namespace mq {

constexpr int WIDE_BX = 256;

#define WIDE_NODE                                                    \
  const int i = blockIdx.x * WIDE_BX + threadIdx.x, j = blockIdx.y; \
  const bool act = i < g.n;                                          \
  const NodeRef nr = node_ref(g, act ? i : 0, j)

// block partials of NV values (one per block, blocks numbered y * gridDim.x + x)
template <int NV>
__device__ inline void wide_partial(double (&v)[NV], double* part) {
  __shared__ double red[2 * (WIDE_BX / 64) * 4];
  int slot = 0;
  block_sum<NV, WIDE_BX / 64>(v, red, slot);
  if (threadIdx.x == 0) {
    const int b = blockIdx.y * gridDim.x + blockIdx.x;
#pragma unroll
    for (int q = 0; q < NV; ++q) part[q * (size_t)gridDim.x * gridDim.y + b] = v[q];
  }
}

template <typename VT>
__device__ inline VT wide_dnode(const Geom& g, const VT* tD, double d_air, int i, int j, const NodeRef& nr) {
  const bool box = i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1;
  return box ? tD[nr.t] : (VT)d_air;
}
template <typename VT>
__device__ inline VT wide_dinv(const Geom& g, const VT* tDi, double d_air, int i, int j, const NodeRef& nr) {
  const bool box = i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1;
  return box ? tDi[nr.t] : (VT)(1.0 / d_air);
}

// per-instance set-up (one workgroup): scaled tables, D^{+-1/2}, Galerkin
// hierarchy, zero halos, initial state, scalars
template <typename VT>
__global__ __launch_bounds__(1024) void k_w_setup(Geom g, MGGeom mg, Solver sv, WidePtrs w, double inv_dt,
                                                  const double* __restrict__ a_init) {
  constexpr int NT = 1024;
  __shared__ int s_dmin;
  const int tid = threadIdx.x, RHW = g.RW * g.RH, n = g.n;
  const double* tab = w.tab;
  VT* tE = (VT*)w.tE;
  VT* tN = (VT*)w.tN;
  VT* tNE = (VT*)w.tNE;
  VT* tD = (VT*)w.tD;
  VT* tDi = (VT*)w.tDi;
  const double d_air = 1.0 / sqrt(4.0 * g.nu_air);
  auto dscale = [&](int i, int j) -> double {
    if (i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1) {
      const int t = (j - g.by0 + 1) * g.RW + (i - g.bx0 + 1);
      return 1.0 / sqrt(tab[T_MC * RHW + t] * inv_dt + tab[T_KC * RHW + t]);
    }
    return d_air;
  };
  if (tid == 0) s_dmin = __float_as_int((float)d_air);
  __syncthreads();
  for (int t = tid; t < RHW; t += NT) {
    const int i = g.bx0 - 1 + t % g.RW, j = g.by0 - 1 + t / g.RW;
    const bool box = i >= g.bx0 && i < g.bx1 && j >= g.by0 && j < g.by1;
    const double di = dscale(i, j);
    if (box) atomicMin(&s_dmin, __float_as_int((float)di));
    double e = -0.25, nn = -0.25, ne = 0.0;
    if (box) {
      e = (tab[T_ME * RHW + t] * inv_dt + tab[T_KE * RHW + t]) * di * dscale(i + 1, j);
      nn = (tab[T_MN * RHW + t] * inv_dt + tab[T_KN * RHW + t]) * di * dscale(i, j + 1);
      ne = tab[T_MNE * RHW + t] * inv_dt * di * dscale(i + 1, j + 1);
    }
    tE[t] = (VT)e;
    tN[t] = (VT)nn;
    tNE[t] = (VT)ne;
    tD[t] = (VT)di;
    tDi[t] = (VT)(1.0 / di);
  }
  for (int idx = tid; idx < n * n; idx += NT) {
    const int gi = (idx / n + 1) * g.P + idx % n + 1;
    w.Av[gi] = a_init ? a_init[gi] : 0.0;
    w.Xv[gi] = 0.0;
    w.Xp[gi] = 0.0;
  }
  __syncthreads();
  auto dn = [&](int i, int j) -> double {
    if (i >= g.bx0 - 1 && i <= g.bx1 && j >= g.by0 - 1 && j <= g.by1)
      return (double)tD[(j - g.by0 + 1) * g.RW + (i - g.bx0 + 1)];
    return d_air;
  };
  build_galerkin<VT>(mg, (VT*)w.ctab, tE, tN, tNE, dn, true, d_air, g.RW, tid, NT);
  for (int l = 1; l <= mg.nlev; ++l) c_zero_halo(clev<VT>(mg, l, (VT*)w.mgreg, (VT*)w.ctab, NT), tid, NT);
  if (tid == 0) {
    const double dmin = (double)__int_as_float(s_dmin) * 0.999;
    WideScal* sc = w.sc;
    sc->floor_fac = sizeof(VT) == 4 ? 0.25 * sv.tol * sv.tol * dmin * dmin : 0.0;
    sc->qsum = 0.0;
    sc->flags = 0;
    sc->it_total = 0;
    sc->sweeps = 0;
    sc->done = 1;
  }
}

// b = J S - K a and partial ||b||^2
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_rhs(Geom g, WidePtrs w, double Jt) {
  WIDE_NODE;
  double v[1] = {0.0};
  if (act) {
    const double b = Jt * w.S[nr.gi] - K_apply(g, w.tab, w.Av, nr);
    w.Bv[nr.gi] = b;
    v[0] = b * b;
  }
  wide_partial<1>(v, w.part);
}

// FP64 residual r64 = b - A x, its scaled VT copy, fresh inner vectors
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_resid(Geom g, WidePtrs w, double inv_dt) {
  WIDE_NODE;
  double v[1] = {0.0};
  if (act) {
    const double res = w.Bv[nr.gi] - A_apply(g, w.tab, w.Xv, nr, inv_dt);
    v[0] = res * res;
    const double d_air = 1.0 / sqrt(4.0 * g.nu_air);
    ((VT*)w.R)[nr.gi] = (VT)(res * (double)wide_dnode<VT>(g, (VT*)w.tD, d_air, i, j, nr));
    ((VT*)w.Y)[nr.gi] = VT(0);
    ((VT*)w.P)[nr.gi] = VT(0);
    ((VT*)w.Q)[nr.gi] = VT(0);
  }
  wide_partial<1>(v, w.part);
}

enum { WRED_RHS = 0, WRED_RES = 1, WRED_RZ = 2, WRED_PQ = 3, WRED_QOI = 4 };

// Sums the block partials in a fixed order and takes the scalar decisions.
template <int KIND, int NV>
__global__ __launch_bounds__(1024) void k_w_reduce(WidePtrs w, Solver sv, int nblk, double inv_dt) {
  __shared__ double red[2 * 16 * 4];
  WideScal* sc = w.sc;
  if (KIND == WRED_RZ || KIND == WRED_PQ) {
    if (sc->done) return;
  }
  double v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 1024) s += w.part[q * (size_t)nblk + b];
    v[q] = s;
  }
  int slot = 0;
  block_sum<NV, 16>(v, red, slot);
  if (threadIdx.x != 0) return;
  if (KIND == WRED_RHS) {
    sc->bb = v[0];
  } else if (KIND == WRED_RES) {
    sc->rr = v[0];
    sc->it = 0;
    sc->rho = 1.0;
    if (!(v[0] == v[0]) || isinf(v[0])) {
      sc->flags |= FLAG_FAILED;
      sc->conv = 1;
    } else {
      sc->conv = v[0] <= sv.tol * sv.tol * sc->bb ? 1 : 0;
    }
    sc->done = sc->conv;
  } else if (KIND == WRED_RZ) {
    const double rz = v[0], rr = v[1];
    double beta = 0.0;
    int done = 0;
    if (sc->it == 0) {
      sc->stop = fmax(sv.inner_rtol * sv.inner_rtol * rr, sc->floor_fac * sc->bb);
      if (!(rr > 0.0) || !(rz > 0.0)) done = 1;
    } else {
      if (rr <= sc->stop || !(rr == rr)) done = 1;
      else beta = rz / sc->rho;
    }
    if (!done) {
      sc->rho = rz;
      if (sc->it == sv.max_iter) {
        done = 1;
      } else {
        sc->beta = beta;
        sc->it += 1;
        sc->it_total += 1;
      }
    }
    sc->done = done;
  } else if (KIND == WRED_PQ) {
    sc->alpha = sc->rho / v[0];
  } else {
    sc->qsum += v[0] * inv_dt;
  }
}

// pre-smoothing from zero: Z = om R, T = D^{1/2} (R - om A R)
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_pre(Geom g, WidePtrs w, VT om) {
  if (w.sc->done) return;
  WIDE_NODE;
  if (!act) return;
  const VT* R = (const VT*)w.R;
  const VT r = R[nr.gi];
  const double d_air = 1.0 / sqrt(4.0 * g.nu_air);
  ((VT*)w.Z)[nr.gi] = om * r;
  ((VT*)w.T)[nr.gi] = (r - om * stencil_scaled<VT>(g, R, (VT*)w.tE, (VT*)w.tN, (VT*)w.tNE, nr)) *
                      wide_dinv<VT>(g, (VT*)w.tDi, d_air, i, j, nr);
}

// restriction of T to level 1: R_1 and Z_1 = om ID R_1 (ID R_1 if level 1 is the coarsest)
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_restrict1(Geom g, MGGeom mg, WidePtrs w, VT om, VT air) {
  if (w.sc->done) return;
  const int nthr = gridDim.x * blockDim.x, me = blockIdx.x * blockDim.x + threadIdx.x;
  const CLev<VT> L1 = clev<VT>(mg, 1, (VT*)w.mgreg, (const VT*)w.ctab, nthr, air);
  const int tx = me & ((1 << L1.txs) - 1), ty = nthr >> L1.txs;
  if (tx >= L1.n) return;
  const bool exact1 = mg.nlev == 1;
  for (int jj = me >> L1.txs; jj < L1.n; jj += ty) {
    const VT rc = restrict_at((const VT*)w.T, g.P, tx, jj);
    const int q = (jj + 1) * L1.np + tx + 1;
    L1.R[q] = rc;
    L1.Z[q] = (exact1 ? VT(1) : om) * clev_id(L1, tx, jj) * rc;
  }
}

enum { WC_RESID = 0, WC_RESTRICT = 1, WC_PROLONG = 2, WC_POST = 3 };

// one coarse-level pass over the whole grid (levels too large for one workgroup)
template <typename VT, int KIND>
__global__ __launch_bounds__(WIDE_BX) void k_w_cpass(MGGeom mg, WidePtrs w, int l, VT om, VT air) {
  if (w.sc->done) return;
  const int nthr = gridDim.x * blockDim.x, me = blockIdx.x * blockDim.x + threadIdx.x;
  VT* reg = (VT*)w.mgreg;
  const VT* ctab = (const VT*)w.ctab;
  const CLev<VT> F = clev<VT>(mg, l, reg, ctab, nthr, air);
  if (KIND == WC_RESID) {
    c_resid(F, me, nthr);
  } else if (KIND == WC_RESTRICT) {
    const CLev<VT> Cc = clev<VT>(mg, l + 1, reg, ctab, nthr, air);
    c_restrict(F, Cc, om, l + 1 == mg.nlev, me, nthr);
  } else if (KIND == WC_PROLONG) {
    const CLev<VT> Cc = clev<VT>(mg, l + 1, reg, ctab, nthr, air);
    c_prolong(F, l + 1 == mg.nlev ? Cc.Z : Cc.T, Cc.np, me, nthr);
  } else {
    c_post(F, om, me, nthr);
  }
}

// the coarse levels from lt down (one workgroup): the shifted hierarchy sub
// has sub.lv[1] = level lt
template <typename VT>
__global__ __launch_bounds__(1024) void k_w_ctail(MGGeom sub, WidePtrs w, VT om, VT air) {
  if (w.sc->done) return;
  (void)coarse_cycle<VT, 1024, true>(sub, (VT*)w.mgreg, (const VT*)w.ctab, om, threadIdx.x, air);
}

// Z += D^{1/2} P z_1
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_prolong(Geom g, MGGeom mg, WidePtrs w, VT air) {
  if (w.sc->done) return;
  WIDE_NODE;
  if (!act) return;
  const CLev<VT> L1 = clev<VT>(mg, 1, (VT*)w.mgreg, (const VT*)w.ctab, 64, air);
  const VT* z1 = mg.nlev == 1 ? L1.Z : L1.T;
  const double d_air = 1.0 / sqrt(4.0 * g.nu_air);
  ((VT*)w.Z)[nr.gi] += prolong_at(z1, L1.np, i, j) * wide_dinv<VT>(g, (VT*)w.tDi, d_air, i, j, nr);
}

// post-smoothing T = Z + om (R - A Z); partials r.T and r.r
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_post(Geom g, WidePtrs w, VT om) {
  if (w.sc->done) return;
  WIDE_NODE;
  double v[2] = {0.0, 0.0};
  if (act) {
    const VT* Z = (const VT*)w.Z;
    const VT r = ((const VT*)w.R)[nr.gi], z = Z[nr.gi];
    const VT zn = z + om * (r - stencil_scaled<VT>(g, Z, (VT*)w.tE, (VT*)w.tN, (VT*)w.tNE, nr));
    ((VT*)w.T)[nr.gi] = zn;
    v[0] = (double)(r * zn);
    v[1] = (double)(r * r);
  }
  wide_partial<2>(v, w.part);
}

// Jacobi preconditioner in place of the V-cycle: the system is already scaled
// to unit diagonal, so z = r (into T); partials r.z and r.r
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_jz(Geom g, WidePtrs w) {
  if (w.sc->done) return;
  WIDE_NODE;
  double v[2] = {0.0, 0.0};
  if (act) {
    const VT r = ((const VT*)w.R)[nr.gi];
    ((VT*)w.T)[nr.gi] = r;
    v[0] = (double)(r * r);
    v[1] = v[0];
  }
  wide_partial<2>(v, w.part);
}

// p = z + beta p, q = A z + beta q (z in T); partial p.q
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_pq(Geom g, WidePtrs w) {
  if (w.sc->done) return;
  WIDE_NODE;
  double v[1] = {0.0};
  if (act) {
    const VT b_ = (VT)w.sc->beta;
    const bool first = w.sc->it == 1;
    const VT* Zt = (const VT*)w.T;
    VT* Pv = (VT*)w.P;
    VT* Qv = (VT*)w.Q;
    const VT az = stencil_scaled<VT>(g, Zt, (VT*)w.tE, (VT*)w.tN, (VT*)w.tNE, nr);
    const VT p = first ? Zt[nr.gi] : Zt[nr.gi] + b_ * Pv[nr.gi];
    const VT q = first ? az : az + b_ * Qv[nr.gi];
    Pv[nr.gi] = p;
    Qv[nr.gi] = q;
    v[0] = (double)(p * q);
  }
  wide_partial<1>(v, w.part);
}

// y += alpha p, r -= alpha q
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_yr(Geom g, WidePtrs w) {
  if (w.sc->done) return;
  WIDE_NODE;
  if (!act) return;
  const VT a_ = (VT)w.sc->alpha;
  ((VT*)w.Y)[nr.gi] += a_ * ((const VT*)w.P)[nr.gi];
  ((VT*)w.R)[nr.gi] -= a_ * ((const VT*)w.Q)[nr.gi];
}

// x += D^{-1/2} y
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_xupd(Geom g, WidePtrs w) {
  WIDE_NODE;
  if (!act) return;
  const double d_air = 1.0 / sqrt(4.0 * g.nu_air);
  w.Xv[nr.gi] += (double)wide_dnode<VT>(g, (VT*)w.tD, d_air, i, j, nr) * (double)((const VT*)w.Y)[nr.gi];
}

// partial x^T M x over the lookup region
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_qoi(Geom g, WidePtrs w) {
  WIDE_NODE;
  double v[1] = {0.0};
  if (act && nr.inL) v[0] = w.Xv[nr.gi] * M_apply(g, w.tab, w.Xv, nr);
  wide_partial<1>(v, w.part);
}

// a += x; next start 2 x - x_prev; x_prev = x
template <typename VT>
__global__ __launch_bounds__(WIDE_BX) void k_w_state(Geom g, WidePtrs w) {
  WIDE_NODE;
  if (!act) return;
  const double d = w.Xv[nr.gi];
  w.Av[nr.gi] += d;
  w.Xv[nr.gi] = 2.0 * d - w.Xp[nr.gi];
  w.Xp[nr.gi] = d;
}

__global__ void k_w_finish(Geom g, WidePtrs w, double q_scale, double* q_out, double* a_out) {
  const int n = g.n;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n * n; idx += gridDim.x * blockDim.x) {
    const int gi = (idx / n + 1) * g.P + idx % n + 1;
    if (a_out) a_out[gi] = w.Av[gi];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && q_out) *q_out = w.sc->qsum * q_scale;
}

// ---- host launchers ----
static dim3 wide_grid(const WideCtx& c) { return dim3((c.g.n + WIDE_BX - 1) / WIDE_BX, c.g.n); }

// 1-D grid with one thread per node of coarse level l (2^s columns >= n_l)
static int wide_cblocks(const MGGeom& mg, int l) {
  int s = 0;
  while ((1 << s) < mg.lv[l].n) ++s;
  const long t = (long)(2 << s) * mg.lv[l].n;
  return (int)((t + WIDE_BX - 1) / WIDE_BX);
}

template <typename VT>
static hipError_t wide_setup_t(const WideCtx& c, double inv_dt, const double* a_init, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  hipLaunchKernelGGL((k_w_setup<VT>), dim3(1), dim3(1024), 0, st, c.g, c.mg, c.sv, c.w, inv_dt, a_init);
  return hipGetLastError();
}
template <typename VT>
static hipError_t wide_rhs_t(const WideCtx& c, double Jt, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  hipLaunchKernelGGL((k_w_rhs<VT>), wide_grid(c), dim3(WIDE_BX), 0, st, c.g, c.w, Jt);
  hipLaunchKernelGGL((k_w_reduce<WRED_RHS, 1>), dim3(1), dim3(1024), 0, st, c.w, c.sv, c.nblk, 0.0);
  return hipGetLastError();
}
template <typename VT>
static hipError_t wide_resid_t(const WideCtx& c, double inv_dt, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  hipLaunchKernelGGL((k_w_resid<VT>), wide_grid(c), dim3(WIDE_BX), 0, st, c.g, c.w, inv_dt);
  hipLaunchKernelGGL((k_w_reduce<WRED_RES, 1>), dim3(1), dim3(1024), 0, st, c.w, c.sv, c.nblk, 0.0);
  return hipGetLastError();
}
template <typename VT>
static hipError_t wide_iteration_t(const WideCtx& c, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  const VT om = (VT)c.sv.mg_omega, air = (VT)c.air;
  const dim3 gr = wide_grid(c), bl(WIDE_BX);
  if (c.mg.nlev == 0) {  // Jacobi-preconditioned CG
    hipLaunchKernelGGL((k_w_jz<VT>), gr, bl, 0, st, c.g, c.w);
    hipLaunchKernelGGL((k_w_reduce<WRED_RZ, 2>), dim3(1), dim3(1024), 0, st, c.w, c.sv, c.nblk, 0.0);
    hipLaunchKernelGGL((k_w_pq<VT>), gr, bl, 0, st, c.g, c.w);
    hipLaunchKernelGGL((k_w_reduce<WRED_PQ, 1>), dim3(1), dim3(1024), 0, st, c.w, c.sv, c.nblk, 0.0);
    hipLaunchKernelGGL((k_w_yr<VT>), gr, bl, 0, st, c.g, c.w);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_w_pre<VT>), gr, bl, 0, st, c.g, c.w, om);
  hipLaunchKernelGGL((k_w_restrict1<VT>), dim3(wide_cblocks(c.mg, 1)), bl, 0, st, c.g, c.mg, c.w, om, air);
  for (int l = 1; l < c.lt; ++l) {
    hipLaunchKernelGGL((k_w_cpass<VT, WC_RESID>), dim3(wide_cblocks(c.mg, l)), bl, 0, st, c.mg, c.w, l, om, air);
    hipLaunchKernelGGL((k_w_cpass<VT, WC_RESTRICT>), dim3(wide_cblocks(c.mg, l + 1)), bl, 0, st, c.mg, c.w, l, om,
                       air);
  }
  hipLaunchKernelGGL((k_w_ctail<VT>), dim3(1), dim3(1024), 0, st, c.sub, c.w, om, air);
  for (int l = c.lt - 1; l >= 1; --l) {
    hipLaunchKernelGGL((k_w_cpass<VT, WC_PROLONG>), dim3(wide_cblocks(c.mg, l)), bl, 0, st, c.mg, c.w, l, om, air);
    hipLaunchKernelGGL((k_w_cpass<VT, WC_POST>), dim3(wide_cblocks(c.mg, l)), bl, 0, st, c.mg, c.w, l, om, air);
  }
  hipLaunchKernelGGL((k_w_prolong<VT>), gr, bl, 0, st, c.g, c.mg, c.w, air);
  hipLaunchKernelGGL((k_w_post<VT>), gr, bl, 0, st, c.g, c.w, om);
  hipLaunchKernelGGL((k_w_reduce<WRED_RZ, 2>), dim3(1), dim3(1024), 0, st, c.w, c.sv, c.nblk, 0.0);
  hipLaunchKernelGGL((k_w_pq<VT>), gr, bl, 0, st, c.g, c.w);
  hipLaunchKernelGGL((k_w_reduce<WRED_PQ, 1>), dim3(1), dim3(1024), 0, st, c.w, c.sv, c.nblk, 0.0);
  hipLaunchKernelGGL((k_w_yr<VT>), gr, bl, 0, st, c.g, c.w);
  return hipGetLastError();
}
template <typename VT>
static hipError_t wide_xupd_t(const WideCtx& c, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  hipLaunchKernelGGL((k_w_xupd<VT>), wide_grid(c), dim3(WIDE_BX), 0, st, c.g, c.w);
  return hipGetLastError();
}
template <typename VT>
static hipError_t wide_end_step_t(const WideCtx& c, double inv_dt, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  hipLaunchKernelGGL((k_w_qoi<VT>), wide_grid(c), dim3(WIDE_BX), 0, st, c.g, c.w);
  hipLaunchKernelGGL((k_w_reduce<WRED_QOI, 1>), dim3(1), dim3(1024), 0, st, c.w, c.sv, c.nblk, inv_dt);
  hipLaunchKernelGGL((k_w_state<VT>), wide_grid(c), dim3(WIDE_BX), 0, st, c.g, c.w);
  return hipGetLastError();
}

#define WIDE_DISPATCH(fn, ...) \
  return c.sv.precision == MQ_PREC_FP64 ? fn<double>(c, __VA_ARGS__) : fn<float>(c, __VA_ARGS__)
hipError_t wide_setup(const WideCtx& c, double inv_dt, const double* a_init, hipStream_t st) {
  WIDE_DISPATCH(wide_setup_t, inv_dt, a_init, st);
}
hipError_t wide_rhs(const WideCtx& c, double Jt, hipStream_t st) { WIDE_DISPATCH(wide_rhs_t, Jt, st); }
hipError_t wide_resid(const WideCtx& c, double inv_dt, hipStream_t st) { WIDE_DISPATCH(wide_resid_t, inv_dt, st); }
hipError_t wide_iteration(const WideCtx& c, hipStream_t st) { WIDE_DISPATCH(wide_iteration_t, st); }
hipError_t wide_xupd(const WideCtx& c, hipStream_t st) { WIDE_DISPATCH(wide_xupd_t, st); }
hipError_t wide_end_step(const WideCtx& c, double inv_dt, hipStream_t st) { WIDE_DISPATCH(wide_end_step_t, inv_dt, st); }
#undef WIDE_DISPATCH
hipError_t wide_finish(const WideCtx& c, double q_scale, double* q_out, double* a_out, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  hipLaunchKernelGGL(k_w_finish, dim3(256), dim3(256), 0, st, c.g, c.w, q_scale, q_out, a_out);
  return hipGetLastError();
}
int wide_blocks(const Geom& g) { return ((g.n + WIDE_BX - 1) / WIDE_BX) * g.n; }

}  // namespace mq
