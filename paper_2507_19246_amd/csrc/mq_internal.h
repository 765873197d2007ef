// Internal declarations shared by the host orchestration and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mq.h"

namespace mq {

// Geometry of one structured mesh as seen by the kernels.
//
// Interior nodes (i, j), 0 <= i, j < n = N - 2, are the unknowns.  FP64 state
// vectors live on the full N x N grid (boundary ring = the Dirichlet zeros)
// with row pitch P: node (i, j) sits at (j + 1) * P + (i + 1).
//
// Only rows of nodes near the conductor depend on the sample.  The "box"
// [bx0, bx1) x [by0, by1) is the bounding rectangle of the interior nodes that
// touch a conductor element, grown by one node; every matrix entry owned by a
// node outside the box (its E, N, NE couplings and its diagonal) is the air
// value.  Stencil tables cover the region R = [bx0-1, bx1+1) x [by0-1, by1+1)
// (RW x RH nodes, air constants outside the box), so a node in the lookup
// region L = [bx0, bx1+1) x [by0, by1+1) reads all six of its couplings
// (own E, N, NE; W = E(i-1, j), S = N(i, j-1), SW = NE(i-1, j-1)) from tables,
// and every other node uses the constant air stencil.
struct Geom {
  int N, n, P;
  int bx0, bx1, by0, by1;
  int lx1, ly1;   // lookup region upper bounds (exclusive, clipped to n)
  int RW, RH;     // table region size
  double h, h2, nu_air;
};

// FP64 coefficient planes of one sample over the table region R, followed by
// the sample's nonlinear curve coefficients k1', k2', k3' (and one pad).
enum { T_MC = 0, T_ME, T_MN, T_MNE, T_KC, T_KE, T_KN, T_NPLANES };
__host__ __device__ inline size_t tab_stride(const Geom& g) { return (size_t)T_NPLANES * g.RW * g.RH + 4; }
// Resident workgroup shape: cw columns x ns slices of sh rows (cw * ns
// threads, sh rows per thread), tp = table pitch in LDS.
struct ResCfg {
  int cw, sh, ns, tp;
};
// The resident shape for this mesh and tile (1: 16 rows per thread, 2: 32 rows
// per thread in 512-thread workgroups where 64..127 interior nodes per side);
// false where the resident path does not apply.
__host__ __device__ inline bool pick_resident(const Geom& g, int tile, ResCfg* c) {
  if (g.n <= 31) {
    *c = {32, 16, 2, 32};
  } else if (g.n <= 63) {
    *c = {64, 16, 4, 64};
  } else if (g.n <= 127) {
    *c = tile == 2 ? ResCfg{128, 32, 4, 64} : ResCfg{128, 16, 8, 64};
  } else {
    return false;
  }
  return g.n <= c->sh * c->ns && g.RW <= c->tp;
}
// doubles of one thread-private [row][thread] plane of the resident kernel
// (multigrid iterate, per-node D^{-1/2}): one element per (row, thread) of the
// largest resident shape this mesh can take (either tile), and at least a
// full-grid plane.  On small meshes the workgroup spans more (row, thread)
// pairs than the grid has nodes.
__host__ __device__ inline size_t res_plane_doubles(const Geom& g) {
  size_t need = (size_t)g.N * g.P;
  for (int tile = 1; tile <= 2; ++tile) {
    ResCfg c;
    if (pick_resident(g, tile, &c)) {
      const size_t rt = (size_t)c.sh * c.cw * c.ns;
      if (rt > need) need = rt;
    }
  }
  return need;
}
// doubles per slot of the time-stepping work buffer: state a, increment x,
// right-hand side b (full-grid planes), the VT iterate plane (thread-private),
// previous increment, Picard increment (full-grid), the per-node D^{-1/2}
// plane (thread-private), then the instance's FP64 tables (planes + k1', k2',
// k3')
// (rounded up to 256 bytes, so that the streaming vectors after the slots
// start 16-byte aligned)
__host__ __device__ inline size_t ie_work_doubles(const Geom& g) {
  const size_t d = 5 * (size_t)g.N * g.P + 2 * res_plane_doubles(g) + (size_t)T_NPLANES * g.RW * g.RH + 3;
  return (d + 31) & ~(size_t)31;
}

// Element data over the cells that touch the box: full-grid cells
// [bx0, bx1 + 1) x [by0, by1 + 1), two triangles per cell
// (t = 0: {(I,J), (I+1,J), (I+1,J+1)}, t = 1: {(I,J), (I+1,J+1), (I,J+1)}).
struct CellRegion {
  int cx0, cy0, cw, ch;  // first cell (full-grid cell coords) and extent
};

// One time-integration instance (a sample on one time grid, or one Parareal
// slice / coarse chain).
struct Inst {
  const double* tab;     // FP64 tables of the sample [T_NPLANES][RH*RW]
  const double* src;     // J(t_k) by global step index k for this dt
  const double* a_init;  // full-grid initial state or null (zeros)
  double* a_out;         // full-grid final state or null
  double* q_out;         // receives q_scale * sum_k d_k^T M d_k / dt
  double q_scale;
  int* stat;             // [STAT_N]: inner iterations, sweeps, max inner per step, flags,
                         // device wall-clock start (lo, hi) and end (lo, hi), eight
                         // phase-time counters (units of 16 wall-clock ticks), Picard
                         // iterations
  double dt;
  int n_steps;           // steps per chain segment
  int k0;                // global index of the first step
  // Parareal coarse-chain mode (n_chain > 0): run segments s = 0..n_chain-1
  // from chain_u[s] ... see kernels for the exact recurrence.
  int n_chain;
  double* const* chain_u;       // U_n full-grid states (in/out)
  const double* const* chain_f; // F_n fine end states
  double* const* chain_c;       // C_old_n coarse values (in/out)
  int sample;                   // sample index (nonlinear coefficients)
  int group;                    // latency group (host bookkeeping: one per sample)
  // Resumable runs (null: none): full-grid start of the next increment solve,
  // [0, FS); previous increment, [FS, 2 FS); unscaled running QoI sum, [2 FS].
  // Written at the end of the launch; read at its start when carry_in != 0,
  // so a run split into launches at any step gives the unsplit result bit for bit.
  double* carry;
  int carry_in;
  // Pieces of one instance in one launch (resident path): a piece with
  // dep_wait waits until that flag is set before it reads a_init and carry;
  // one with dep_done sets that flag once its a_out and carry are written.
  const int* dep_wait;
  int* dep_done;
  // Completion record in coherent pinned host memory (null: none), written
  // by the entry's last action so that the host sees Q as soon as it exists.
  struct HostDone* host_done;
  // Parareal in one persistent launch (para null: none).  Every entry may wait
  // (dep_wait) only on flags set by entries queued before it, so every wait ends.
  const struct ParaCtl* para;
  int para_iter;    // iteration j of this entry (0: the initial coarse pass)
  int para_chain;   // 1: coarse chain of iteration j (j >= 1: decides, then corrects)
  // chain j >= 1: the interfaces n = j..M-1 (fine end state F_n^(j), previous
  // U_n^(j-1)) and the done flags of the fine slices n = j..M
  const double* const* jump_f;
  const double* const* jump_u;
  const int* const* jump_wait;
  int n_jump;       // M - j
  double* u_first;        // U_j <- F_j^(j) before the correction chain
  const double* f_first;
  int* first_done;        // set once U_j is written
  int* const* seg_done;   // per chain segment: set once its U_n is written
};

// Control record of one Parareal launch (device memory).
struct ParaCtl {
  int* K;        // [S]: iteration at which the sample stopped (0 while it runs)
  double* J;     // [S][kcap]: largest relative interface jump of each iteration
  int* flags;    // [S]: FLAG_PARAREAL_KMAX, FLAG_FAILED
  int* abort;    // set by a wait that timed out: later waits give up at once
  double tol;
  int fixed_k, kcap;
};

// Longest wait of a Parareal entry for its input, 60 s of the device wall clock
// (chains of a long run legitimately take seconds); past it the entry runs
// flagged FLAG_FAILED.
constexpr unsigned long long PARA_WAIT_TICKS = 6000000000ull;

// One launch entry's completion as the host sees it: the kernel stores q and
// flags, then sets done with a system-scope release store.
struct HostDone {
  double q;
  int flags;
  int done;
};

// Longest wait of a piece for its predecessor, 5 s of the device wall clock
// (100 MHz), far above one piece's run time; past it the piece runs flagged
// FLAG_FAILED instead of waiting on.
constexpr unsigned long long DEP_WAIT_TICKS = 500000000ull;

// Geometric multigrid hierarchy of the resident path (fine interior n = 2^k - 1;
// level l+1 has (n_l - 1)/2 nodes per side, coarse node c sits at fine 2c + 1).
// Each coarse level keeps Galerkin 7-point tables (C, E, N, NE planes, pitch
// RW) over its box +- 1 ring; its vectors r, z, t (n_l^2 each, no halo) sit
// at vec_off inside the LDS region shared with the fine exchange grid.
constexpr int MG_MAX_LEVELS = 12;
struct MGLevel {
  int n, bx0, bx1, by0, by1, lx1, ly1, RW, RH, tab_off, vec_off;
};
struct MGGeom {
  int nlev;          // coarse levels (lv[1..nlev]); 0 = multigrid unavailable
  int region_elems;  // LDS elements of the shared region (fine grid or coarse vectors)
  int ctab_elems;    // LDS elements of all coarse tables
  MGLevel lv[MG_MAX_LEVELS];
};
bool build_mg(const Geom& g, int lp, MGGeom* mg);

// Quad tables of the streaming kernel's float4 passes: the scaled E, N and NE
// coefficients and D^{1/2} of the table region, laid out so that the four
// nodes of a quad (first column i0 = 0 mod 4) are one aligned float4.  Columns
// qx0 .. qx0 + qw - 1 (qx0 = 4 floor(bx0 / 4) - 4, qw = 0 mod 4) cover every
// quad that meets the lookup columns [bx0, lx1) plus the column left of it;
// rows by0 - 2 .. ly1 - 1 (row r = j - by0 + 2; row 0 is not read).
// Positions outside the table region hold the air values (-1/4, -1/4, 0;
// D^{1/2} of air off the box).  A quad outside the lookup region reads no
// table (air constants).
struct QTab {
  int qx0, qw, rows;
};
__host__ __device__ inline QTab qtab_geom(const Geom& g) {
  QTab q;
  q.qx0 = ((g.bx0 >> 2) << 2) - 4;
  const int hi = g.lx1 > g.bx0 ? (((g.lx1 - 1) >> 2) << 2) + 4 : q.qx0 + 8;
  q.qw = hi - q.qx0 < 8 ? 8 : hi - q.qx0;
  q.rows = g.RH + 1;
  return q;
}

// Quad-table base of the quad (i0, j) inside the lookup region, else -1.
__host__ __device__ inline int qbase(const Geom& g, const QTab& q, int i0, int j) {
  const bool in = j >= g.by0 && j < g.ly1 && i0 + 3 >= g.bx0 && i0 < g.lx1;
  return in ? (j - g.by0 + 2) * q.qw + (i0 - q.qx0) : -1;
}

struct Solver {
  int precond;     // 0 = Jacobi scaling only, 1 = multigrid V(1,1) (resident path)
  double mg_omega; // damped-Jacobi weight of the multigrid smoother
  int precision;   // MQ_PREC_*
  double tol, inner_rtol;
  int max_iter, max_sweeps;
  // nonlinear material
  int nonlinear;
  double picard_tol;
  int picard_max;
  int tile;        // resident workgroup shape (host-side dispatch)
  int mg_levels;   // coarse levels in use (0: all)
  int mg_coarse_sweeps;  // damped-Jacobi sweeps at the coarsest level in use
  int mg_block_min;      // coarse levels with at least this many nodes per side use the whole workgroup
  int para;              // 1: the launch holds one-launch Parareal entries (kernels with the entry prologue)
  int lds_limit = 0;     // LDS bytes one workgroup may use
  int lds_lev = 0;       // streaming multigrid: first coarse level held in LDS (0: none; set by the launcher)
};

enum { FLAG_NOT_CONVERGED = 1, FLAG_FAILED = 2, FLAG_PICARD_CAP = 4, FLAG_PARAREAL_KMAX = 8 };
// Coarse levels in use (mg_levels caps them).
__host__ __device__ inline int stream_levels_used(const MGGeom& mg, const Solver& sv) {
  return (sv.mg_levels > 0 && sv.mg_levels < mg.nlev) ? sv.mg_levels : mg.nlev;
}
// Elements of levels la..lz's vectors / tables (contiguous in the layout).
__host__ __device__ inline int lds_vec_elems(const MGGeom& mg, int la, int lz) {
  const MGLevel& z = mg.lv[lz];
  return z.vec_off + 3 * (z.n + 2) * (z.n + 2) - mg.lv[la].vec_off;
}
__host__ __device__ inline int lds_tab_elems(const MGGeom& mg, int la, int lz) {
  const MGLevel& z = mg.lv[lz];
  return z.tab_off + 5 * z.RW * z.RH - mg.lv[la].tab_off;
}

// First coarse level the streaming kernel keeps in LDS: the largest tail of
// the levels in use that fits `budget` bytes, starting at level 2 or deeper,
// every level above it a whole-workgroup level (0: none fits).
inline int stream_lds_level(const MGGeom& mg, const Solver& sv, size_t vt, size_t budget, size_t* bytes) {
  *bytes = 0;
  const int lz = stream_levels_used(mg, sv);
  for (int la = 2; la <= lz; ++la) {
    if (mg.lv[la - 1].n < sv.mg_block_min) return 0;
    const size_t b = (size_t)(lds_vec_elems(mg, la, lz) + lds_tab_elems(mg, la, lz)) * vt;
    if (b <= budget) {
      *bytes = b;
      return la;
    }
  }
  return 0;
}

// bits that make a call return MQ_WARN_NOT_CONVERGED
constexpr int FLAG_WARN = FLAG_NOT_CONVERGED | FLAG_FAILED | FLAG_PICARD_CAP;
enum { STAT_N = 17 };

// Wide path (one instance over the whole device): solver scalars in device
// memory, the instance's buffers, and the launch context.
struct WideScal {
  double bb, rr, rho, beta, alpha, stop, floor_fac, qsum;
  int it, done, conv, flags, it_total, sweeps;
};
struct WidePtrs {
  double *Av, *Xv, *Bv, *Xp;                 // FP64 full grid
  void *R, *Y, *P, *Z, *T, *Q;               // VT full grid
  void *tE, *tN, *tNE, *tD, *tDi, *mgreg, *ctab;
  double* part;                              // block partials [2][blocks]
  WideScal* sc;
  const double* tab;                         // the sample's FP64 tables
  const double* S;
};
struct WideCtx {
  Geom g;
  MGGeom mg;   // full hierarchy
  MGGeom sub;  // levels lt..nlev renumbered from 1 (run by one workgroup)
  Solver sv;
  WidePtrs w;
  int lt;      // first coarse level handled by one workgroup
  int nblk;    // blocks of a fine-level pass
  double air;  // air diagonal of the coarse levels (4 nu_air)
};
hipError_t wide_setup(const WideCtx& c, double inv_dt, const double* a_init, hipStream_t st);
hipError_t wide_rhs(const WideCtx& c, double Jt, hipStream_t st);
hipError_t wide_resid(const WideCtx& c, double inv_dt, hipStream_t st);
hipError_t wide_iteration(const WideCtx& c, hipStream_t st);
hipError_t wide_xupd(const WideCtx& c, hipStream_t st);
hipError_t wide_end_step(const WideCtx& c, double inv_dt, hipStream_t st);
hipError_t wide_finish(const WideCtx& c, double q_scale, double* q_out, double* a_out, hipStream_t st);
int wide_blocks(const Geom& g);

// Launch helpers implemented in the .hip translation units.
// tile: resident workgroup shape (1: 16 rows per thread, 2: 32 rows per thread)
int resident_supported(const Geom& g, const MGGeom* mg, int precision, int lds_limit, int* lds_bytes, int tile);
int resident_lp(const Geom& g, int tile);
int ie_block_threads(const Geom& g, int path, int tile);
hipError_t launch_assemble(const Geom& g, const CellRegion& cr, const uint8_t* cond,
                           const double* kltab, int n_modes, int material, const double* xi,
                           int n_xi, int n_samples, const double* mat_params, double* tables,
                           hipStream_t st);
hipError_t launch_ie(const Geom& g, const MGGeom& mg, const Solver& sv, const Inst* insts, int n_inst,
                     int* counter, double* work, int n_slots, int max_grid, const double* S, int path,
                     int precision, const CellRegion& cr, const uint8_t* cond,
                     const double* nl_params, int* grid_out, int* block_out, hipStream_t st);
hipError_t launch_apply(const Geom& g, int which, double dt, const double* tables, int n,
                        const double* x, double* y, hipStream_t st);
hipError_t launch_to_interior(const Geom& g, int n, const double* const* full, double* out,
                              hipStream_t st);
hipError_t launch_to_full(const Geom& g, int n, const double* in, double* const* full,
                          hipStream_t st);
hipError_t launch_level_stats(int n_levels, const int* n_per_level, const double* const* qf,
                              const double* const* qc, double* out, hipStream_t st);
// Work queue of the next persistent launch (counter: 4 ints): entries [0,
// n_first) form queue 0, the rest queue 1; workgroups below grid_first start
// on queue 0.
hipError_t launch_queue_init(int* counter, int n_first, int grid_first, hipStream_t st);
// Device address of the allocation-free call's workspace on `device` (looked
// up once per device with that device current; noalloc.hip).
hipError_t noalloc_workspace(int device, char** ptr);
// Parareal (one-launch run): Q per sample from the per-iteration slice sums
// q [S][kcap][M] and the stopping iterations K [S] (device int32)
hipError_t launch_para_qoi(const double* qb, const int* K, int kcap, int M, int n_samples, double T, double* q,
                           hipStream_t st);
// Row-sum lumping of the mass planes of n_samples tables (mass = MQ_MASS_LUMPED).
hipError_t launch_lump_mass(const Geom& g, int n_samples, double* tables, hipStream_t st);
hipError_t launch_fill_zero(double* p, size_t n, hipStream_t st);
hipError_t launch_fill_zero_i(int* p, size_t n, hipStream_t st);
hipError_t launch_check_finite(const double* x, size_t n, int* bad, hipStream_t st);
int ie_slots_per_cu(const Geom& g, const MGGeom* mg, int path, int precision, int tile);
// VT elements per slot of the streaming kernel (mg: its multigrid hierarchy, or null)
size_t stream_vwork_elems(const Geom& g, const MGGeom* mg);

}  // namespace mq
