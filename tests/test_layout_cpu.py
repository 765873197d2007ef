"""Host-side check of the resident work-slot layout: for every mesh size and
both resident workgroup shapes, the thread-private [row][thread] planes hold
one element per (row, thread) of the shape the launcher picks, and at least a
full-grid plane (the plane size and the launch shape come from one function,
and this pins that they stay consistent)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_19246_amd", "csrc")

PROG = r'''
#include <cstdio>
#include "setup.h"
int main() {
  int bad = 0, checked = 0;
  for (int n = 3; n <= 300; ++n) {
    mq_problem_desc d{};
    d.n_nodes = n;
    d.material = MQ_MAT_KL;
    d.conductor[0] = 0.3; d.conductor[1] = 0.7; d.conductor[2] = 0.3; d.conductor[3] = 0.7;
    d.strip[0] = 0.1; d.strip[1] = 0.2;
    d.J0 = 1e6; d.freq = 50; d.sigma0 = 5e6; d.nu_cond = 795.7747154594767; d.nu_air = 795774.7154594767;
    d.n_modes = 8; d.corr_len = 0.2; d.s_kl = 0.3;
    mq::HostMesh hm = mq::build_host_mesh(d);
    const mq::Geom& g = hm.g;
    const size_t plane = mq::res_plane_doubles(g);
    if (plane < (size_t)g.N * g.P) { std::printf("n=%d plane below a full grid\n", n); ++bad; }
    for (int tile = 1; tile <= 2; ++tile) {
      mq::ResCfg c;
      if (!mq::pick_resident(g, tile, &c)) continue;
      ++checked;
      if ((size_t)c.sh * c.cw * c.ns > plane) { std::printf("n=%d tile=%d rows x threads above the plane\n", n, tile); ++bad; }
      if (g.n > c.sh * c.ns || g.n > c.cw) { std::printf("n=%d tile=%d shape does not cover the mesh\n", n, tile); ++bad; }
    }
  }
  std::printf("checked %d bad %d\n", checked, bad);
  return bad ? 1 : 0;
}
'''


def test_resident_planes_hold_every_picked_shape(tmp_path):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "layout.cpp"
    src.write_text(PROG)
    exe = tmp_path / "layout"
    inc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")
    cmd = [hipcc, "-x", "c++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", f"-I{inc}", f"-I{CSRC}",
           str(src), os.path.join(CSRC, "setup.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-3000:]
    out = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert out.returncode == 0, out.stdout
    assert "checked" in out.stdout and " bad 0" in out.stdout


QUAD = r"""
#include <cstdio>
#include <cstdlib>
#include "setup.h"
// Host check of the streaming kernel's float4 passes: for every mesh with a
// multigrid hierarchy and many conductor boxes, every quad-table position a
// quad reads lies inside the quad tables, in its own row, and is the same
// table-region position that the scalar stencil reads for that node; and the
// LDS tail of coarse levels fits the budget.
int main() {
  int bad = 0, quads = 0, meshes = 0;
  const int Ns[] = {5, 9, 17, 33, 65, 129, 257, 513, 1025};
  srand(7);
  for (int N : Ns) {
    for (int rep = 0; rep < 24; ++rep) {
      mq_problem_desc d{};
      d.n_nodes = N;
      d.material = MQ_MAT_KL;
      double x0 = 0.05 + 0.5 * (rand() / (double)RAND_MAX), y0 = 0.05 + 0.5 * (rand() / (double)RAND_MAX);
      double wx = 0.02 + 0.4 * (rand() / (double)RAND_MAX), wy = 0.02 + 0.4 * (rand() / (double)RAND_MAX);
      if (rep == 0) { x0 = 0.3; wx = 0.4; y0 = 0.3; wy = 0.4; }
      d.conductor[0] = x0; d.conductor[1] = x0 + wx; d.conductor[2] = y0; d.conductor[3] = y0 + wy;
      d.strip[0] = 0.1; d.strip[1] = 0.2;
      d.J0 = 1e6; d.freq = 50; d.sigma0 = 5e6; d.nu_cond = 795.7747154594767; d.nu_air = 795774.7154594767;
      d.n_modes = 8; d.corr_len = 0.2; d.s_kl = 0.3;
      mq::HostMesh hm = mq::build_host_mesh(d);
      const mq::Geom& g = hm.g;
      ++meshes;
      if (g.P != g.N + 3) { std::printf("N=%d pitch %d is not N + 3\n", N, g.P); ++bad; continue; }
      const mq::QTab q = mq::qtab_geom(g);
      if (q.qw % 4 != 0 || q.qx0 % 4 != 0) { std::printf("N=%d quad table not aligned\n", N); ++bad; }
      const int n = g.n, nq = (n + 1) / 4;
      for (int j = 0; j < n; ++j)
        for (int qi = 0; qi < nq; ++qi) {
          const int i0 = 4 * qi;
          const int b = mq::qbase(g, q, i0, j);
          bool any_in = false;
          for (int k = 0; k < 4; ++k) {
            const int i = i0 + k;
            if (i < n && i >= g.bx0 && i < g.lx1 && j >= g.by0 && j < g.ly1) any_in = true;
          }
          if (any_in && b < 0) { std::printf("N=%d quad (%d,%d) holds a lookup node but reads no table\n", N, i0, j); ++bad; }
          if (b < 0) continue;
          ++quads;
          const int r = b / q.qw, c = b % q.qw;
          // float4 rows at b and b - qw, single loads at b - 1 and b - qw - 1
          if (r < 2 || r >= q.rows || c < 1 || c + 3 >= q.qw) {
            std::printf("N=%d quad (%d,%d): base row %d col %d outside the tables\n", N, i0, j, r, c); ++bad;
          }
          // same positions as the scalar stencil's table reads (t, t - 1, t - RW, t - RW - 1)
          for (int k = 0; k < 4; ++k) {
            const int i = i0 + k;
            if (!(i < n && i >= g.bx0 && i < g.lx1 && j >= g.by0 && j < g.ly1)) continue;
            const int ci = i - g.bx0 + 1, cj = j - g.by0 + 1;  // table-region position
            const int qi_ = q.qx0 + (c + k), qj_ = g.by0 - 2 + r;  // node of the quad-table position
            if (qi_ != i || qj_ != j || ci < 1 || ci >= g.RW || cj < 1 || cj >= g.RH) {
              std::printf("N=%d node (%d,%d): quad position (%d,%d)\n", N, i, j, qi_, qj_); ++bad;
            }
          }
        }
      // LDS tail of the coarse levels (streaming, mixed precision)
      mq::MGGeom mg;
      if (mq::build_mg(g, 0, &mg)) {
        mq::Solver sv{};
        sv.mg_block_min = 15;
        const size_t budget = 160 * 1024 - 4096;
        size_t bytes = 0;
        const int la = mq::stream_lds_level(mg, sv, sizeof(float), budget, &bytes);
        if (la > 0 && (bytes > budget || la < 2 || la > mg.nlev || mg.lv[la - 1].n < 15)) {
          std::printf("N=%d LDS tail from level %d: %zu bytes\n", N, la, bytes); ++bad;
        }
        if (la > 0 && bytes != (size_t)(mq::lds_vec_elems(mg, la, mg.nlev) + mq::lds_tab_elems(mg, la, mg.nlev)) * 4) {
          std::printf("N=%d LDS bytes mismatch\n", N); ++bad;
        }
      }
    }
  }
  std::printf("meshes %d quads %d bad %d\n", meshes, quads, bad);
  return bad ? 1 : 0;
}
"""


def test_stream_quad_tables_cover_every_read(tmp_path):
    """The float4 stencil's quad-table reads (five float4 rows and two single
    values per quad in the lookup region) stay inside the per-slot quad
    tables, in the quad's own row, at the same table positions as the scalar
    stencil; and the coarse levels put in LDS fit the LDS budget."""
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "quad.cpp"
    src.write_text(QUAD)
    exe = tmp_path / "quad"
    inc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")
    cmd = [hipcc, "-x", "c++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", f"-I{inc}", f"-I{CSRC}",
           str(src), os.path.join(CSRC, "setup.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-3000:]
    out = subprocess.run([str(exe)], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert out.returncode == 0, out.stdout[-3000:]
    assert " bad 0" in out.stdout
