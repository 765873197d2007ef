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
