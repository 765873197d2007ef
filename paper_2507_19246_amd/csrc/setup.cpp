// Host-side mesh set-up: region masks, the sample-dependent box, the load
// shape and the Karhunen-Loeve table (Section II-A, Eqs. (2)-(5); the KL
// field of the conductivity input).
#include "setup.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace mq {

namespace {

// Element centroid of triangle t of full-grid cell (ci, cj): t = 0 is
// {(I,J), (I+1,J), (I+1,J+1)}, t = 1 is {(I,J), (I+1,J+1), (I,J+1)}.
inline void centroid(int ci, int cj, int t, double h, double* x, double* y) {
  if (t == 0) {
    *x = (3.0 * ci + 2.0) * h / 3.0;
    *y = (3.0 * cj + 1.0) * h / 3.0;
  } else {
    *x = (3.0 * ci + 1.0) * h / 3.0;
    *y = (3.0 * cj + 2.0) * h / 3.0;
  }
}

inline bool in_rect(double x, double y, const double r[4]) {
  return x >= r[0] && x <= r[1] && y >= r[2] && y <= r[3];
}

// Root of f on [lo, hi] (sign change) by bisection to full double precision.
template <class F>
double bisect(F f, double lo, double hi) {
  double flo = f(lo);
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double fm = f(mid);
    if ((fm < 0) == (flo < 0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

struct Mode1D {
  double w;
  int odd;
};

// 1-D eigenpairs of exp(-c|s - t|) on [-a, a] in ascending w.  Each interval
// [k pi/a, (k pi + pi/2)/a] holds one root of c cos(wa) = w sin(wa) (cosine
// modes) and [(k pi + pi/2)/a, (k+1) pi/a] one of w cos(wa) = -c sin(wa)
// (sine modes); these smooth forms have no poles inside the intervals.
std::vector<Mode1D> modes_1d(double a, double c, int count) {
  std::vector<Mode1D> m;
  const double pi = M_PI;
  for (int k = 0; (int)m.size() < count; ++k) {
    auto fe = [&](double w) { return c * std::cos(w * a) - w * std::sin(w * a); };
    auto fo = [&](double w) { return w * std::cos(w * a) + c * std::sin(w * a); };
    m.push_back({bisect(fe, k * pi / a, (k * pi + 0.5 * pi) / a), 0});
    m.push_back({bisect(fo, (k * pi + 0.5 * pi) / a, (k + 1) * pi / a), 1});
  }
  std::sort(m.begin(), m.end(), [](const Mode1D& x, const Mode1D& y) { return x.w < y.w; });
  m.resize(count);
  return m;
}

double phi(double s, const Mode1D& md, double a) {
  const double w = md.w;
  if (!md.odd) return std::cos(w * s) / std::sqrt(a + std::sin(2 * w * a) / (2 * w));
  return std::sin(w * s) / std::sqrt(a - std::sin(2 * w * a) / (2 * w));
}

}  // namespace

HostMesh build_host_mesh(const mq_problem_desc& d) {
  HostMesh hm;
  Geom& g = hm.g;
  const int N = d.n_nodes;
  g.N = N;
  g.n = N - 2;
  g.P = (N + 3) & ~3;  // 32-byte aligned rows of doubles
  g.h = 1.0 / (N - 1);
  g.h2 = g.h * g.h;
  g.nu_air = d.nu_air;
  const int n = g.n;

  // Interior nodes touching a conductor element.
  int mx0 = n, mx1 = -1, my0 = n, my1 = -1;
  for (int cj = 0; cj < N - 1; ++cj)
    for (int ci = 0; ci < N - 1; ++ci)
      for (int t = 0; t < 2; ++t) {
        double x, y;
        centroid(ci, cj, t, g.h, &x, &y);
        if (!in_rect(x, y, d.conductor)) continue;
        // vertices in full-grid coords
        int vx[3] = {ci, ci + 1, t == 0 ? ci + 1 : ci};
        int vy[3] = {cj, t == 0 ? cj : cj + 1, cj + 1};
        for (int v = 0; v < 3; ++v) {
          int i = vx[v] - 1, j = vy[v] - 1;
          if (i < 0 || j < 0 || i >= n || j >= n) continue;
          mx0 = std::min(mx0, i);
          mx1 = std::max(mx1, i);
          my0 = std::min(my0, j);
          my1 = std::max(my1, j);
        }
      }
  if (mx1 < 0) {  // no conductor: an empty box
    g.bx0 = g.bx1 = g.by0 = g.by1 = 0;
  } else {
    g.bx0 = std::max(0, mx0 - 1);
    g.bx1 = std::min(n, mx1 + 2);
    g.by0 = std::max(0, my0 - 1);
    g.by1 = std::min(n, my1 + 2);
  }
  g.lx1 = std::min(n, g.bx1 + 1);
  g.ly1 = std::min(n, g.by1 + 1);
  if (g.bx1 == g.bx0) { g.lx1 = g.bx0; }
  if (g.by1 == g.by0) { g.ly1 = g.by0; }
  g.RW = (g.bx1 - g.bx0) + 2;
  g.RH = (g.by1 - g.by0) + 2;

  // Cells whose triangles touch box nodes: full-grid cells [bx0, bx1+1) x [by0, by1+1).
  CellRegion& cr = hm.cr;
  cr.cx0 = g.bx0;
  cr.cy0 = g.by0;
  cr.cw = (g.bx1 - g.bx0) + 1;
  cr.ch = (g.by1 - g.by0) + 1;
  const int ne = cr.cw * cr.ch * 2;
  hm.cond.assign(ne, 0);
  hm.cx.assign(ne, 0.0);
  hm.cy.assign(ne, 0.0);
  for (int r = 0; r < cr.ch; ++r)
    for (int c = 0; c < cr.cw; ++c)
      for (int t = 0; t < 2; ++t) {
        int e = (r * cr.cw + c) * 2 + t;
        double x, y;
        centroid(cr.cx0 + c, cr.cy0 + r, t, g.h, &x, &y);
        hm.cx[e] = x;
        hm.cy[e] = y;
        hm.cond[e] = in_rect(x, y, d.conductor) ? 1 : 0;
      }

  // Load shape S_i = sum over strip elements e containing node i of |T_e|/3.
  hm.S.assign((size_t)N * g.P, 0.0);
  const double third_area = 0.5 * g.h2 / 3.0;
  for (int cj = 0; cj < N - 1; ++cj)
    for (int ci = 0; ci < N - 1; ++ci)
      for (int t = 0; t < 2; ++t) {
        double x, y;
        centroid(ci, cj, t, g.h, &x, &y);
        if (!(x >= d.strip[0] && x <= d.strip[1])) continue;
        int vx[3] = {ci, ci + 1, t == 0 ? ci + 1 : ci};
        int vy[3] = {cj, t == 0 ? cj : cj + 1, cj + 1};
        for (int v = 0; v < 3; ++v) {
          if (vx[v] <= 0 || vy[v] <= 0 || vx[v] >= N - 1 || vy[v] >= N - 1) continue;
          hm.S[(size_t)vy[v] * g.P + vx[v]] += third_area;
        }
      }

  // KL table sqrt(lam_k) phi_k(c_e) for conductor elements of the cell region.
  hm.n_modes = 0;
  if (d.material == MQ_MAT_KL) {
    const int nm = d.n_modes;
    const double ax = 0.5 * (d.conductor[1] - d.conductor[0]);
    const double ay = 0.5 * (d.conductor[3] - d.conductor[2]);
    const double xc = 0.5 * (d.conductor[0] + d.conductor[1]);
    const double yc = 0.5 * (d.conductor[2] + d.conductor[3]);
    const double c = 1.0 / d.corr_len;
    const int n1 = std::max(12, nm + 4);
    std::vector<Mode1D> mx = modes_1d(ax, c, n1), my = modes_1d(ay, c, n1);
    struct Cand {
      double lam;
      int i, j;
    };
    std::vector<Cand> cand;
    for (int i = 0; i < n1; ++i)
      for (int j = 0; j < n1; ++j) {
        double li = 2 * c / (mx[i].w * mx[i].w + c * c);
        double lj = 2 * c / (my[j].w * my[j].w + c * c);
        cand.push_back({li * lj, i, j});
      }
    std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
      if (a.lam != b.lam) return a.lam > b.lam;
      return a.i < b.i;
    });
    hm.n_modes = nm;
    hm.kl_lambda.resize(nm);
    hm.kl.assign((size_t)ne * nm, 0.0);
    for (int k = 0; k < nm; ++k) {
      const Cand& cd = cand[k];
      hm.kl_lambda[k] = cd.lam;
      const double sl = std::sqrt(cd.lam);
      for (int e = 0; e < ne; ++e) {
        if (!hm.cond[e]) continue;
        hm.kl[(size_t)e * nm + k] = sl * phi(hm.cx[e] - xc, mx[cd.i], ax) * phi(hm.cy[e] - yc, my[cd.j], ay);
      }
    }
  }
  return hm;
}

bool build_mg(const Geom& g, int lp, MGGeom* mg) {
  mg->nlev = 0;
  mg->region_elems = 0;
  mg->ctab_elems = 0;
  const int n = g.n;
  if (n < 3 || ((n + 1) & n) != 0) return false;  // n = 2^k - 1
  MGLevel& f = mg->lv[0];
  f.n = n;
  f.bx0 = g.bx0;
  f.bx1 = g.bx1;
  f.by0 = g.by0;
  f.by1 = g.by1;
  f.lx1 = g.lx1;
  f.ly1 = g.ly1;
  f.RW = g.RW;
  f.RH = g.RH;
  f.tab_off = 0;
  f.vec_off = 0;
  int l = 0, vec = 0, tab = 0;
  while (mg->lv[l].n > 1) {
    if (l + 1 >= MG_MAX_LEVELS) return false;
    const MGLevel& F = mg->lv[l];
    const int nc = (F.n - 1) / 2;
    MGLevel c{};
    c.n = nc;
    // coarse node ic owns non-air entries iff the fine rows 2ic..2ic+2 meet
    // the fine lookup region [bx0, lx1)
    auto range = [&](int f0, int f1, int* c0, int* c1) {
      *c0 = nc;
      *c1 = 0;
      if (f1 <= f0) {
        *c0 = *c1 = 0;
        return;
      }
      for (int ic = 0; ic < nc; ++ic)
        if (2 * ic + 2 >= f0 && 2 * ic <= f1 - 1) {
          if (ic < *c0) *c0 = ic;
          *c1 = ic + 1;
        }
      if (*c1 <= *c0) *c0 = *c1 = 0;
    };
    range(F.bx0, F.lx1, &c.bx0, &c.bx1);
    range(F.by0, F.ly1, &c.by0, &c.by1);
    if (c.bx1 == c.bx0 || c.by1 == c.by0) c.bx0 = c.bx1 = c.by0 = c.by1 = 0;
    c.lx1 = c.bx1 > c.bx0 ? std::min(nc, c.bx1 + 1) : c.bx0;
    c.ly1 = c.by1 > c.by0 ? std::min(nc, c.by1 + 1) : c.by0;
    c.RW = (c.bx1 - c.bx0) + 2;
    c.RH = (c.by1 - c.by0) + 2;
    c.tab_off = tab;
    tab += 5 * c.RW * c.RH;
    c.vec_off = vec;
    vec += 3 * (nc + 2) * (nc + 2);
    mg->lv[++l] = c;
  }
  mg->nlev = l;
  mg->region_elems = std::max((n + 2) * lp, vec);
  mg->ctab_elems = tab;
  return true;
}

}  // namespace mq
