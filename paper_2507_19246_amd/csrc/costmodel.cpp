// Time-to-solution and effort model of MLMC with Parareal on the finest level
// (Section II-C, Eqs. (13)-(16); Section II-D, Eqs. (17)-(25) and the
// finite-core speedup that follows Eq. (25)).  Host arithmetic only.
#include <cmath>
#include <cstring>

#include "problem.h"

extern "C" int mq_cost_model(const mq_cost_in* in, mq_cost_out* out) {
  using mq::fail;
  if (!in || !out) return fail(MQ_ERR_INVALID_ARG, "null argument");
  const int nl = in->n_levels, L = nl - 1, K = in->K, M = in->M;
  if (nl < 3 || nl > 16) return fail(MQ_ERR_INVALID_ARG, "n_levels must be in [3, 16] (the coarse propagator is level L-2)");
  if (M < 1 || K < 1 || K > M || in->n_cores < 1) return fail(MQ_ERR_INVALID_ARG, "need 1 <= K <= M and n_cores >= 1");
  for (int l = 0; l < nl; ++l)
    if (!(in->C[l] > 0) || !(in->N[l] >= 1)) return fail(MQ_ERR_INVALID_ARG, "C_l > 0 and N_l >= 1 required");
  std::memset(out, 0, sizeof(*out));
  const double* C = in->C;
  const double* N = in->N;
  // Parareal on level L: fine = level L, coarse = level L-2 (the design rule of Section II-D)
  const double tf = C[L], tc = C[L - 2], k = K, m = M;
  out->tau_para = k / m * (tf + (m - (k + 1) / 2) * tc);                       // Eq. (15)
  out->effort_para = k / m * (m - (k + 1) / 2) * (tf + tc) + k / m * tf;       // Eq. (16)
  double sum_c = 0, sum_c_low = 0, eff_ref = 0, eff_low = 0;
  for (int l = 0; l < nl; ++l) {
    sum_c += C[l];
    eff_ref += N[l] * C[l];
    if (l < L) {
      sum_c_low += C[l];
      eff_low += N[l] * C[l];
    }
  }
  out->tau_ref = sum_c;                                                        // Eq. (17)
  out->effort_ref = eff_ref;
  out->tau_comb = sum_c_low + out->tau_para;                                   // Eq. (18)
  out->effort_comb = eff_low + N[L] * out->effort_para;                        // Eq. (19)
  out->speedup = out->tau_ref / out->tau_comb;
  out->s_inf = sum_c / (sum_c_low + C[L - 1]);                                 // Eq. (21), tau_para -> C_{L-1}
  out->eps_inf = out->effort_comb / out->effort_ref;                           // Eq. (23)
  // Eq. (22): the largest K with tau_para <= C_{L-1}, r = C_L / C_{L-1}, n = M slices
  const double r = C[L] / C[L - 1];
  out->r = r;
  const double b = 2 * r * r + 2 * m - 1;
  out->kappa = (int32_t)std::floor((b - std::sqrt(b * b - 8 * m * r)) / 2);
  // Eq. (24): batches per level on n_c cores (a level's sample costs C_l + C_{l-1})
  const double nc = in->n_cores;
  for (int l = 0; l < nl; ++l) {
    const double ratio = l == 0 ? 0.0 : C[l - 1] / C[l];
    out->batches[l] = (int32_t)std::ceil(N[l] * (1 + ratio) / nc);
  }
  // Eq. (25): cores per Parareal sample
  const int np = (int)std::floor(nc / (N[L] * (1 + C[L - 1] / C[L])));
  out->n_c_para = np;
  // finite-core speedup; its bracket is read as tau_F + (n_p - (K+1)/2) tau_C with
  // tau_F = C_L, tau_C = C_{L-2} (equal to the printed r^L, r^{L-2} form when C_0 = 1)
  if (np >= 1) {
    double num = 0, den = 0;
    for (int l = 0; l < nl; ++l) {
      num += out->batches[l] * C[l];
      if (l < L) den += out->batches[l] * C[l];
    }
    den += k / np * (C[L] + (np - (k + 1) / 2) * C[L - 2]);
    out->s_nc = num / den;
  }
  return MQ_OK;
}
