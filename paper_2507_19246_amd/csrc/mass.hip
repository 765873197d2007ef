// Row-sum lumped mass matrix (test option, mq_problem_desc.mass = MQ_MASS_LUMPED).
//
// The consistent P1 mass matrix of Section II-A, Eq. (4), has, at every node,
// off-diagonal entries that sum to its diagonal: each of the six triangles
// around a node adds sigma |T| / 12 to the diagonal and sigma |T| / 24 to each
// of its two edges from that node.  The row sum, taken over all neighbours
// including the Dirichlet boundary nodes, is therefore exactly twice the
// consistent diagonal, sigma |T| / 3 summed over the triangles.  Lumping thus
// doubles the C plane and clears the E, N and NE planes of every table node.
#include <hip/hip_runtime.h>

#include "mq_internal.h"

namespace mq {

__global__ void k_lump_mass(int rhw, size_t stride, int n_samples, double* __restrict__ tables) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int smp = blockIdx.y;
  if (t >= rhw || smp >= n_samples) return;
  double* T = tables + (size_t)smp * stride;
  T[T_MC * rhw + t] *= 2.0;
  T[T_ME * rhw + t] = 0.0;
  T[T_MN * rhw + t] = 0.0;
  T[T_MNE * rhw + t] = 0.0;
}

hipError_t launch_lump_mass(const Geom& g, int n_samples, double* tables, hipStream_t st) {
  (void)hipGetLastError();  // clear errors of earlier calls: report this launch's only
  const int rhw = g.RW * g.RH;
  if (n_samples < 1 || rhw < 1) return hipSuccess;
  hipLaunchKernelGGL(k_lump_mass, dim3((rhw + 255) / 256, n_samples), dim3(256), 0, st, rhw,
                     tab_stride(g), n_samples, tables);
  return hipGetLastError();
}

}  // namespace mq
