// Host-side mesh set-up (see setup.cpp).
#pragma once

#include <vector>

#include "mq_internal.h"

namespace mq {

struct HostMesh {
  Geom g;
  CellRegion cr;
  std::vector<uint8_t> cond;     // conductor flag per cell-region element
  std::vector<double> cx, cy;    // centroids per cell-region element
  std::vector<double> S;         // load shape on the full grid (pitch P)
  int n_modes;
  std::vector<double> kl;        // [element][mode] sqrt(lam) phi at centroids
  std::vector<double> kl_lambda; // 2-D eigenvalues in use
};

HostMesh build_host_mesh(const mq_problem_desc& d);

}  // namespace mq
