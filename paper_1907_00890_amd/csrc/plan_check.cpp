// Host-only parts of the plan interface: argument checks and the device
// footprint of a plan (no HIP calls; also used by the request server).
#include <cmath>

#include "limits.hpp"
#include "vofpoisson.h"

static_assert(vp::kMaxBatch == VP_MAX_BATCH, "batch limit of the kernels and the C interface");

namespace {
bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }
}  // namespace

extern "C" {

int poisson_plan_check(int nx, int ny, int nz, double dx, double dy, const double* dz,
                       const char* bc, int precision, int max_batch) {
  if (!dz || !bc || nx <= 0 || ny <= 0 || nz <= 0 || !(dx > 0) || !(dy > 0) || max_batch < 1 ||
      max_batch > VP_MAX_BATCH || !std::isfinite(dx) || !std::isfinite(dy))
    return VP_EINVAL;
  bool dirichlet = false;
  for (int d = 0; d < 3; ++d) {
    const char ch = bc[d];
    if (ch == 'D' || ch == 'd') dirichlet = true;
    else if (ch != 'P' && ch != 'p' && ch != 'N' && ch != 'n') return VP_EINVAL;
  }
  if (bc[3] != '\0') return VP_EINVAL;
  for (int k = 0; k < nz; ++k)
    if (!(dz[k] > 0) || !std::isfinite(dz[k])) return VP_EINVAL;
  if ((bc[2] == 'P' || bc[2] == 'p') && nz < 3) return VP_EINVAL;
  if (precision != VP_PRECISION_FP64 && precision != VP_PRECISION_MIXED) return VP_EINVAL;
  if (dirichlet) return VP_EUNSUPPORTED;
  if (!pow2_in(nx, 8, 1024) || !pow2_in(ny, 8, 1024) || nz > 1024) return VP_EUNSUPPORTED;
  return VP_OK;
}

long long poisson_plan_footprint(int nx, int ny, int nz, int precision, int max_batch) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || max_batch < 1 || max_batch > VP_MAX_BATCH) return -1;
  const long long n = (long long)nx * ny * nz * max_batch;
  const long long tables = 2LL * nx + 2 * (nx / 2 + 1) + 2LL * ny + 2 * (ny / 2 + 1);
  long long b = 8 * (tables + nx + ny + 4LL * nz + 3 * vp::kMaxBatch) + 8 * n;
  if (precision == VP_PRECISION_MIXED)
    b += 4 * tables + 4 * n + 8 * n + 16LL * vp::kResidualMaxBlocks * max_batch +
         8LL * 4 * vp::kMaxBatch + 4LL * vp::kMaxBatch + 8LL * ny * nz * max_batch;
  return b;
}

}  // extern "C"
