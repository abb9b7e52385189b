// Host-only parts of the plan interface: argument checks and the device
// footprint of a plan (no HIP calls; also used by the request server).
#include <cmath>

#include "bc.hpp"
#include "limits.hpp"
#include "vofpoisson.h"

static_assert(vp::kMaxBatch == VP_MAX_BATCH, "batch limit of the kernels and the C interface");

namespace {
bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }
}  // namespace

namespace vp {

bool fft_length(int n) {
  return pow2_in(n, 8, 1024) || (n % 5 == 0 && pow2_in(n / 5, 8, 128)) ||
         (n % 3 == 0 && pow2_in(n / 3, 8, 256));
}

int parse_ends(const char* bc, char e[6]) {
  if (!bc) return VP_EINVAL;
  int n = 0;
  while (n < 7 && bc[n]) ++n;
  if (n != 3 && n != 6) return VP_EINVAL;
  for (int i = 0; i < 6; ++i) {
    char c = n == 3 ? bc[i / 2] : bc[i];
    if (c >= 'a' && c <= 'z') c = (char)(c - 'a' + 'A');
    if (c != 'P' && c != 'N' && c != 'D') return VP_EINVAL;
    e[i] = c;
  }
  for (int d = 0; d < 3; ++d)
    if ((e[2 * d] == 'P') != (e[2 * d + 1] == 'P')) return VP_EINVAL;
  return VP_OK;
}

int direction_code(char lo, char hi) {
  if (lo == 'P') return BC_P;
  if (lo == hi) return lo == 'N' ? BC_N : BC_D;
  return lo == 'N' ? BC_ND : BC_DN;
}

}  // namespace vp

extern "C" {

int poisson_plan_check(int nx, int ny, int nz, double dx, double dy, const double* dz,
                       const char* bc, int precision, int max_batch) {
  if (!dz || !bc || nx <= 0 || ny <= 0 || nz <= 0 || !(dx > 0) || !(dy > 0) || max_batch < 1 ||
      max_batch > VP_MAX_BATCH || !std::isfinite(dx) || !std::isfinite(dy))
    return VP_EINVAL;
  char e[6];
  if (vp::parse_ends(bc, e) != VP_OK) return VP_EINVAL;
  for (int k = 0; k < nz; ++k)
    if (!(dz[k] > 0) || !std::isfinite(dz[k])) return VP_EINVAL;
  if (e[4] == 'P' && nz < 3) return VP_EINVAL;
  if (precision != VP_PRECISION_FP64 && precision != VP_PRECISION_MIXED) return VP_EINVAL;
  if (!vp::fft_length(nx) || !vp::fft_length(ny) || nz > 1024) return VP_EUNSUPPORTED;
  return VP_OK;
}

long long poisson_plan_footprint(int nx, int ny, int nz, int precision, int max_batch) {
  if (nx <= 0 || ny <= 0 || nz <= 0 || max_batch < 1 || max_batch > VP_MAX_BATCH) return -1;
  const long long n = (long long)nx * ny * nz * max_batch;
  const long long tables = 2LL * nx + 2 * (nx / 2 + 1) + 2LL * ny + 2 * (ny / 2 + 1);
  long long b = 8 * (tables + nx + ny + 4LL * nz + 3 * vp::kMaxBatch) + 8 * n;
  if (precision == VP_PRECISION_MIXED)
    b += 4 * n + 8LL * 4 * vp::kMaxBatch + 4LL * vp::kMaxBatch + 8LL * ny * nz * max_batch;
  return b;
}

}  // extern "C"
