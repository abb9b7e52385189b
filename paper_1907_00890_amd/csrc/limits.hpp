// Sizes shared by the kernels, the plan and the host-only checks.
#pragma once

namespace vp {
constexpr int kMaxBatch = 16;             // fields per batched launch
}  // namespace vp
