// Sizes shared by the kernels, the plan and the host-only checks.
#pragma once

namespace vp {
constexpr int kMaxBatch = 16;             // fields per batched launch
constexpr int kResidualMaxBlocks = 16384;  // partial sums of one residual launch
}  // namespace vp
