// BF16 matrix-core form of the per-species network (placeholder until the MFMA
// kernel lands: reports itself unavailable so that model creation rejects it).
#include "plan.h"

namespace qnep {

bool mlp_bf16_supported(int, int) { return false; }

hipError_t launch_mlp_bf16(const Plan &) { return hipErrorNotSupported; }

}  // namespace qnep
