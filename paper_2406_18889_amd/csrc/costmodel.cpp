// Learned step-cost model used by the path search (placeholder until a
// model is loaded).
#include "plan.h"

namespace lf {
const CostFn* mlp_cost_fn() { return nullptr; }
}  // namespace lf
