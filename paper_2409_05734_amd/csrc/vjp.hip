#include "plan.hpp"
namespace sr {
sr_status vjp_forward(sr_plan_s*, const float2*, const float2*, float2*, float*) { return fail(SR_E_UNSUPPORTED, "not built yet"); }
sr_status vjp_adjoint(sr_plan_s*, const float2*, const float2*, float2*, float*) { return fail(SR_E_UNSUPPORTED, "not built yet"); }
}
