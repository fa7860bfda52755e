#include "plan.hpp"
namespace sr {
sr_status dense_forward(sr_plan_s*, const float2*, float2*, float*) { return fail(SR_E_UNSUPPORTED, "dense path not built yet"); }
sr_status dense_adjoint(sr_plan_s*, const float2*, float2*) { return fail(SR_E_UNSUPPORTED, "dense path not built yet"); }
sr_status dense_gd(sr_plan_s*, const float*, float2*, int, const float*, float*) { return fail(SR_E_UNSUPPORTED, "dense path not built yet"); }
sr_status dense_spectral(sr_plan_s*, const float*, const float2*, int, float, float2*) { return fail(SR_E_UNSUPPORTED, "dense path not built yet"); }
}
