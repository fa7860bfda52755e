// GD losses: the weight w of the residual r = w z that the adjoint maps to
// the gradient, and each measurement's term of the loss trace.
//   l2 intensity loss (section II-B.1, Eq. (2)): sum (|z|^2 - y)^2,
//     w = |z|^2 - y;
//   Poisson negative log-likelihood of the intensities (section II-B.1 leaves
//   the loss to the noise model): sum |z|^2 - y log(|z|^2 + eps), guard
//   eps > 0, w = 1 - y / (|z|^2 + eps).
#pragma once
#include <hip/hip_runtime.h>

namespace sr {

enum LossKind : int { LOSS_L2 = 0, LOSS_POISSON = 1 };  // values of the C ABI's SR_LOSS_*

__device__ __forceinline__ float poisson_weight(float z2, float y, float eps) { return 1.f - y / (z2 + eps); }
__device__ __forceinline__ float poisson_term(float z2, float y, float eps) { return z2 - y * logf(z2 + eps); }


}  // namespace sr
