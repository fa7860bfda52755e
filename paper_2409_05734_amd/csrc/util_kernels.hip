// Small deterministic reductions and scalings used by the solvers: sum(y),
// squared norms, reduction of per-workgroup partials, and the final scaling
// of the spectral estimate (section II-B.2, Eq. (4)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "fft_core.hpp"
#include "plan.hpp"

namespace sr {

namespace {

template <int NT>
__device__ double block_sum_d(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// out = sum of part[0..n) in index order (one thread: order is fixed);
// thread t does the t-th of `count` sets of n partials, into out[t * ostride]
// (used for loss traces: a non-finite loss raises the plan's flag nf)
__global__ void reduce_partials_kernel(const float* __restrict__ part, int n, float* out, int count, int ostride,
                                       unsigned* nf) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (t < count) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += (double)part[(long long)t * n + i];
    out[(long long)t * ostride] = (float)acc;
    bad = !(fabs(acc) <= 3.402823466e38);
  }
  flag_nonfinite(nf, bad);
}

// Two-stage deterministic reductions: stage 1 gives workgroup g the
// contiguous chunk [g*chunk, (g+1)*chunk) (fixed strided order + fixed tree),
// stage 2 sums the per-workgroup partials in index order.
constexpr int kRedGroups = 1024;
constexpr int kRedStage1 = 256;

// (blockIdx.y: one of several equal-length arrays laid end to end)
__global__ void __launch_bounds__(kRedStage1) sum_floats_stage1(const float* __restrict__ y, long long n,
                                                                long long chunk, double* part) {
  __shared__ double red[kRedStage1];
  y += blockIdx.y * n;
  part += blockIdx.y * gridDim.x;
  const long long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  double acc = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += kRedStage1) acc += (double)y[i];
  const double s = block_sum_d<kRedStage1>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kRedStage1) norm2_stage1(const float2* __restrict__ x, long long n, long long chunk,
                                                           double* part) {
  __shared__ double red[kRedStage1];
  x += blockIdx.y * n;
  part += blockIdx.y * gridDim.x;
  const long long lo = blockIdx.x * chunk, hi = min(n, lo + chunk);
  double acc = 0.0;
  for (long long i = lo + threadIdx.x; i < hi; i += kRedStage1) {
    const float2 v = x[i];
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  const double s = block_sum_d<kRedStage1>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// stage 2: out = sum of part[0..g) in index order; as double or as float
// (thread t: the t-th of `count` arrays, whose partials follow one another)
__global__ void reduce_stage2(const double* __restrict__ part, int g, double* out_d, float* out_f, int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) {
    double acc = 0.0;
    for (int i = 0; i < g; ++i) acc += part[(long long)t * g + i];
    if (out_d) out_d[t] = acc;
    if (out_f) out_f[t] = (float)acc;
  }
}

// x *= sqrt(sum(y) * inv_mc) / ||x||, ||x||^2 = sum of the partials
// (blockIdx.y: one of several problems, each with its x, partials and sum)
// (the spectral estimate's last step: a NaN or Inf in it raises the flag nf)
__global__ void final_scale_kernel(float2* x, long long n, const float* __restrict__ part, int npart,
                                   const double* __restrict__ ysum, float inv_mc, unsigned* nf) {
  x += blockIdx.y * n;
  part += blockIdx.y * npart;
  ysum += blockIdx.y;
  double acc = 0.0;
  for (int i = 0; i < npart; ++i) acc += (double)part[i];
  const float sc = (float)(sqrt(*ysum * (double)inv_mc) / sqrt(acc));
  bool bad = false;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float2 v = cscale(x[i], sc);
    x[i] = v;
    bad |= !finite2(v);
  }
  flag_nonfinite(nf, bad);
}

// out[i] = exp(i theta[i])
__global__ void phase_table_kernel(const float* __restrict__ th, long long n, float2* __restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[i] = phase<false>(th[i], 1.f);
}

// dst[i] = v.v[i] for i < count: host values that travel as kernel
// arguments (copied at launch), so the caller's array is free on return and
// nothing waits for the stream
constexpr int kArgFloats = 256;
struct ArgFloats {
  float v[kArgFloats];
};
__global__ void __launch_bounds__(kArgFloats) put_floats_kernel(float* dst, ArgFloats v, int count) {
  if ((int)threadIdx.x < count) dst[threadIdx.x] = v.v[threadIdx.x];
}

}  // namespace

void red_shape(long long n, int* groups, long long* chunk) {
  long long g = (n + 4095) / 4096;
  if (g > kRedGroups) g = kRedGroups;
  if (g < 1) g = 1;
  *groups = (int)g;
  *chunk = (n + g - 1) / g;
}

sr_status put_floats(sr_plan_s* p, float* dst, const float* host, int count) {
  for (int lo = 0; lo < count; lo += kArgFloats) {
    ArgFloats v;
    const int c = std::min(kArgFloats, count - lo);
    std::memcpy(v.v, host + lo, sizeof(float) * c);
    hipLaunchKernelGGL(put_floats_kernel, dim3(1), dim3(kArgFloats), 0, p->stream, dst + lo, v, c);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SR_OK : hip_fail(e, "put_floats");
}

sr_status fill_phase_table(sr_plan_s* p) {
  if (p->eph == nullptr || p->theta_len <= 0) return SR_OK;
  const long long n = p->theta_len;
  const int groups = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(phase_table_kernel, dim3(groups), dim3(256), 0, p->stream, p->theta, n, p->eph);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SR_OK : hip_fail(e, "phase table");
}

sr_status reduce_partials(sr_plan_s* p, const float* part, int n, float* out, int count, int ostride) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((count + 63) / 64), dim3(64), 0, p->stream, part, n, out, count,
                     ostride, p->sync + 2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SR_OK : hip_fail(e, "reduce_partials");
}

// `count` arrays of n elements laid end to end, each reduced on its own (the
// same chunks and order as alone), as many per launch as the kRedGroups
// stage-1 partials hold.
sr_status sum_floats(sr_plan_s* p, const float* y, int64_t n, double* out, int count) {
  int g;
  long long chunk;
  red_shape(n, &g, &chunk);
  const int per = std::max(1, kRedGroups / g);
  for (int c0 = 0; c0 < count; c0 += per) {
    const int c = std::min(per, count - c0);
    hipLaunchKernelGGL(sum_floats_stage1, dim3(g, c), dim3(kRedStage1), 0, p->stream, y + (int64_t)c0 * n,
                       (long long)n, chunk, p->red_ws);
    hipLaunchKernelGGL(reduce_stage2, dim3((c + 63) / 64), dim3(64), 0, p->stream, p->red_ws, g, out + c0,
                       (float*)nullptr, c);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SR_OK : hip_fail(e, "sum_floats");
}

sr_status norm2_partial(sr_plan_s* p, const float2* x, int64_t n, float* out, int count) {
  int g;
  long long chunk;
  red_shape(n, &g, &chunk);
  const int per = std::max(1, kRedGroups / g);
  for (int c0 = 0; c0 < count; c0 += per) {
    const int c = std::min(per, count - c0);
    hipLaunchKernelGGL(norm2_stage1, dim3(g, c), dim3(kRedStage1), 0, p->stream, x + (int64_t)c0 * n, (long long)n,
                       chunk, p->red_ws);
    hipLaunchKernelGGL(reduce_stage2, dim3((c + 63) / 64), dim3(64), 0, p->stream, p->red_ws, g, (double*)nullptr,
                       out + c0, c);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SR_OK : hip_fail(e, "norm2");
}

sr_status final_scale(sr_plan_s* p, float2* x, int64_t n, const float* part, int npart, const double* ysum,
                      float inv_mc, int count) {
  int groups = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(final_scale_kernel, dim3(groups, count), dim3(256), 0, p->stream, x, (long long)n, part, npart,
                     ysum, inv_mc, p->sync + 2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SR_OK : hip_fail(e, "final_scale");
}

}  // namespace sr
