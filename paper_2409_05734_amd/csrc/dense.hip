// Dense i.i.d. complex Gaussian sensing model (section II-A) on FP32 MFMA:
// the baseline the structured operator is compared against.
//
// A complex m x n matrix stored row-major as interleaved (re, im) floats is,
// read as floats, a real m x 2n matrix At.  For a batch of nb signals the
// complex products become single real GEMMs with FP32 matrix cores
// (v_mfma_f32_16x16x4f32), with no copy or conversion of A:
//
//   Z = A X   :  C (m x 2nb)  = At (m x 2n) . Bx (2n x 2nb),
//                Bx[2k][2p] = Re x_pk, Bx[2k+1][2p] = -Im x_pk,
//                Bx[2k][2p+1] = Im x_pk, Bx[2k+1][2p+1] = Re x_pk,
//                z_pi = C[i][2p] + i C[i][2p+1];
//   G = A^H R :  P (2n x 2nb) = At^T (2n x m) . Br (m x 2nb),
//                Br[i][2p] = Re r_pi, Br[i][2p+1] = Im r_pi,
//                g_pk = (P[2k][2p] + P[2k+1][2p+1]) + i (P[2k][2p+1] - P[2k+1][2p]).
//
// The epilogues fuse the solver arithmetic: |z|^2, the GD residual
// (|z|^2 - y) z with loss partials, the spectral weight T(y) z, and the GD or
// spectral update of the iterate with norm partials.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "fft_core.hpp"
#include "plan.hpp"

namespace sr {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64;   // output rows per workgroup
constexpr int BN = 64;   // output columns per workgroup (32 signals, re/im)
constexpr int BK = 64;   // reduction chunk
constexpr int PADK = BK + 4;
constexpr int NT = 256;  // 4 waves, 2 x 2 wave tiles of 32 x 32

enum AMode : int { A_ROWS = 0, A_TRANS = 1 };
enum Epi : int {
  E1_STORE = 0,  // GEMM 1: z and/or |z|^2
  E1_GD = 1,     // GEMM 1: r = (|z|^2 - y) z, loss partials
  E1_SPEC = 2,   // GEMM 1: r = T(y/mean(y)) z
  E2_STORE = 3,  // GEMM 2: x_out = A^H r * scale
  E2_GD = 4,     // GEMM 2: x <- x - step * A^H r
  E2_SPEC = 5    // GEMM 2: u <- step * A^H r - 2 lambda u / ||u||, norm partials
};

struct DenseArgs {
  const float* A;          // m x 2n floats
  int m, n, nb;
  const float2* src;       // GEMM 1: X (nb x n); GEMM 2: R (nb x m)
  const float* src_scale;  // per-signal scale of src (spectral 1/||u||), nullable
  float2* z_out;           // GEMM 1 store / residual out (nb x m)
  float* y_out;            // GEMM 1 store: |z|^2 (nb x m)
  const float* y;          // measurements (nb x m)
  const double* ysum;      // per-signal sum(y) (spectral)
  float lam;
  float2* x;               // GEMM 2: output / iterate (nb x n)
  float step;
  float* part;             // partial sums [signal][row tile]
  int part_ld;             // row tiles
  const float* prev_scale; // GEMM 2 spectral: 1/||u_p|| of the previous iterate
};

__device__ __forceinline__ f4 ld4(const float* p) { return *reinterpret_cast<const f4*>(p); }

template <int AM, int EPI>
__global__ void __launch_bounds__(NT) dense_gemm_kernel(const DenseArgs a) {
  constexpr bool G1 = (AM == A_ROWS);
  // GEMM 1: M = m, K = 2n; GEMM 2: M = 2n, K = m
  const int M = G1 ? a.m : 2 * a.n;
  const int K = G1 ? 2 * a.n : a.m;
  const int lda = 2 * a.n;
  const int i0 = blockIdx.x * BM;
  const int p0 = blockIdx.y * (BN / 2);  // first signal of this column tile

  __shared__ __attribute__((aligned(16))) float As[BM][PADK];
  __shared__ __attribute__((aligned(16))) float Bs[BN][PADK];
  __shared__ float Cs[BM][BN + 1];
  __shared__ float red[NT];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int g = lane >> 4;      // k group of this lane in the MFMA
  const int l16 = lane & 15;

  f4 acc[2][2];
#pragma unroll
  for (int a0 = 0; a0 < 2; ++a0)
#pragma unroll
    for (int b0 = 0; b0 < 2; ++b0) acc[a0][b0] = f4{0.f, 0.f, 0.f, 0.f};

  // Per-thread staging of one chunk (register prefetch of the next chunk
  // overlaps its global loads with the MFMAs of the current one).
  f4 ar[4];   // A: 16 floats
  f4 br[4];   // B: 16 floats (two rows of the tile)
  const int pl = tid >> 3;  // signal within the column tile (0..31)
  const int p_ld = p0 + pl;
  const float sc = (a.src_scale != nullptr && p_ld < a.nb) ? a.src_scale[p_ld] : 1.f;

  auto load_chunk = [&](int k0) {
    if constexpr (AM == A_ROWS) {
      // row tid/4, k' = k0 + 16*(tid&3) .. +16
      const int gi = i0 + (tid >> 2);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int gk = k0 + (tid & 3) * 16 + 4 * h;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (gi < M) {
          if (gk + 3 < K) {
            v = ld4(a.A + (long long)gi * lda + gk);
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (gk + q < K) v[q] = a.A[(long long)gi * lda + gk + q];
          }
        }
        ar[h] = v;
      }
    } else {
      // k = k0 + tid/4 (an A row), i = i0 + 16*(tid&3) .. +16
      const int gk = k0 + (tid >> 2);
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int gi = i0 + (tid & 3) * 16 + 4 * h;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (gk < K) {
          if (gi + 3 < M) {
            v = ld4(a.A + (long long)gk * lda + gi);
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (gi + q < M) v[q] = a.A[(long long)gk * lda + gi + q];
          }
        }
        ar[h] = v;
      }
    }
    if constexpr (G1) {
      // 4 complex entries of x_p: k' = k0 + 8*(tid&7) .. +8
      const int kc = (k0 + (tid & 7) * 8) / 2;
      float2 xv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        xv[q] = make_float2(0.f, 0.f);
        if (p_ld < a.nb && kc + q < a.n) xv[q] = cscale(a.src[(long long)p_ld * a.n + kc + q], sc);
      }
      br[0] = f4{xv[0].x, -xv[0].y, xv[1].x, -xv[1].y};
      br[1] = f4{xv[2].x, -xv[2].y, xv[3].x, -xv[3].y};
      br[2] = f4{xv[0].y, xv[0].x, xv[1].y, xv[1].x};
      br[3] = f4{xv[2].y, xv[2].x, xv[3].y, xv[3].x};
    } else {
      // 8 complex entries of r_p: i = k0 + 8*(tid&7) .. +8
      const int ib = k0 + (tid & 7) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float2 r = make_float2(0.f, 0.f);
        if (p_ld < a.nb && ib + q < a.m) r = cscale(a.src[(long long)p_ld * a.m + ib + q], sc);
        br[q >> 2][q & 3] = r.x;
        br[2 + (q >> 2)][q & 3] = r.y;
      }
    }
  };

  auto store_chunk = [&]() {
    if constexpr (AM == A_ROWS) {
#pragma unroll
      for (int h = 0; h < 4; ++h) *reinterpret_cast<f4*>(&As[tid >> 2][(tid & 3) * 16 + 4 * h]) = ar[h];
    } else {
#pragma unroll
      for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q) As[(tid & 3) * 16 + 4 * h + q][tid >> 2] = ar[h][q];
    }
    const int kq = (tid & 7) * 8;
    *reinterpret_cast<f4*>(&Bs[2 * pl][kq]) = br[0];
    *reinterpret_cast<f4*>(&Bs[2 * pl][kq + 4]) = br[1];
    *reinterpret_cast<f4*>(&Bs[2 * pl + 1][kq]) = br[2];
    *reinterpret_cast<f4*>(&Bs[2 * pl + 1][kq + 4]) = br[3];
  };

  load_chunk(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    store_chunk();
    __syncthreads();
    if (k0 + BK < K) load_chunk(k0 + BK);
    // MFMA over the chunk: blocks of 16 k; lane group g owns k = 16 kb + 4 g + kk
#pragma unroll
    for (int kb = 0; kb < BK / 16; ++kb) {
      f4 av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        av[t] = *reinterpret_cast<const f4*>(&As[32 * wr + 16 * t + l16][16 * kb + 4 * g]);
        bv[t] = *reinterpret_cast<const f4*>(&Bs[32 * wc + 16 * t + l16][16 * kb + 4 * g]);
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
          for (int tj = 0; tj < 2; ++tj)
            acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ti][kk], bv[tj][kk], acc[ti][tj], 0, 0, 0);
    }
    __syncthreads();
  }

  // ---- accumulators -> Cs (D[4*(lane/16)+r][lane%16] per 16x16 tile)
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) Cs[32 * wr + 16 * ti + 4 * g + r][32 * wc + 16 * tj + l16] = acc[ti][tj][r];
  __syncthreads();

  float part = 0.f;
  const int p = p_ld;
  if constexpr (G1) {
    // rows i0 + 8*(tid&7) .. +8 of signal p
    const int ib = (tid & 7) * 8;
    float ybar = 0.f;
    if constexpr (EPI == E1_SPEC) ybar = p < a.nb ? (float)(a.ysum[p] / (double)a.m) : 0.f;
    if (p < a.nb) {
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int il = ib + q;
        const int gi = i0 + il;
        if (gi >= a.m) break;
        const float2 z = make_float2(Cs[il][2 * pl], Cs[il][2 * pl + 1]);
        const long long o = (long long)p * a.m + gi;
        if constexpr (EPI == E1_STORE) {
          if (a.z_out) a.z_out[o] = z;
          if (a.y_out) a.y_out[o] = cabs2(z);
        } else if constexpr (EPI == E1_GD) {
          const float d = cabs2(z) - a.y[o];
          part += d * d;
          a.z_out[o] = cscale(z, d);
        } else {
          const float yy = a.y[o];
          float w = a.lam;
          if (yy > 0.f) w = fmaxf(1.f - ybar / yy, a.lam);
          a.z_out[o] = cscale(z, w);
        }
      }
    }
  } else {
    // entries k0 + 4*(tid&7) .. +4 of signal p (rows 2k, 2k+1 of the tile)
    const int kb = (tid & 7) * 4;
    if (p < a.nb) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kl = kb + q;
        const int gk = i0 / 2 + kl;
        if (gk >= a.n) break;
        const float2 gv = make_float2(Cs[2 * kl][2 * pl] + Cs[2 * kl + 1][2 * pl + 1],
                                      Cs[2 * kl][2 * pl + 1] - Cs[2 * kl + 1][2 * pl]);
        const long long o = (long long)p * a.n + gk;
        if constexpr (EPI == E2_STORE) {
          a.x[o] = cscale(gv, a.step);
        } else if constexpr (EPI == E2_GD) {
          const float2 xo = a.x[o];
          a.x[o] = make_float2(xo.x - a.step * gv.x, xo.y - a.step * gv.y);
        } else {
          // u_new = step * M v - 2 lambda v, v = u / ||u|| (the 1/||u|| was applied to R's source in GEMM 1)
          const float2 uo = a.x[o];
          const float c = 2.f * a.lam * a.prev_scale[p];
          const float2 nu = make_float2(a.step * gv.x - c * uo.x, a.step * gv.y - c * uo.y);
          a.x[o] = nu;
          part += cabs2(nu);
        }
      }
    }
  }
  if constexpr (EPI == E1_GD || EPI == E2_SPEC) {
    // per-signal partials: the 8 threads of signal pl are consecutive
    red[tid] = part;
    __syncthreads();
    if ((tid & 7) == 0 && p < a.nb) {
      float s = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) s += red[tid + q];
      a.part[(long long)p * a.part_ld + blockIdx.x] = s;
    }
  }
}

// inv[p] = 1/sqrt(sum_t part[p][t])  (fixed order)
__global__ void inv_norms_kernel(const float* __restrict__ part, int ld, int cnt, int nb, float* inv) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nb) return;
  double acc = 0.0;
  for (int t = 0; t < cnt; ++t) acc += (double)part[(long long)p * ld + t];
  inv[p] = (float)(1.0 / sqrt(acc));
}

// out[p * stride] = sum_t part[p][t]  (fixed order)
__global__ void sum_rows_kernel(const float* __restrict__ part, int ld, int cnt, int nb, float* out, int stride) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nb) return;
  double acc = 0.0;
  for (int t = 0; t < cnt; ++t) acc += (double)part[(long long)p * ld + t];
  out[(long long)p * stride] = (float)acc;
}

// per-signal sum of y (one workgroup per signal, fixed order)
__global__ void __launch_bounds__(256) row_sums_kernel(const float* __restrict__ y, int m, double* out) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += 256) acc += (double)y[(long long)p * m + i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[p] = red[0];
}

// per-signal squared norms (one workgroup per signal)
__global__ void __launch_bounds__(256) row_norm2_kernel(const float2* __restrict__ x, int n, float* part, int ld) {
  __shared__ double red[256];
  const int p = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float2 v = x[(long long)p * n + i];
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)p * ld] = (float)red[0];
}

// x_p *= sqrt(sum(y_p) * inv_mc) * inv[p]
__global__ void dense_final_scale_kernel(float2* x, int n, int nb, const double* ysum, const float* inv,
                                         float inv_mc) {
  const long long tot = (long long)n * nb;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(e / n);
    x[e] = cscale(x[e], (float)sqrt(ysum[p] * (double)inv_mc) * inv[p]);
  }
}

template <int AM, int EPI>
hipError_t gemm(const DenseArgs& a, hipStream_t s) {
  const int M = AM == A_ROWS ? a.m : 2 * a.n;
  dim3 grid((M + BM - 1) / BM, (a.nb + BN / 2 - 1) / (BN / 2));
  hipLaunchKernelGGL((dense_gemm_kernel<AM, EPI>), grid, dim3(NT), 0, s, a);
  return hipGetLastError();
}

DenseArgs base(const sr_plan_s* p) {
  DenseArgs a{};
  a.A = (const float*)p->dense_A;
  a.m = (int)p->geo[0].m;
  a.n = (int)p->geo[0].n;
  a.nb = (int)p->geo.size();
  return a;
}

int row_tiles_g1(const DenseArgs& a) { return (a.m + BM - 1) / BM; }
int row_tiles_g2(const DenseArgs& a) { return (2 * a.n + BM - 1) / BM; }

#define DN_HIP(x)                                     \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #x);    \
  } while (0)

}  // namespace

// Scratch layout for dense plans: bufA holds R (nb x m complex); fscratch
// holds per-signal scalars; part holds per-signal partials.
sr_status dense_forward(sr_plan_s* p, const float2* x, float2* z, float* y) {
  DenseArgs a = base(p);
  a.src = x;
  a.z_out = z;
  a.y_out = y;
  DN_HIP((gemm<A_ROWS, E1_STORE>(a, p->stream)));
  return SR_OK;
}

sr_status dense_adjoint(sr_plan_s* p, const float2* r, float2* x) {
  DenseArgs a = base(p);
  a.src = r;
  a.x = x;
  a.step = 1.f;
  DN_HIP((gemm<A_TRANS, E2_STORE>(a, p->stream)));
  return SR_OK;
}

sr_status dense_gd(sr_plan_s* p, const float* y, float2* x, int iters, const float* eta, float* loss_trace) {
  DenseArgs a = base(p);
  for (int i = 1; i < a.nb; ++i)
    if (eta[i] != eta[0]) return fail(SR_E_UNSUPPORTED, "dense plans take one step size for all signals");
  const int t1 = row_tiles_g1(a);
  if ((long long)a.nb * t1 > 2LL * p->part_cap) return fail(SR_E_NOMEM, "partial buffer too small");
  for (int it = 0; it < iters; ++it) {
    DenseArgs g1 = a;
    g1.src = x;
    g1.y = y;
    g1.z_out = p->bufA;
    g1.part = p->part;
    g1.part_ld = t1;
    DN_HIP((gemm<A_ROWS, E1_GD>(g1, p->stream)));
    if (loss_trace) {
      hipLaunchKernelGGL(sum_rows_kernel, dim3((a.nb + 63) / 64), dim3(64), 0, p->stream, p->part, t1, t1, a.nb,
                         loss_trace + it, iters);
      DN_HIP(hipGetLastError());
    }
    DenseArgs g2 = a;
    g2.src = p->bufA;
    g2.x = x;
    g2.step = eta[0] / (float)a.m;
    DN_HIP((gemm<A_TRANS, E2_GD>(g2, p->stream)));
  }
  return SR_OK;
}

sr_status dense_spectral(sr_plan_s* p, const float* y, const float2* v0, int iters, float lam, float2* x0) {
  DenseArgs a = base(p);
  const int t2 = row_tiles_g2(a);
  if ((long long)a.nb * t2 > 2LL * p->part_cap) return fail(SR_E_NOMEM, "partial buffer too small");
  float* inv = p->fscratch;  // nb floats: 1/||u_p||
  double* ysum = p->ysum;
  hipLaunchKernelGGL(row_sums_kernel, dim3(a.nb), dim3(256), 0, p->stream, y, a.m, ysum);
  DN_HIP(hipGetLastError());
  DN_HIP(hipMemcpyAsync(x0, v0, sizeof(float2) * (size_t)a.n * a.nb, hipMemcpyDeviceToDevice, p->stream));
  hipLaunchKernelGGL(row_norm2_kernel, dim3(a.nb), dim3(256), 0, p->stream, x0, a.n, p->part, t2);
  DN_HIP(hipGetLastError());
  int cnt = 1;
  const float inv_mc = 1.f / (float)a.m;  // dense CN(0,1): c = 1
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(inv_norms_kernel, dim3((a.nb + 63) / 64), dim3(64), 0, p->stream, p->part, t2, cnt, a.nb, inv);
    DN_HIP(hipGetLastError());
    DenseArgs g1 = a;  // r = T(y) . A (u / ||u||)
    g1.src = x0;
    g1.src_scale = inv;
    g1.y = y;
    g1.ysum = ysum;
    g1.lam = lam;
    g1.z_out = p->bufA;
    DN_HIP((gemm<A_ROWS, E1_SPEC>(g1, p->stream)));
    DenseArgs g2 = a;  // u <- A^H r / (m c) - 2 lambda u / ||u||
    g2.src = p->bufA;
    g2.x = x0;
    g2.step = inv_mc;
    g2.lam = lam;
    g2.prev_scale = inv;
    g2.part = p->part;
    g2.part_ld = t2;
    DN_HIP((gemm<A_TRANS, E2_SPEC>(g2, p->stream)));
    cnt = t2;
  }
  hipLaunchKernelGGL(inv_norms_kernel, dim3((a.nb + 63) / 64), dim3(64), 0, p->stream, p->part, t2, cnt, a.nb, inv);
  DN_HIP(hipGetLastError());
  const long long tot = (long long)a.n * a.nb;
  const int groups = (int)std::min<long long>((tot + 255) / 256, 2048);
  hipLaunchKernelGGL(dense_final_scale_kernel, dim3(groups), dim3(256), 0, p->stream, x0, a.n, a.nb, ysum, inv, inv_mc);
  DN_HIP(hipGetLastError());
  return SR_OK;
}

}  // namespace sr
