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
#include <hipblaslt/hipblaslt.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "fft_core.hpp"
#include "loss.hpp"
#include "plan.hpp"

namespace sr {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

// Both products are skinny GEMMs (N = 2 nb <= 64 real columns per tile)
// whose reduction runs over the long dimension of A.  The reduction is split
// over S workgroups (S chosen so that a launch has about four workgroups per
// CU); each writes its 64 x 64 partial tile, and an epilogue kernel sums the S
// partials in a fixed order and applies the solver arithmetic.  A is read in
// its natural row-major layout in both products: in A X it is the MFMA's
// first operand (rows i, reduction along 2n), in A^H R the second one
// (reduction along m, columns 2n), computing P^T = Br^T At.
constexpr int BT = 64;    // tile rows and columns
constexpr int BK = 64;    // reduction chunk
constexpr int PADK = BK + 4;
constexpr int NT = 256;   // 4 waves, 2 x 2 wave tiles of 32 x 32
constexpr int kTargetGroups = 1024;
constexpr int kMaxSplit = 8;  // the epilogue sums at most this many partial tiles

enum Epi : int {
  E1_STORE = 0,  // after A X: z and/or |z|^2
  E1_GD = 1,     // after A X: r = (|z|^2 - y) z (or the Poisson residual), loss partials
  E1_SPEC = 2,   // after A X: r = T(y/mean(y)) z
  E2_STORE = 3,  // after A^H R: x_out = A^H r * scale
  E2_GD = 4,     // after A^H R: x <- x - step * A^H r
  E2_SPEC = 5    // after A^H R: u <- step * A^H r - 2 lambda u / ||u||, norm partials
};

struct DenseArgs {
  const float* A;          // m x 2n floats
  int m, n, nb;
  const float2* src;       // A X: X (nb x n); A^H R: R (nb x m)
  const float* src_scale;  // per-signal scale of src (spectral 1/||u||), nullable
  float2* z_out;           // A X store / residual out (nb x m)
  float* y_out;            // A X store: |z|^2 (nb x m)
  const float* y;          // measurements (nb x m)
  const double* ysum;      // per-signal sum(y) (spectral)
  float lam;
  float2* x;               // A^H R: output / iterate (nb x n)
  float step;
  float* part;             // partial sums [signal][row tile]
  int part_ld;             // row tiles
  const float* prev_scale; // A^H R spectral: 1/||u_p|| of the previous iterate
  // split reduction
  float* split;            // S partial products
  int S;                   // reduction splits
  int kchunk;              // reduction length per split (multiple of BK)
  int q_ld;                // 2 * (signals rounded up to 32): row length of the partials of A X
  int loss;                // E1_GD: LOSS_L2 or LOSS_POISSON
  float loss_eps;          // E1_GD: Poisson guard
  unsigned* nf;            // E2_GD / E2_SPEC: set to 1 when an updated entry is NaN or Inf
};

__device__ __forceinline__ f4 ld4(const float* p) { return *reinterpret_cast<const f4*>(p); }

// Split-reduction GEMM.  G = 1: C (m x 2nb) = At . Bx over k in [0, 2n);
// partial s stored at split[(s * m + i) * q_ld + q].  G = 2: C^T (2nb x 2n) =
// Br^T . At over i in [0, m); partial s stored at split[(s * q_ld + q) * 2n + j].
// grid.x = tiles * S (split index fastest), grid.y = signal tiles of 32.
template <int G>
__global__ void __launch_bounds__(NT) dense_mm_kernel(const DenseArgs a) {
  const int M = G == 1 ? a.m : 2 * a.n;   // the big matrix's output extent
  const int K = G == 1 ? 2 * a.n : a.m;
  const int lda = 2 * a.n;
  const int s = blockIdx.x % a.S;
  const int i0 = (blockIdx.x / a.S) * BT;       // first output row (G1) / column (G2) of A
  const int p0 = blockIdx.y * (BT / 2);         // first signal of this tile
  const int kbeg = s * a.kchunk;
  const int kend = min(K, kbeg + a.kchunk);

  // G1: As[i][k] (from A), Bs[q][k] (from X).  G2: As[q][k] (from R), Bs[k][j] (from A).
  __shared__ __attribute__((aligned(16))) float As[BT][PADK];
  __shared__ __attribute__((aligned(16))) float Bs[BT][PADK];

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
  f4 ar[4];   // 16 floats of A
  f4 br[4];   // 16 floats of the small operand (two rows of the tile)
  const int pl = tid >> 3;  // signal within the tile (0..31)
  const int p_ld = p0 + pl;
  const float sc = (a.src_scale != nullptr && p_ld < a.nb) ? a.src_scale[p_ld] : 1.f;

  auto load_chunk = [&](int k0) {
    if constexpr (G == 1) {
      // A rows i0 + tid/16 + 16h, k = k0 + 4*(tid&15) .. +4: sixteen lanes read
      // one row's 256 contiguous bytes
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int gi = i0 + (tid >> 4) + 16 * h;
        const int gk = k0 + (tid & 15) * 4;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (gi < M) {
          if (gk + 3 < kend) {
            v = ld4(a.A + (long long)gi * lda + gk);
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (gk + q < kend) v[q] = a.A[(long long)gi * lda + gk + q];
          }
        }
        ar[h] = v;
      }
      // 4 complex entries of x_p: k' = k0 + 8*(tid&7) .. +8
      const int kc = (k0 + (tid & 7) * 8) / 2;
      float2 xv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        xv[q] = make_float2(0.f, 0.f);
        if (p_ld < a.nb && 2 * (kc + q) < kend) xv[q] = cscale(a.src[(long long)p_ld * a.n + kc + q], sc);
      }
      br[0] = f4{xv[0].x, -xv[0].y, xv[1].x, -xv[1].y};
      br[1] = f4{xv[2].x, -xv[2].y, xv[3].x, -xv[3].y};
      br[2] = f4{xv[0].y, xv[0].x, xv[1].y, xv[1].x};
      br[3] = f4{xv[2].y, xv[2].x, xv[3].y, xv[3].x};
    } else {
      // A rows k = k0 + tid/16 + 16h (m indices), columns j = i0 + 4*(tid&15) .. +4
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int gk = k0 + (tid >> 4) + 16 * h;
        const int gj = i0 + (tid & 15) * 4;
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (gk < kend) {
          if (gj + 3 < M) {
            v = ld4(a.A + (long long)gk * lda + gj);
          } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (gj + q < M) v[q] = a.A[(long long)gk * lda + gj + q];
          }
        }
        ar[h] = v;
      }
      // 8 complex entries of r_p: i = k0 + 8*(tid&7) .. +8
      const int ib = k0 + (tid & 7) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        float2 r = make_float2(0.f, 0.f);
        if (p_ld < a.nb && ib + q < kend) r = cscale(a.src[(long long)p_ld * a.m + ib + q], sc);
        br[q >> 2][q & 3] = r.x;
        br[2 + (q >> 2)][q & 3] = r.y;
      }
    }
  };

  auto store_chunk = [&]() {
    // A: natural layout in both products (row tid/16 + 16h, 4 consecutive floats)
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      float* dst = G == 1 ? &As[(tid >> 4) + 16 * h][(tid & 15) * 4] : &Bs[(tid >> 4) + 16 * h][(tid & 15) * 4];
      *reinterpret_cast<f4*>(dst) = ar[h];
    }
    float(*S2)[PADK] = G == 1 ? Bs : As;
    const int kq = (tid & 7) * 8;
    *reinterpret_cast<f4*>(&S2[2 * pl][kq]) = br[0];
    *reinterpret_cast<f4*>(&S2[2 * pl][kq + 4]) = br[1];
    *reinterpret_cast<f4*>(&S2[2 * pl + 1][kq]) = br[2];
    *reinterpret_cast<f4*>(&S2[2 * pl + 1][kq + 4]) = br[3];
  };

  if (kbeg < kend) {
    load_chunk(kbeg);
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      store_chunk();
      __syncthreads();
      if (k0 + BK < kend) load_chunk(k0 + BK);
      // blocks of 16 k; lane group g owns k = 16 kb + 4 g + kk
#pragma unroll
      for (int kb = 0; kb < BK / 16; ++kb) {
        f4 av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          av[t] = *reinterpret_cast<const f4*>(&As[32 * wr + 16 * t + l16][16 * kb + 4 * g]);
          if constexpr (G == 1) {
            bv[t] = *reinterpret_cast<const f4*>(&Bs[32 * wc + 16 * t + l16][16 * kb + 4 * g]);
          } else {
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) bv[t][kk] = Bs[16 * kb + 4 * g + kk][32 * wc + 16 * t + l16];
          }
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
  }

  // ---- partial tile out: D[4*(lane/16)+r][lane%16] of each 16 x 16 block
  const int q0 = 2 * p0;
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 32 * wr + 16 * ti + 4 * g + r;
        const int col = 32 * wc + 16 * tj + l16;
        if constexpr (G == 1) {
          if (i0 + row < M) a.split[((long long)s * a.m + i0 + row) * a.q_ld + q0 + col] = acc[ti][tj][r];
        } else {
          if (i0 + col < M) a.split[((long long)s * a.q_ld + q0 + row) * M + i0 + col] = acc[ti][tj][r];
        }
      }
}

// Epilogue after A X: z_pi = sum_s C_s[i][2p] + i C_s[i][2p+1] for 64 rows and
// 32 signals, then the E1 arithmetic.  grid (row tiles, signal tiles).
template <int EPI>
__global__ void __launch_bounds__(NT) dense_epi1_kernel(const DenseArgs a) {
  __shared__ float2 zs[BT][33];
  __shared__ float red[NT];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * BT;
  const int p0 = blockIdx.y * 32;
  {
    // gather: thread (row il = tid/32 + 8u, signal pl = tid%32): coalesced over signals
    const int pl = tid & 31;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int il = (tid >> 5) + 8 * u;
      const int gi = i0 + il;
      float2 z = make_float2(0.f, 0.f);
      if (gi < a.m) {
#pragma unroll
        for (int s = 0; s < kMaxSplit; ++s) {
          if (s < a.S) {
            const float2 c =
                *reinterpret_cast<const float2*>(&a.split[((long long)s * a.m + gi) * a.q_ld + 2 * (p0 + pl)]);
            z.x += c.x;
            z.y += c.y;
          }
        }
      }
      zs[il][pl] = z;
    }
  }
  __syncthreads();
  // apply: thread (signal pl = tid/8, rows 8*(tid&7) .. +8): coalesced over rows
  const int pl = tid >> 3;
  const int p = p0 + pl;
  const int ib = (tid & 7) * 8;
  float part = 0.f;
  float ybar = 0.f;
  if constexpr (EPI == E1_SPEC) ybar = p < a.nb ? (float)(a.ysum[p] / (double)a.m) : 0.f;
  if (p < a.nb) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int il = ib + q;
      const int gi = i0 + il;
      if (gi >= a.m) break;
      const float2 z = zs[il][pl];
      const long long o = (long long)p * a.m + gi;
      if constexpr (EPI == E1_STORE) {
        if (a.z_out) a.z_out[o] = z;
        if (a.y_out) a.y_out[o] = cabs2(z);
      } else if constexpr (EPI == E1_GD) {
        const float z2 = cabs2(z), yy = a.y[o];
        if (a.loss == LOSS_POISSON) {
          part += poisson_term(z2, yy, a.loss_eps);
          a.z_out[o] = cscale(z, poisson_weight(z2, yy, a.loss_eps));
        } else {
          const float d = z2 - yy;
          part += d * d;
          a.z_out[o] = cscale(z, d);
        }
      } else {
        const float yy = a.y[o];
        float w = a.lam;
        if (yy > 0.f) w = fmaxf(1.f - ybar / yy, a.lam);
        a.z_out[o] = cscale(z, w);
      }
    }
  }
  if constexpr (EPI == E1_GD) {
    // per-signal partials: the 8 threads of signal pl are consecutive
    red[tid] = part;
    __syncthreads();
    if ((tid & 7) == 0 && p < a.nb) {
      float t = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) t += red[tid + q];
      a.part[(long long)p * a.part_ld + blockIdx.x] = t;
    }
  }
}

// Epilogue after A^H R: g_pk = (P[2k][2p] + P[2k+1][2p+1]) + i (P[2k][2p+1] -
// P[2k+1][2p]), P = sum_s P_s, for 32 entries k and 32 signals, then the E2
// arithmetic.  grid (k tiles of 32, signal tiles).
template <int EPI>
__global__ void __launch_bounds__(NT) dense_epi2_kernel(const DenseArgs a) {
  __shared__ float red[NT];
  const int tid = threadIdx.x;
  const int pl = tid >> 3;
  const int p = blockIdx.y * 32 + pl;
  const int kb = blockIdx.x * 32 + (tid & 7) * 4;
  const int J = 2 * a.n;
  float part = 0.f;
  bool bad = false;
  if (p < a.nb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int gk = kb + q;
      if (gk >= a.n) break;
      float2 re = make_float2(0.f, 0.f), im = make_float2(0.f, 0.f);  // (P[2k][2p], P[2k+1][2p]), (.., 2p+1)
#pragma unroll
      for (int s = 0; s < kMaxSplit; ++s) {
        if (s < a.S) {
          const float2 u = *reinterpret_cast<const float2*>(&a.split[((long long)s * a.q_ld + 2 * p) * J + 2 * gk]);
          const float2 v =
              *reinterpret_cast<const float2*>(&a.split[((long long)s * a.q_ld + 2 * p + 1) * J + 2 * gk]);
          re.x += u.x;
          re.y += u.y;
          im.x += v.x;
          im.y += v.y;
        }
      }
      const float2 gv = make_float2(re.x + im.y, im.x - re.y);
      const long long o = (long long)p * a.n + gk;
      if constexpr (EPI == E2_STORE) {
        a.x[o] = cscale(gv, a.step);
      } else if constexpr (EPI == E2_GD) {
        const float2 xo = a.x[o];
        const float2 nx = make_float2(xo.x - a.step * gv.x, xo.y - a.step * gv.y);
        a.x[o] = nx;
        bad |= !finite2(nx);
      } else {
        // u_new = step * M v - 2 lambda v, v = u / ||u|| (the 1/||u|| was applied to R's source in A X)
        const float2 uo = a.x[o];
        const float c = 2.f * a.lam * a.prev_scale[p];
        const float2 nu = make_float2(a.step * gv.x - c * uo.x, a.step * gv.y - c * uo.y);
        a.x[o] = nu;
        part += cabs2(nu);
        bad |= !finite2(nu);
      }
    }
  }
  if constexpr (EPI == E2_GD || EPI == E2_SPEC) flag_nonfinite(a.nf, bad);
  if constexpr (EPI == E2_SPEC) {
    red[tid] = part;
    __syncthreads();
    if ((tid & 7) == 0 && p < a.nb) {
      float t = 0.f;
#pragma unroll
      for (int q = 0; q < 8; ++q) t += red[tid + q];
      a.part[(long long)p * a.part_ld + blockIdx.x] = t;
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
// (a NaN or Inf in the estimate raises the flag nf)
__global__ void dense_final_scale_kernel(float2* x, int n, int nb, const double* ysum, const float* inv,
                                         float inv_mc, unsigned* nf) {
  const long long tot = (long long)n * nb;
  bool bad = false;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(e / n);
    const float2 v = cscale(x[e], (float)sqrt(ysum[p] * (double)inv_mc) * inv[p]);
    x[e] = v;
    bad |= !finite2(v);
  }
  flag_nonfinite(nf, bad);
}

// ---- the library GEMM (hipBLASLt) for the two real products
// The same products as dense_mm_kernel with S = 1, in column-major terms
// (A's floats are the column-major 2n x m matrix At_cm, leading dimension 2n):
//   A X  : D1 (q x m)  = Bxt (q x 2n) . At_cm,   Bxt = Bx^T, q = 64 per signal tile;
//   A^H R: D2 (2n x q) = At_cm . Br (m x q),     Br[i][2p] = Re r_pi, [2p+1] = Im r_pi.
// D1 and D2 land in the split buffer in exactly the layouts the epilogue
// kernels read for one partial, so the epilogues are shared.

// Bxt (q x 2n, column-major, leading dimension q) from the signals x (nb x n)
__global__ void pack_bx_kernel(const float2* __restrict__ x, const float* __restrict__ scale, int n, int nb, int q,
                               float* __restrict__ bxt) {
  const long long tot = (long long)n * q / 2;  // (signal slot, k) pairs
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int ps = (int)(e % (q / 2));
    const int k = (int)(e / (q / 2));
    float2 v = make_float2(0.f, 0.f);
    if (ps < nb) v = cscale(x[(long long)ps * n + k], scale != nullptr ? scale[ps] : 1.f);
    float* c0 = bxt + (long long)(2 * k) * q + 2 * ps;      // column 2k
    float* c1 = bxt + (long long)(2 * k + 1) * q + 2 * ps;  // column 2k+1
    c0[0] = v.x;
    c0[1] = v.y;
    c1[0] = -v.y;
    c1[1] = v.x;
  }
}

// Br (m x q, column-major, leading dimension m) from the residuals r (nb x m)
__global__ void pack_br_kernel(const float2* __restrict__ r, const float* __restrict__ scale, int m, int nb, int q,
                               float* __restrict__ br) {
  const long long tot = (long long)m * (q / 2);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % m);
    const int ps = (int)(e / m);
    float2 v = make_float2(0.f, 0.f);
    if (ps < nb) v = cscale(r[(long long)ps * m + i], scale != nullptr ? scale[ps] : 1.f);
    br[(long long)(2 * ps) * m + i] = v.x;
    br[(long long)(2 * ps + 1) * m + i] = v.y;
  }
}

}  // namespace

constexpr int kLibCandidates = 8;  // library algorithms timed per product at plan creation

struct DenseLib {
  hipblasLtHandle_t h = nullptr;
  hipblasLtMatmulDesc_t desc = nullptr;
  hipblasLtMatrixLayout_t l1[3] = {nullptr, nullptr, nullptr};  // Bxt, At_cm, D1
  hipblasLtMatrixLayout_t l2[3] = {nullptr, nullptr, nullptr};  // At_cm, Br, D2
  hipblasLtMatmulAlgo_t algo[2];
  bool ok[2] = {false, false};   // the product has a library algorithm
  bool use[2] = {false, false};  // the product runs on it (else dense_mm_kernel)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  float* pack = nullptr;  // Bxt or Br
  ~DenseLib() {
    for (auto l : l1)
      if (l) (void)hipblasLtMatrixLayoutDestroy(l);
    for (auto l : l2)
      if (l) (void)hipblasLtMatrixLayoutDestroy(l);
    if (desc) (void)hipblasLtMatmulDescDestroy(desc);
    if (h) (void)hipblasLtDestroy(h);
    if (ws) (void)hipFree(ws);
    if (pack) (void)hipFree(pack);
  }
};

void destroy_dense_lib(DenseLib* d) { delete d; }

namespace {

constexpr size_t kLibWorkspace = size_t(64) << 20;

// Reduction splits of one product: about kTargetGroups workgroups, every
// split a whole number of BK chunks.
void plan_split(int tiles, int K, int* S, int* kchunk) {
  const int chunks = (K + BK - 1) / BK;
  int want = std::max(1, std::min(std::min(chunks, kMaxSplit), (kTargetGroups + tiles - 1) / tiles));
  const int per = (chunks + want - 1) / want;
  *kchunk = per * BK;
  *S = (chunks + per - 1) / per;
}

int signal_tiles(const DenseArgs& a) { return (a.nb + 31) / 32; }

// The product of kind G: on the library (lib != nullptr and chosen for G)
// or on dense_mm_kernel; then the epilogue EPI.
template <int G, int EPI>
hipError_t gemm(DenseArgs a, float* split, hipStream_t st, const DenseLib* lib = nullptr) {
  const int M = G == 1 ? a.m : 2 * a.n;
  const int K = G == 1 ? 2 * a.n : a.m;
  const int tiles = (M + BT - 1) / BT;
  a.split = split;
  a.q_ld = 64 * signal_tiles(a);
  hipError_t e = hipSuccess;
  if (lib != nullptr && lib->use[G - 1]) {
    a.S = 1;
    const long long pairs = G == 1 ? (long long)a.n * a.q_ld / 2 : (long long)a.m * (a.q_ld / 2);
    const int groups = (int)std::min<long long>((pairs + 255) / 256, 8192);
    if constexpr (G == 1)
      hipLaunchKernelGGL(pack_bx_kernel, dim3(groups), dim3(256), 0, st, a.src, a.src_scale, a.n, a.nb, a.q_ld,
                         lib->pack);
    else
      hipLaunchKernelGGL(pack_br_kernel, dim3(groups), dim3(256), 0, st, a.src, a.src_scale, a.m, a.nb, a.q_ld,
                         lib->pack);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const float one = 1.f, zero = 0.f;
    const hipblasLtMatrixLayout_t* l = G == 1 ? lib->l1 : lib->l2;
    const void* opA = G == 1 ? (const void*)lib->pack : (const void*)a.A;
    const void* opB = G == 1 ? (const void*)a.A : (const void*)lib->pack;
    const hipblasStatus_t bs = hipblasLtMatmul(lib->h, lib->desc, &one, opA, l[0], opB, l[1], &zero, split, l[2],
                                               split, l[2], &lib->algo[G - 1], lib->ws, lib->ws_bytes, st);
    if (bs != HIPBLAS_STATUS_SUCCESS) return hipErrorLaunchFailure;
  } else {
    plan_split(tiles * signal_tiles(a), K, &a.S, &a.kchunk);
    hipLaunchKernelGGL((dense_mm_kernel<G>), dim3(tiles * a.S, signal_tiles(a)), dim3(NT), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if constexpr (G == 1) {
    hipLaunchKernelGGL((dense_epi1_kernel<EPI>), dim3(tiles, signal_tiles(a)), dim3(NT), 0, st, a);
  } else {
    hipLaunchKernelGGL((dense_epi2_kernel<EPI>), dim3((a.n + 31) / 32, signal_tiles(a)), dim3(NT), 0, st, a);
  }
  return hipGetLastError();
}

DenseArgs base(const sr_plan_s* p) {
  DenseArgs a{};
  a.A = (const float*)p->dense_A;
  a.m = (int)p->geo[0].m;
  a.n = (int)p->geo[0].n;
  a.nb = (int)p->geo.size();
  a.nf = p->sync + 2;
  return a;
}

int row_tiles_g1(const DenseArgs& a) { return (a.m + BT - 1) / BT; }
int row_tiles_g2(const DenseArgs& a) { return (a.n + 31) / 32; }

#define DN_HIP(x)                                     \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) return hip_fail(e_, #x);    \
  } while (0)

}  // namespace

// Floats of split-reduction partials a dense plan of this shape needs: the
// larger of the two products' S x (rows) x (64 per signal tile).
size_t dense_split_floats(int m, int n, int nb) {
  DenseArgs a{};
  a.m = m;
  a.n = n;
  a.nb = nb;
  const int st = signal_tiles(a);
  int S1, S2, kc;
  plan_split(((m + BT - 1) / BT) * st, 2 * n, &S1, &kc);
  plan_split(((2 * n + BT - 1) / BT) * st, m, &S2, &kc);
  const size_t f1 = (size_t)S1 * m * 64 * st;
  const size_t f2 = (size_t)S2 * 2 * n * 64 * st;
  return std::max(f1, f2);
}

// Scratch layout for dense plans: bufA holds R (nb x m complex); fscratch
// holds per-signal scalars; part holds per-signal partials.
sr_status dense_lib_setup(sr_plan_s* p) {
  const char* force = std::getenv("SR_DENSE_GEMM");
  if (force != nullptr && std::strcmp(force, "own") == 0) return SR_OK;
  DenseArgs a = base(p);
  const uint64_t q = 64 * (uint64_t)signal_tiles(a), m = (uint64_t)a.m, n2 = 2 * (uint64_t)a.n;
  DenseLib* d = new (std::nothrow) DenseLib();
  if (d == nullptr) return SR_OK;
  auto give_up = [&]() {
    delete d;
    return SR_OK;  // the hand-written products serve every plan
  };
  if (hipblasLtCreate(&d->h) != HIPBLAS_STATUS_SUCCESS) return give_up();
  if (hipblasLtMatmulDescCreate(&d->desc, HIPBLAS_COMPUTE_32F, HIP_R_32F) != HIPBLAS_STATUS_SUCCESS) return give_up();
  if (hipblasLtMatrixLayoutCreate(&d->l1[0], HIP_R_32F, q, n2, (int64_t)q) != HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatrixLayoutCreate(&d->l1[1], HIP_R_32F, n2, m, (int64_t)n2) != HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatrixLayoutCreate(&d->l1[2], HIP_R_32F, q, m, (int64_t)q) != HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatrixLayoutCreate(&d->l2[0], HIP_R_32F, n2, m, (int64_t)n2) != HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatrixLayoutCreate(&d->l2[1], HIP_R_32F, m, q, (int64_t)m) != HIPBLAS_STATUS_SUCCESS ||
      hipblasLtMatrixLayoutCreate(&d->l2[2], HIP_R_32F, n2, q, (int64_t)n2) != HIPBLAS_STATUS_SUCCESS)
    return give_up();
  hipblasLtMatmulPreference_t pref = nullptr;
  if (hipblasLtMatmulPreferenceCreate(&pref) != HIPBLAS_STATUS_SUCCESS) return give_up();
  const uint64_t wmax = kLibWorkspace;
  (void)hipblasLtMatmulPreferenceSetAttribute(pref, HIPBLASLT_MATMUL_PREF_MAX_WORKSPACE_BYTES, &wmax, sizeof(wmax));
  // up to kLibCandidates of the library's algorithms per product, in its
  // heuristic's order
  hipblasLtMatmulAlgo_t cand[2][kLibCandidates];
  int ncand[2] = {0, 0};
  size_t need = 0;
  for (int g = 0; g < 2; ++g) {
    const hipblasLtMatrixLayout_t* l = g == 0 ? d->l1 : d->l2;
    hipblasLtMatmulHeuristicResult_t res[kLibCandidates];
    int cnt = 0;
    if (hipblasLtMatmulAlgoGetHeuristic(d->h, d->desc, l[0], l[1], l[2], l[2], pref, kLibCandidates, res, &cnt) !=
        HIPBLAS_STATUS_SUCCESS)
      cnt = 0;
    for (int i = 0; i < cnt; ++i) {
      if (res[i].state != HIPBLAS_STATUS_SUCCESS) continue;
      cand[g][ncand[g]++] = res[i].algo;
      need = std::max(need, res[i].workspaceSize);
    }
    if (ncand[g] > 0) {
      d->algo[g] = cand[g][0];
      d->ok[g] = true;
    }
  }
  (void)hipblasLtMatmulPreferenceDestroy(pref);
  if (!d->ok[0] && !d->ok[1]) return give_up();
  if (need > 0 && hipMalloc(&d->ws, need) != hipSuccess) return give_up();
  d->ws_bytes = need;
  if (hipMalloc(&d->pack, sizeof(float) * std::max(q * n2, m * q)) != hipSuccess) return give_up();
  // per product: the fastest of dense_mm_kernel and the library's candidates
  // (best of three applications each after a warm-up, on the plan's own
  // matrix; the source is scratch of the right size, the epilogue writes
  // nothing but scratch); SR_DENSE_GEMM=lib leaves dense_mm_kernel out
  const bool all_lib = force != nullptr && std::strcmp(force, "lib") == 0;
  const bool can_time = (size_t)a.n <= (size_t)a.m;  // bufB (m x nb) holds the A^H R output
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!can_time || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    if (!all_lib) return give_up();
    for (int g = 0; g < 2; ++g) d->use[g] = d->ok[g];  // the heuristic's first choice, untimed
    e0 = e1 = nullptr;
  } else {
    for (int g = 0; g < 2; ++g) {
      if (!d->ok[g]) continue;
      auto time_it = [&]() -> float {
        DenseArgs t = a;
        t.src = p->bufA;
        t.x = p->bufB;
        t.step = 1.f;
        float best = 1e30f;
        for (int rep = 0; rep < 4; ++rep) {
          (void)hipEventRecord(e0, p->stream);
          const hipError_t e = g == 0 ? gemm<1, E1_STORE>(t, p->dsplit, p->stream, d)
                                      : gemm<2, E2_STORE>(t, p->dsplit, p->stream, d);
          (void)hipEventRecord(e1, p->stream);
          if (e != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 1e30f;
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (rep > 0) best = std::min(best, ms);  // the first is a warm-up
        }
        return best;
      };
      float best = 1e30f;
      int pick = -1;  // -1: dense_mm_kernel
      if (!all_lib) {
        d->use[g] = false;
        best = time_it();
      }
      d->use[g] = true;
      for (int c = 0; c < ncand[g]; ++c) {
        d->algo[g] = cand[g][c];
        const float t = time_it();
        if (t < best) {
          best = t;
          pick = c;
        }
      }
      if (all_lib && pick < 0) pick = 0;
      d->use[g] = pick >= 0;
      if (pick >= 0) d->algo[g] = cand[g][pick];
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (hipStreamSynchronize(p->stream) != hipSuccess) return give_up();
  if (!d->use[0] && !d->use[1]) return give_up();
  p->dense_lib = d;
  return SR_OK;
}

sr_status dense_forward(sr_plan_s* p, const float2* x, float2* z, float* y) {
  DenseArgs a = base(p);
  a.src = x;
  a.z_out = z;
  a.y_out = y;
  DN_HIP((gemm<1, E1_STORE>(a, p->dsplit, p->stream, p->dense_lib)));
  return SR_OK;
}

sr_status dense_adjoint(sr_plan_s* p, const float2* r, float2* x) {
  DenseArgs a = base(p);
  a.src = r;
  a.x = x;
  a.step = 1.f;
  DN_HIP((gemm<2, E2_STORE>(a, p->dsplit, p->stream, p->dense_lib)));
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
    g1.loss = p->loss;
    g1.loss_eps = p->loss_eps;
    DN_HIP((gemm<1, E1_GD>(g1, p->dsplit, p->stream, p->dense_lib)));
    if (loss_trace) {
      hipLaunchKernelGGL(sum_rows_kernel, dim3((a.nb + 63) / 64), dim3(64), 0, p->stream, p->part, t1, t1, a.nb,
                         loss_trace + it, iters);
      DN_HIP(hipGetLastError());
    }
    DenseArgs g2 = a;
    g2.src = p->bufA;
    g2.x = x;
    g2.step = eta[0] / (float)a.m;
    DN_HIP((gemm<2, E2_GD>(g2, p->dsplit, p->stream, p->dense_lib)));
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
    DN_HIP((gemm<1, E1_SPEC>(g1, p->dsplit, p->stream, p->dense_lib)));
    DenseArgs g2 = a;  // u <- A^H r / (m c) - 2 lambda u / ||u||
    g2.src = p->bufA;
    g2.x = x0;
    g2.step = inv_mc;
    g2.lam = lam;
    g2.prev_scale = inv;
    g2.part = p->part;
    g2.part_ld = t2;
    DN_HIP((gemm<2, E2_SPEC>(g2, p->dsplit, p->stream, p->dense_lib)));
    cnt = t2;
  }
  hipLaunchKernelGGL(inv_norms_kernel, dim3((a.nb + 63) / 64), dim3(64), 0, p->stream, p->part, t2, cnt, a.nb, inv);
  DN_HIP(hipGetLastError());
  const long long tot = (long long)a.n * a.nb;
  const int groups = (int)std::min<long long>((tot + 255) / 256, 2048);
  hipLaunchKernelGGL(dense_final_scale_kernel, dim3(groups), dim3(256), 0, p->stream, x0, a.n, a.nb, ysum, inv, inv_mc,
                     a.nf);
  DN_HIP(hipGetLastError());
  return SR_OK;
}

}  // namespace sr
