// LDS-resident kernels for one-dimensional problems: the whole m-vector of a
// problem lives in one workgroup (registers + LDS), so an operator
// application, or every iteration of a GD / spectral solve, runs in a single
// launch with no global-memory round trip between layers or iterations.
//
// 1D operator (section III, Eq. (5)): A x = S F D_L ... F D_1 U x with F the
// unitary DFT on a grid of max(n, m) points, U the centred zero padding
// (m > n) and S the centred trimming to the m measurements (m < n).
#pragma once
#include "fft_core.hpp"
#include "loss.hpp"

namespace sr {

// Capacity of the per-workgroup table of layer phases (L*m entries).
constexpr int kFused1DPhaseSlots = 4096;

enum Fused1DOp : int { F1_FORWARD = 0, F1_ADJOINT = 1, F1_GD = 2, F1_SPECTRAL = 3, F1_FWD_VJP = 4, F1_ADJ_VJP = 5 };

struct Fused1DArgs {
  int n, m, L, off;          // signal length, grid length, layers, pad offset
  int mw, moff;              // measurement window [moff, moff + mw) of the grid
  const float* theta;        // L*m phases
  const float2* tw;          // exp(-2 pi i e/m), e = 0..m-1
  const float2* x_in;        // forward: x; spectral: v0
  float2* x_out;             // adjoint / spectral: output; GD: iterate (in place)
  const float2* r_in;        // adjoint input
  float2* z_out;             // forward: z (nullable)
  float* y_out;              // forward: |z|^2 (nullable)
  const float* y;            // GD / spectral measurements
  int iters;
  float step;                // GD: eta/m; spectral: 1/(m c)
  float lam;                 // spectral lambda
  float* loss_trace;         // GD: loss before each step (nullable)
  int loss;                  // GD: LOSS_L2 or LOSS_POISSON
  float loss_eps;            // GD: Poisson guard
  float* gth;                // derivatives: phase-cotangent accumulator (L*m)
  unsigned* nf;              // GD / spectral: set to 1 when the result holds NaN or Inf (nullable)
};

// The transform shape of the 1D kernels: the narrow shape (four elements per
// thread, twice the threads) where the length has one.  A single 1D problem
// is one workgroup whose whole solve is a chain of dependent transforms, so
// its time is the chain's latency: halving each lane's arithmetic shortens
// it more than the extra exchange stage lengthens it (the default shape of
// the shorter lengths does not even fill one wave).
// (The host passes the matching twiddle table: the narrow one where the
// length has it.)
template <int N>
using F1Tile = TileV<N, 1, false, true, HasNarrow<N>::value ? 1 : 0>;

template <int N, int OP>
__device__ __forceinline__ void fused1d_body(const Fused1DArgs& a) {
  using T = F1Tile<N>;
  constexpr int E = T::E;
  constexpr int NT = T::THREADS;
  __shared__ float2 lds[2 * T::BUF];
  __shared__ float2 dl[kFused1DPhaseSlots];  // e^{i theta_l}, L*m <= slots
  __shared__ float red[NT];
  const int t = threadIdx.x;
  const float s = rsqrtf((float)N);
  const int L = a.L;

  for (int e = t; e < L * N; e += NT) {
    float sn, cs;
    sincosf(a.theta[e], &sn, &cs);
    dl[e] = make_float2(cs, sn);
  }
  __syncthreads();

  auto in_window = [&](int k) { return k >= a.off && k < a.off + a.n; };
  auto in_meas = [&](int k) { return k >= a.moff && k < a.moff + a.mw; };  // measurement window
  typename T::Twiddles w;
  T::load_twiddles(w, a.tw, t);
  int ph = 0;
  float2 v[E];

  // forward layers from v = U x (already in registers); leaves z = A x in v
  auto forward_layers = [&]() {
    for (int l = 0; l < L; ++l) {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = cmul(v[j], dl[l * N + T::elem(t, j)]);
      T::template fft<false>(v, lds, ph, w, t, 0);
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = cscale(v[j], s);
    }
  };
  // adjoint layers from v = r; leaves D_1^* F^H ... in v (crop left to caller)
  auto adjoint_layers = [&]() {
    for (int l = L - 1; l >= 0; --l) {
      T::template fft<true>(v, lds, ph, w, t, 0);
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = cscale(cmulc(v[j], dl[l * N + T::elem(t, j)]), s);
    }
  };

  if constexpr (OP == F1_FORWARD) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      v[j] = in_window(k) ? a.x_in[k - a.off] : make_float2(0.f, 0.f);
    }
    forward_layers();
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      if (!in_meas(k)) continue;
      if (a.z_out) a.z_out[k - a.moff] = v[j];
      if (a.y_out) a.y_out[k - a.moff] = cabs2(v[j]);
    }
  } else if constexpr (OP == F1_ADJOINT) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      v[j] = in_meas(k) ? a.r_in[k - a.moff] : make_float2(0.f, 0.f);
    }
    adjoint_layers();
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      if (in_window(k)) a.x_out[k - a.off] = v[j];
    }
  } else if constexpr (OP == F1_GD) {
    float2 x[E];
    float yv[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      x[j] = in_window(k) ? a.x_out[k - a.off] : make_float2(0.f, 0.f);
      yv[j] = in_meas(k) ? a.y[k - a.moff] : 0.f;
    }
    for (int it = 0; it < a.iters; ++it) {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = x[j];
      forward_layers();
      float acc = 0.f;
      if (a.loss == LOSS_POISSON) {
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const bool in = in_meas(T::elem(t, j));  // zero residual outside the window
          const float z2 = cabs2(v[j]);
          if (a.loss_trace) acc += in ? poisson_term(z2, yv[j], a.loss_eps) : 0.f;
          v[j] = cscale(v[j], in ? poisson_weight(z2, yv[j], a.loss_eps) : 0.f);
        }
      } else {
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const float d = in_meas(T::elem(t, j)) ? cabs2(v[j]) - yv[j] : 0.f;  // zero outside the window
          acc += d * d;
          v[j] = cscale(v[j], d);
        }
      }
      if (a.loss_trace) {
        float tot = block_sum<NT>(acc, red);
        if (t == 0) a.loss_trace[it] = tot;
      }
      adjoint_layers();
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k = T::elem(t, j);
        if (in_window(k)) x[j] = make_float2(x[j].x - a.step * v[j].x, x[j].y - a.step * v[j].y);
      }
    }
    bool bad = false;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      if (in_window(k)) {
        a.x_out[k - a.off] = x[j];
        bad |= !finite2(x[j]);
      }
    }
    flag_nonfinite(a.nf, bad);
  } else if constexpr (OP == F1_FWD_VJP) {
    // x_in = x, r_in = cotangent of A x; x_out = A^H gz (nullable); gth += dtheta
    __shared__ float2 sv[kFused1DPhaseSlots];  // u_l = D_l w_{l-1}
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      v[j] = in_window(k) ? a.x_in[k - a.off] : make_float2(0.f, 0.f);
    }
    for (int l = 0; l < L; ++l) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k = T::elem(t, j);
        v[j] = cmul(v[j], dl[l * N + k]);
        sv[l * N + k] = v[j];
      }
      T::template fft<false>(v, lds, ph, w, t, 0);
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = cscale(v[j], s);
    }
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      v[j] = in_meas(k) ? a.r_in[k - a.moff] : make_float2(0.f, 0.f);
    }
    for (int l = L - 1; l >= 0; --l) {
      T::template fft<true>(v, lds, ph, w, t, 0);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k = T::elem(t, j);
        const float2 u = cscale(v[j], s);
        const float2 su = sv[l * N + k];
        a.gth[l * N + k] += u.y * su.x - u.x * su.y;  // Im(u conj(u_l))
        v[j] = cmulc(u, dl[l * N + k]);
      }
    }
    if (a.x_out) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k = T::elem(t, j);
        if (in_window(k)) a.x_out[k - a.off] = v[j];
      }
    }
  } else if constexpr (OP == F1_ADJ_VJP) {
    // r_in = r, x_in = cotangent of A^H r; z_out = A gv (nullable); gth += dtheta
    __shared__ float2 sv[kFused1DPhaseSlots];  // q_l = D_l^* F^H s_l
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      v[j] = in_meas(k) ? a.r_in[k - a.moff] : make_float2(0.f, 0.f);
    }
    for (int l = L - 1; l >= 0; --l) {
      T::template fft<true>(v, lds, ph, w, t, 0);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k = T::elem(t, j);
        v[j] = cscale(cmulc(v[j], dl[l * N + k]), s);
        sv[l * N + k] = v[j];
      }
    }
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      v[j] = in_window(k) ? a.x_in[k - a.off] : make_float2(0.f, 0.f);
    }
    for (int l = 0; l < L; ++l) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k = T::elem(t, j);
        const float2 q = sv[l * N + k];
        a.gth[l * N + k] += v[j].x * q.y - v[j].y * q.x;  // Im(conj(qbar) q_l)
        v[j] = cmul(v[j], dl[l * N + k]);
      }
      T::template fft<false>(v, lds, ph, w, t, 0);
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = cscale(v[j], s);
    }
    if (a.z_out) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k = T::elem(t, j);
        if (in_meas(k)) a.z_out[k - a.moff] = v[j];
      }
    }
  } else {  // F1_SPECTRAL
    float yv[E];
    float2 u[E];
    float ys = 0.f, un = 0.f;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      yv[j] = in_meas(k) ? a.y[k - a.moff] : 0.f;
      ys += yv[j];
      u[j] = in_window(k) ? a.x_in[k - a.off] : make_float2(0.f, 0.f);
      un += cabs2(u[j]);
    }
    const float ysum = block_sum<NT>(ys, red);
    const float ybar = ysum / (float)a.mw;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      float w = a.lam;
      if (yv[j] > 0.f) w = fmaxf(1.f - ybar / yv[j], a.lam);
      yv[j] = in_meas(T::elem(t, j)) ? w : 0.f;  // yv now holds T(y), zero outside the window
    }
    float inv = rsqrtf(block_sum<NT>(un, red));
    for (int it = 0; it < a.iters; ++it) {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        u[j] = cscale(u[j], inv);  // v_k = u / ||u||
        v[j] = u[j];
      }
      forward_layers();
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = cscale(v[j], yv[j]);
      adjoint_layers();
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k = T::elem(t, j);
        float2 nu = make_float2(0.f, 0.f);
        if (in_window(k))
          nu = make_float2(a.step * v[j].x - 2.f * a.lam * u[j].x, a.step * v[j].y - 2.f * a.lam * u[j].y);
        u[j] = nu;
        acc += cabs2(nu);
      }
      inv = rsqrtf(block_sum<NT>(acc, red));
    }
    const float scale = sqrtf(ysum * a.step) * inv;  // sqrt(sum(y)/(m c)) / ||u||
    bool bad = false;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      if (in_window(k)) {
        const float2 o = cscale(u[j], scale);
        a.x_out[k - a.off] = o;
        bad |= !finite2(o);
      }
    }
    flag_nonfinite(a.nf, bad);
  }
}

// One problem per launch.
template <int N, int OP>
__global__ void __launch_bounds__((F1Tile<N>::THREADS)) fused1d_kernel(const Fused1DArgs a) {
  fused1d_body<N, OP>(a);
}

// Many problems of one length per launch, one workgroup each.
template <int N, int OP>
__global__ void __launch_bounds__((F1Tile<N>::THREADS)) fused1d_batch_kernel(const Fused1DArgs* __restrict__ as) {
  const Fused1DArgs a = as[blockIdx.x];
  fused1d_body<N, OP>(a);
}

}  // namespace sr
