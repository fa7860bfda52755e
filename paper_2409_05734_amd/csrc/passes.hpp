// Fused FFT pass kernels for the 2D structured operator.
//
// The 2D unitary DFT factors into commuting axis transforms F = F_1 F_0.
// Layer l of A = F D_L ... F D_1 U applies its two axis transforms in the
// order (0,1) when l is odd and (1,0) when l is even, so consecutive
// transforms along the same axis meet and fuse with the phase diagonal
// between them.  One pass = one read and one write of the m-grid:
//
//   forward : [U D_1 F_0] [F_1 D_2 F_1] [F_0 D_3 F_0] ... [F_a -> z, |z|^2]
//   adjoint : [F_a^H] ... [F_0^H D_3^* F_0^H] [F_1^H D_2^* F_1^H] [F_0^H D_1^* U^H]
//   GD/spectral iteration: forward passes, a turnaround pass
//   [F_a -> residual or spectral weight -> F_a^H], then the adjoint passes,
//   the last of which also applies the solver update.
//
// Column-mode passes (transforms along axis 0) read and write tiles of B
// adjacent columns; row-mode passes tiles of B rows.  Passes next to the
// zero-padded support only touch the N_2 support columns ("compact" buffers).
#pragma once
#include "fft_core.hpp"

namespace sr {

enum PreOp : int { PRE_NONE = 0, PRE_PHASE = 1 };
enum MidOp : int {
  MID_NONE = 0,
  MID_PHASE = 1,            // v <- D v
  MID_PHASE_CONJ = 2,       // v <- D^* v
  MID_GD = 3,               // v <- (|v|^2 - y) v, loss partials
  MID_SPEC = 4,             // v <- T(y) v
  MID_STORE = 5,            // z <- v, |z|^2
  // reverse-mode variants (value u after the first transform; save/gth per layer)
  MID_PHASE_SAVE = 6,       // u <- D v, save <- u                  (forward recompute)
  MID_PHASE_CONJ_GT = 7,    // gth += Im(v conj(save)), v <- D^* v   (forward VJP)
  MID_PHASE_CONJ_SAVE = 8,  // q <- D^* v, save <- q                (adjoint recompute)
  MID_PHASE_GT = 9          // gth += Im(conj(v) save), v <- D v     (adjoint VJP)
};
enum PostOp : int {
  POST_STORE = 0,
  POST_PHASE_CONJ_STORE = 1,
  POST_GD = 2,            // x <- x - step g
  POST_SPEC = 3,          // u <- s (step g - 2 lambda u), s = 1/||u|| (deferred normalisation)
  POST_PHASE_CONJ_GT = 4,  // gth_1 += Im(v conj(D_1 U x)), then D_1^* and crop
  // the next iteration's first pass fused behind the update: the new iterate,
  // still in registers, is padded, multiplied by D_1 and transformed along
  // axis 0 into out2 (the compact buffer the next row pass reads)
  POST_GD_FWD = 5,
  POST_SPEC_FWD = 6
};

struct PassArgs {
  // input buffer: element (transform b, position k) for k in [in_lo, in_hi)
  // row mode: in[b*in_ld + k - in_lo]; column mode: in[(k - in_lo)*in_ld + b]
  const float2* in;
  long long in_ld;
  int in_lo, in_hi;
  // output buffer with the same addressing over the window [out_lo, out_hi)
  float2* out;
  long long out_ld;
  int out_lo, out_hi;
  int ntr;            // number of transforms (rows or columns) in this pass
  int tr_lo;          // grid coordinate of transform 0 on the other axis
  long long grid_ld;  // M2, row stride of the full measurement grid
  const float2* tw;   // exp(-2 pi i e/N), e = 0..N-1
  const float* th_pre;
  const float* th_mid;
  const float* th_post;
  // optional precomputed exp(i theta) tables for the same diagonals; when
  // set they replace the phases (one 8-byte load instead of sincos)
  const float2* ep_pre;
  const float2* ep_mid;
  const float2* ep_post;
  float scale_pre, scale_mid, scale_out;
  // epilogues
  const float* y;        // measurements on the grid (MID_GD, MID_SPEC)
  const double* ysum;    // sum(y) (MID_SPEC)
  float inv_m;           // 1/m
  float lam;             // spectral threshold lambda
  float2* z_out;         // MID_STORE: z = A x on the grid (nullable)
  float* y_out;          // MID_STORE: |z|^2 on the grid (nullable)
  float* part_out;       // per-workgroup partial sums (loss or squared norm), nullable
  const float* part_in;  // squared-norm partials of the previous iterate (spectral), nullable
  int npart;
  // solver updates (POST_GD, POST_SPEC)
  float step;            // GD: eta/m; spectral: 1/(m c)
  float two_lam;         // spectral: 2 lambda
  // reverse mode
  float2* save;          // per-layer intermediate on the grid (written or read)
  float* gth;            // phase-cotangent accumulator of this pass's diagonal (grid layout)
  const float2* xin;     // POST_PHASE_CONJ_GT: the signal x (crop layout = output layout)
  float2* out2;          // POST_*_FWD: compact output of the fused forward transform
  long long out2_ld;
};

// Sum of previous-iterate partials, identical on every thread (fixed order).
__device__ __forceinline__ float inv_norm_from_partials(const float* part, int n) {
  double acc = 0.0;
  for (int i = 0; i < n; ++i) acc += (double)part[i];
  return (float)(1.0 / sqrt(acc));
}

// One tile (B transforms) of a fused pass.  `lds` holds 2*B*N complex
// elements, `red` one float per thread.  part_in/npart/part_out override the
// partial-sum pointers of `a` (persistent kernels alternate them per
// iteration); partial sums are written at index `tile`.
//
// Every global load the tile needs (input, phases, measurements, twiddles,
// the previous iterate) is issued up front, so a pass costs one memory
// round trip plus its arithmetic, not one round trip per stage.
template <int N, int B, bool COL, int PRE, int MID, bool FFT2, bool INV1, bool INV2, int POST, bool DB = true>
__device__ __forceinline__ void pass_tile(const PassArgs& a, int tile, float2* lds, float* red, const float* part_in,
                                          int npart, float* part_out) {
  using T = Tile<N, B, COL, DB>;
  constexpr int E = T::E;
  constexpr bool MID_PH = (MID == MID_PHASE || MID == MID_PHASE_CONJ || MID >= MID_PHASE_SAVE);
  constexpr bool MID_SAVED = (MID == MID_PHASE_CONJ_GT || MID == MID_PHASE_GT);
  constexpr bool MID_Y = (MID == MID_GD || MID == MID_SPEC);
  constexpr bool POST_PH = (POST != POST_STORE);
  constexpr bool POST_X = (POST == POST_GD || POST == POST_SPEC || POST == POST_GD_FWD || POST == POST_SPEC_FWD);
  constexpr bool POST_FWD = (POST == POST_GD_FWD || POST == POST_SPEC_FWD);
  constexpr bool POST_IS_GD = (POST == POST_GD || POST == POST_GD_FWD);
  constexpr bool POST_IS_SPEC = (POST == POST_SPEC || POST == POST_SPEC_FWD);
  const int t = T::thread_t();
  const int bl = T::thread_b();
  const int b = tile * B + bl;
  const bool active = b < a.ntr;
  const int gb = a.tr_lo + b;  // grid coordinate of this transform

  auto gidx = [&](int k) -> long long {
    return COL ? (long long)k * a.grid_ld + gb : (long long)gb * a.grid_ld + k;
  };
  auto in_addr = [&](int k) -> long long {
    return COL ? (long long)(k - a.in_lo) * a.in_ld + b : (long long)b * a.in_ld + (k - a.in_lo);
  };
  auto out_addr = [&](int k) -> long long {
    return COL ? (long long)(k - a.out_lo) * a.out_ld + b : (long long)b * a.out_ld + (k - a.out_lo);
  };
  auto in_win = [&](int k) { return active && k >= a.in_lo && k < a.in_hi; };
  auto out_win = [&](int k) { return active && k >= a.out_lo && k < a.out_hi; };

  // ---- issue every global load
  float2 v[E];
  float2 dp[E];   // pre-diagonal entries e^{i theta}
  float2 dm[E];   // mid-diagonal entries
  float yv[E];    // measurements
  float2 dq[E];   // post-diagonal entries
  float2 xo[E];   // previous iterate (or x for POST_PHASE_CONJ_GT)
  float2 sv[E];   // saved intermediate
  float gt[E];    // phase-cotangent accumulator
  typename T::Twiddles w;
  T::load_twiddles(w, a.tw, t);
  const bool tab_pre = a.ep_pre != nullptr;
  const bool tab_mid = a.ep_mid != nullptr;
  const bool tab_post = a.ep_post != nullptr;
  const float2 one = make_float2(1.f, 0.f);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int k = T::elem(t, j);
    const bool iw = in_win(k);
    v[j] = iw ? a.in[in_addr(k)] : make_float2(0.f, 0.f);
    if constexpr (PRE == PRE_PHASE) {
      if (tab_pre) dp[j] = iw ? a.ep_pre[gidx(k)] : one;
      else dp[j].x = iw ? a.th_pre[gidx(k)] : 0.f;
    }
    if constexpr (MID_PH) {
      if (tab_mid) dm[j] = active ? a.ep_mid[gidx(k)] : one;
      else dm[j].x = active ? a.th_mid[gidx(k)] : 0.f;
    }
    if constexpr (MID_Y) yv[j] = active ? a.y[gidx(k)] : 0.f;
    if constexpr (MID_SAVED) {
      sv[j] = active ? a.save[gidx(k)] : make_float2(0.f, 0.f);
      gt[j] = active ? a.gth[gidx(k)] : 0.f;
    }
    if constexpr (MID != MID_STORE) {
      const bool ow = out_win(k);
      if constexpr (POST_PH) {
        if (tab_post) dq[j] = ow ? a.ep_post[gidx(k)] : one;
        else dq[j].x = ow ? a.th_post[gidx(k)] : 0.f;
      }
      if constexpr (POST_X) xo[j] = ow ? a.out[out_addr(k)] : make_float2(0.f, 0.f);
      if constexpr (POST == POST_PHASE_CONJ_GT) {
        xo[j] = ow ? a.xin[out_addr(k)] : make_float2(0.f, 0.f);
        gt[j] = ow ? a.gth[gidx(k)] : 0.f;
      }
    }
  }
  // phases -> diagonal entries where no table was given
#pragma unroll
  for (int j = 0; j < E; ++j) {
    if constexpr (PRE == PRE_PHASE)
      if (!tab_pre) dp[j] = phase<false>(dp[j].x, 1.f);
    if constexpr (MID_PH)
      if (!tab_mid) dm[j] = phase<false>(dm[j].x, 1.f);
    if constexpr (POST_PH)
      if (!tab_post) dq[j] = phase<false>(dq[j].x, 1.f);
  }

  float s_pre = a.scale_pre;
  float s_prev = 1.f;  // 1/||u_prev|| for the spectral update
  if (part_in != nullptr) {
    s_prev = inv_norm_from_partials(part_in, npart);
    if (PRE == PRE_PHASE) s_pre *= s_prev;
  }

  // ---- pre-diagonal, first transform
#pragma unroll
  for (int j = 0; j < E; ++j) {
    if constexpr (PRE == PRE_PHASE) v[j] = cmul(v[j], cscale(dp[j], s_pre));
    else v[j] = cscale(v[j], s_pre);
  }
  int ph = 0;
  T::template fft<INV1>(v, lds, ph, w, t, bl);

  // ---- mid operation
  float acc = 0.f;
  if constexpr (MID == MID_PHASE || MID == MID_PHASE_CONJ) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const float2 d = cscale(dm[j], a.scale_mid);
      v[j] = (MID == MID_PHASE_CONJ) ? cmulc(v[j], d) : cmul(v[j], d);
    }
  } else if constexpr (MID >= MID_PHASE_SAVE) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      const float2 u = cscale(v[j], a.scale_mid);
      if constexpr (MID == MID_PHASE_SAVE) {
        v[j] = cmul(u, dm[j]);
        if (active) a.save[gidx(k)] = v[j];
      } else if constexpr (MID == MID_PHASE_CONJ_SAVE) {
        v[j] = cmulc(u, dm[j]);
        if (active) a.save[gidx(k)] = v[j];
      } else if constexpr (MID == MID_PHASE_CONJ_GT) {
        // Im(u conj(s)) = u.y s.x - u.x s.y
        if (active) a.gth[gidx(k)] = gt[j] + (u.y * sv[j].x - u.x * sv[j].y);
        v[j] = cmulc(u, dm[j]);
      } else {  // MID_PHASE_GT: Im(conj(u) s) = u.x s.y - u.y s.x
        if (active) a.gth[gidx(k)] = gt[j] + (u.x * sv[j].y - u.y * sv[j].x);
        v[j] = cmul(u, dm[j]);
      }
    }
  } else if constexpr (MID == MID_GD) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      float2 z = cscale(v[j], a.scale_mid);
      float d = cabs2(z) - yv[j];
      acc += active ? d * d : 0.f;
      v[j] = cscale(z, d);
    }
  } else if constexpr (MID == MID_SPEC) {
    const float ybar = (float)(*a.ysum * (double)a.inv_m);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      float2 z = cscale(v[j], a.scale_mid);
      float wgt = a.lam;
      if (yv[j] > 0.f) wgt = fmaxf(1.f - ybar / yv[j], a.lam);
      v[j] = cscale(z, wgt);
    }
  } else if constexpr (MID == MID_STORE) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      float2 z = cscale(v[j], a.scale_mid);
      if (active) {
        if (a.z_out) a.z_out[gidx(k)] = z;
        if (a.y_out) a.y_out[gidx(k)] = cabs2(z);
      }
    }
  }

  // ---- second transform, post-diagonal, update, store
  if constexpr (FFT2) T::template fft<INV2>(v, lds, ph, w, t, bl);

  if constexpr (MID != MID_STORE) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      float2 val = make_float2(0.f, 0.f);
      if (out_win(k)) {
        val = cscale(v[j], a.scale_out);
        if constexpr (POST == POST_PHASE_CONJ_GT) {
          const float2 u1 = cmul(xo[j], dq[j]);  // u_1 = D_1 U x at this position
          a.gth[gidx(k)] = gt[j] + (val.y * u1.x - val.x * u1.y);
        }
        if constexpr (POST_PH) val = cmulc(val, dq[j]);
        if constexpr (POST_IS_GD) {
          val = make_float2(xo[j].x - a.step * val.x, xo[j].y - a.step * val.y);
        } else if constexpr (POST_IS_SPEC) {
          val = make_float2(s_prev * (a.step * val.x - a.two_lam * xo[j].x),
                            s_prev * (a.step * val.y - a.two_lam * xo[j].y));
          acc += cabs2(val);
        }
        a.out[out_addr(k)] = val;
      }
      if constexpr (POST_FWD) v[j] = cmul(val, dq[j]);  // zero outside the support window
    }
  }

  if constexpr (POST_FWD) {
    T::template fft<false>(v, lds, ph, w, t, bl);
    const float s1 = a.scale_out;  // 1/sqrt(M1) for both transforms of this column pass
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      if (active) a.out2[(long long)k * a.out2_ld + b] = cscale(v[j], s1);
    }
  }

  if constexpr (MID == MID_GD || POST_IS_SPEC) {
    if (part_out != nullptr) {
      float sum = block_sum<T::THREADS>(acc, red);
      if (threadIdx.x == 0) part_out[tile] = sum;
    }
  }
}

template <int N, int B, bool COL, int PRE, int MID, bool FFT2, bool INV1, bool INV2, int POST, bool DB = true>
__global__ void __launch_bounds__((Tile<N, B, COL, DB>::THREADS)) pass_kernel(const PassArgs a) {
  extern __shared__ float2 lds[];
  __shared__ float red[Tile<N, B, COL, DB>::THREADS];
  pass_tile<N, B, COL, PRE, MID, FFT2, INV1, INV2, POST, DB>(a, xcd_tile(blockIdx.x, gridDim.x), lds, red, a.part_in,
                                                              a.npart, a.part_out);
}

}  // namespace sr
