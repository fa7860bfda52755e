// LDS-resident solver for small 2D problems: the whole M1 x M2 grid of one
// problem lives in the LDS of one workgroup, which runs every fused pass of
// every iteration of a gradient-descent solve (section II-B.1, Eq. (2)) or a
// spectral initialisation (section II-B.2, Eq. (3)-(4)) with barriers between
// passes instead of kernel boundaries and without any global round trip of
// the grid; only the iterate, the phases and the measurements are read from
// global memory.  One launch runs the whole solve of many problems (one
// workgroup each).
//
// The passes follow the same schedule as the multi-kernel path: the 2D DFT
// splits into commuting axis transforms; layer l uses axis order (0,1) for
// odd l and (1,0) for even l, so pass k (1-based) runs along axis 0 for odd
// k and fuses [F_a D_k F_a]; the turnaround pass applies the residual or the
// spectral weight between F_a and F_a^H; the adjoint passes mirror the
// forward ones; the update pass [F_0^H D_1^* U^H, update] is fused with the
// next iteration's [U D_1 F_0].  Each axis transform is scaled by 1/sqrt(N)
// (unitary DFT).  The grid is stored row-major with rows padded as in the
// row-mode tiles; transforms exchange in place in their own grid lines.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "launch.hpp"
#include "loss.hpp"
#include "plan.hpp"

namespace sr {

namespace {

constexpr int kF2Threads = 512;
constexpr int kF2GridBytes = 150 * 1024;  // LDS budget of the grid

enum F2Op : int { F2_GD = 0, F2_SPEC = 1 };

struct F2Desc {
  int M1, M2, N1, N2, o1, o2, L;
  int ldr;           // padded row length of the LDS grid
  int pad2;          // pad shift of the row index (0: none)
  const float* th;   // L x M1 x M2 phases
  const float2* eph; // exp(i theta) tables, same layout (nullable: then sincos)
  const float* y;    // M1 x M2 measurements
  float2* x;         // GD: iterate (in place); spectral: output
  const float2* v0;  // spectral: start vector
  const float2* tw0; // thread-order twiddles of M1 (default shape)
  const float2* tw1; // ... of M2
  float step;        // GD: eta / m; spectral: 1 / (m c)
  float lam;         // spectral lambda
  float inv_m;
  int iters;
  int op;
  int loss;          // GD: LOSS_L2 or LOSS_POISSON
  float loss_eps;    // GD: Poisson guard
  unsigned* nf;      // set to 1 when the result holds NaN or Inf
};

template <int N>
using F2T = Tile<N, 1, false>;  // default shape: E, TPT, radices, twiddle slots

// In-place Stockham stages over one line per thread group; g[idx(k)] is the
// LDS slot of element k of this thread's line.  v: canonical registers.
// Every thread of the workgroup must call it (barriers); inactive threads
// compute on zeros and neither read nor write LDS.
template <int N, bool INV, int S, class Idx>
__device__ __forceinline__ void f2_stage(float2 (&v)[F2T<N>::E], const typename F2T<N>::Twiddles& w, int t,
                                         bool active, float2* g, const Idx& idx) {
  using T = F2T<N>;
  using RL = typename FftShape<N>::R;
  constexpr int E = T::E;
  constexpr int TPT = T::TPT;
  if constexpr (S < RL::count) {
    constexpr int R = RL::values[S];
    constexpr int P = RL::span(S);
    constexpr int Q = E / R;
    if constexpr (S > 0) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = active ? g[idx(t + j * TPT)] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      float2 u[R];
#pragma unroll
      for (int r = 0; r < R; ++r) u[r] = v[q + r * Q];
      const int i = t + q * TPT;
      const int k = i % P;
      if constexpr (S > 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float2 tf = w[T::tw_offset(S) + q * (R - 1) + (r - 1)];
          u[r] = INV ? cmulc(u[r], tf) : cmul(u[r], tf);
        }
      }
      Dft<R, INV>::run(u);
      if constexpr (S + 1 < RL::count) {
        if (q == 0) __syncthreads();  // every read of the line is done before it is overwritten
        const int base = (i / P) * P * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (active) g[idx(base + r * P)] = u[r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[q + r * Q] = u[r];
      }
    }
    f2_stage<N, INV, S + 1>(v, w, t, active, g, idx);
  }
}

// unitary transform: 1/sqrt(N) after the butterflies
template <int N, bool INV, class Idx>
__device__ __forceinline__ void f2_fft(float2 (&v)[F2T<N>::E], const typename F2T<N>::Twiddles& w, int t,
                                       bool active, float2* g, const Idx& idx) {
  f2_stage<N, INV, 0>(v, w, t, active, g, idx);
  const float s = rsqrtf((float)N);
#pragma unroll
  for (int j = 0; j < F2T<N>::E; ++j) v[j] = cscale(v[j], s);
}

// diagonal entry of D_l (1-based layer) at grid index gi
__device__ __forceinline__ float2 f2_phase(const F2Desc& d, int l, int gi, bool conj) {
  const long long o = (long long)(l - 1) * d.M1 * d.M2 + gi;
  float2 e;
  if (d.eph != nullptr) {
    e = d.eph[o];
  } else {
    float s, c;
    sincosf(d.th[o], &s, &c);
    e = make_float2(c, s);
  }
  return conj ? cconj(e) : e;
}

enum F2Pass : int {
  F2P_FIRST = 0,  // support columns: [U D_1 F_0] from the global iterate
  F2P_MID = 1,    // [F_a D_k F_a] (or its adjoint) in the grid
  F2P_TURN = 2,   // [F_a -> residual / spectral weight -> F_a^H] in the grid
  F2P_LAST = 3    // support columns: [F_0^H D_1^* U^H, update] (+ next [U D_1 F_0])
};

struct F2PassArgs {
  int k;           // layer of the mid diagonal (F2P_MID)
  bool adj;        // adjoint pass (F2P_MID)
  float in_scale;  // multiplies the grid on load (deferred spectral normalisation)
  float s_prev;    // spectral: 1/||u|| of the current iterate
  float ybar;      // spectral: mean(y)
  bool next;       // F2P_LAST: also run the next iteration's first pass
};

// One pass of length N along axis 0 (COL) or 1 over the LDS grid g; returns
// this thread's share of the pass's sum (GD loss or squared norm).  Not
// inlined: every (length, axis, kind) gets its own register allocation.
template <int N, bool COL, int KIND>
__device__ __noinline__ float f2_pass(const F2Desc* __restrict__ dp, float2* g, F2PassArgs pa) {
  const F2Desc& d = *dp;
  using T = F2T<N>;
  constexpr int E = T::E;
  constexpr int TPT = T::TPT;
  constexpr int B = kF2Threads / TPT > 0 ? kF2Threads / TPT : 1;  // lines per batch
  static_assert(TPT <= kF2Threads && kF2Threads % TPT == 0, "transform does not tile the workgroup");
  constexpr bool SUPPORT = (KIND == F2P_FIRST || KIND == F2P_LAST);
  const int tid = threadIdx.x;
  const int t = COL ? tid / B : tid % TPT;
  const int bl = COL ? tid % B : tid / TPT;
  typename T::Twiddles w;
  T::load_twiddles(w, COL ? d.tw0 : d.tw1, t);
  const int ldr = d.ldr, pad2 = d.pad2, M2 = d.M2;
  auto padc = [&](int c) { return pad2 ? c + (c >> pad2) : c; };
  float acc = 0.f;
  // lines: support columns for the first/last passes, else every row/column
  const int line_lo = SUPPORT ? d.o2 : 0;
  const int nlines = SUPPORT ? d.N2 : (COL ? d.M2 : d.M1);
  for (int b0 = 0; b0 < nlines; b0 += B) {
    __syncthreads();  // the previous pass (other axis) or batch has finished with the grid
    const int line = line_lo + b0 + bl;
    const bool active = (b0 + bl) < nlines;
    const int lbase = COL ? padc(line) : line * ldr;
    auto idx = [&](int k) -> int { return COL ? lbase + k * ldr : lbase + padc(k); };
    auto gidx = [&](int k) -> int { return COL ? k * M2 + line : line * M2 + k; };
    // operands read from global memory, issued before any transform
    float2 dg[E];  // diagonal entries of this pass (D_k, D_k^* or D_1)
    float yv[E];   // measurements (turnaround)
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = t + j * TPT;
      if constexpr (KIND == F2P_MID) dg[j] = active ? f2_phase(d, pa.k, gidx(k), pa.adj) : make_float2(0.f, 0.f);
      if constexpr (SUPPORT)
        dg[j] = (active && k >= d.o1 && k < d.o1 + d.N1) ? f2_phase(d, 1, gidx(k), false) : make_float2(0.f, 0.f);
      if constexpr (KIND == F2P_TURN) yv[j] = active ? d.y[gidx(k)] : 0.f;
    }
    float2 v[E];
    if constexpr (KIND == F2P_FIRST) {
      // U x: rows [o1, o1 + N1) of support column `line`, times D_1
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k = t + j * TPT;
        float2 u = make_float2(0.f, 0.f);
        if (active && k >= d.o1 && k < d.o1 + d.N1)
          u = cmul(cscale(d.x[(k - d.o1) * d.N2 + (line - d.o2)], pa.s_prev), dg[j]);
        v[j] = u;
      }
      f2_fft<N, false>(v, w, t, active, g, idx);
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) v[j] = active ? cscale(g[idx(t + j * TPT)], pa.in_scale) : make_float2(0.f, 0.f);
      if constexpr (KIND == F2P_MID) {
        if (pa.adj) f2_fft<N, true>(v, w, t, active, g, idx);
        else f2_fft<N, false>(v, w, t, active, g, idx);
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = cmul(v[j], dg[j]);
        if (pa.adj) f2_fft<N, true>(v, w, t, active, g, idx);
        else f2_fft<N, false>(v, w, t, active, g, idx);
      } else if constexpr (KIND == F2P_TURN) {
        f2_fft<N, false>(v, w, t, active, g, idx);
        if (d.op == F2_GD) {
          // residual weight of the plan's loss (no loss trace on this path)
          if (d.loss == LOSS_POISSON) {
#pragma unroll
            for (int j = 0; j < E; ++j) v[j] = cscale(v[j], poisson_weight(cabs2(v[j]), yv[j], d.loss_eps));
          } else {
#pragma unroll
            for (int j = 0; j < E; ++j) v[j] = cscale(v[j], cabs2(v[j]) - yv[j]);
          }
        } else {
#pragma unroll
          for (int j = 0; j < E; ++j) {
            float wgt = d.lam;
            if (yv[j] > 0.f) wgt = fmaxf(1.f - pa.ybar / yv[j], d.lam);
            v[j] = cscale(v[j], wgt);
          }
        }
        f2_fft<N, true>(v, w, t, active, g, idx);
      } else {  // F2P_LAST
        f2_fft<N, true>(v, w, t, active, g, idx);
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const int k = t + j * TPT;
          const bool in = active && k >= d.o1 && k < d.o1 + d.N1;
          float2 nv = make_float2(0.f, 0.f);
          if (in) {
            const float2 gk = cmulc(v[j], dg[j]);
            float2* xp = &d.x[(k - d.o1) * d.N2 + (line - d.o2)];
            const float2 xo = *xp;
            if (d.op == F2_GD) {
              nv = make_float2(xo.x - d.step * gk.x, xo.y - d.step * gk.y);
            } else {
              // u_new = step * A^H T A v - 2 lambda v, v = s_prev * u_old
              const float c = 2.f * d.lam * pa.s_prev;
              nv = make_float2(d.step * gk.x - c * xo.x, d.step * gk.y - c * xo.y);
              acc += cabs2(nv);
            }
            *xp = nv;
          }
          // next iteration's [U D_1 F_0] on the new iterate (spectral: unnormalised)
          v[j] = (pa.next && in) ? cmul(nv, dg[j]) : make_float2(0.f, 0.f);
        }
        if (pa.next) {
          __syncthreads();  // the adjoint transform's last reads of the line are done
          f2_fft<N, false>(v, w, t, active, g, idx);
        }
      }
    }
    if (KIND != F2P_LAST || pa.next) {
      __syncthreads();  // the transforms' last reads of the lines are done
#pragma unroll
      for (int j = 0; j < E; ++j)
        if (active) g[idx(t + j * TPT)] = v[j];
    }
  }
  return acc;
}

// Runtime length -> templated pass.
template <bool COL, int KIND>
__device__ __forceinline__ float f2_pass_len(int N, const F2Desc* dp, float2* g, const F2PassArgs& pa) {
  switch (N) {
    case 16: return f2_pass<16, COL, KIND>(dp, g, pa);
    case 32: return f2_pass<32, COL, KIND>(dp, g, pa);
    case 64: return f2_pass<64, COL, KIND>(dp, g, pa);
    case 96: return f2_pass<96, COL, KIND>(dp, g, pa);
    case 128: return f2_pass<128, COL, KIND>(dp, g, pa);
    case 192: return f2_pass<192, COL, KIND>(dp, g, pa);
    case 256: return f2_pass<256, COL, KIND>(dp, g, pa);
    default: return 0.f;
  }
}

// zero the grid outside the support columns
__device__ __forceinline__ void f2_clear_outside(const F2Desc& d, float2* g) {
  const int w = d.M2 - d.N2;
  for (int e = threadIdx.x; e < d.M1 * w; e += kF2Threads) {
    const int r = e / w, q = e % w;
    const int c = q < d.o2 ? q : q + d.N2;
    g[r * d.ldr + (d.pad2 ? c + (c >> d.pad2) : c)] = make_float2(0.f, 0.f);
  }
}

// A whole GD solve or spectral initialisation of one problem per workgroup.
__global__ void __launch_bounds__(kF2Threads) fused2d_kernel(const F2Desc* __restrict__ descs) {
  extern __shared__ float2 grid[];
  __shared__ double redd[kF2Threads / 64];
  const F2Desc* dp = descs + blockIdx.x;
  const F2Desc& d = *dp;
  const int L = d.L;
  F2PassArgs pa{};
  pa.in_scale = 1.f;
  pa.s_prev = 1.f;
  float scale_out = 1.f;
  if (d.op == F2_SPEC) {
    // x <- v0; s_prev = 1/||v0||; mean(y)
    double ys = 0.0, vs = 0.0;
    for (int e = threadIdx.x; e < d.M1 * d.M2; e += kF2Threads) ys += (double)d.y[e];
    for (int e = threadIdx.x; e < d.N1 * d.N2; e += kF2Threads) {
      const float2 v = d.v0[e];
      d.x[e] = v;
      vs += (double)v.x * v.x + (double)v.y * v.y;
    }
    const double ysum = block_sum_t<kF2Threads, double>(ys, redd);
    const double vsum = block_sum_t<kF2Threads, double>(vs, redd);
    pa.ybar = (float)(ysum * (double)d.inv_m);
    pa.s_prev = (float)(1.0 / sqrt(vsum));
    scale_out = (float)sqrt(ysum * (double)d.step);  // sqrt(sum(y) / (m c)), step = 1/(m c)
    __syncthreads();
  }
  f2_clear_outside(d, grid);
  f2_pass_len<true, F2P_FIRST>(d.M1, dp, grid, pa);
  for (int it = 0; it < d.iters; ++it) {
    const float s_cur = pa.s_prev;  // normalisation of the iterate that entered this iteration
    // forward middle passes k = 2..L, turnaround k = L + 1
    for (int k = 2; k <= L + 1; ++k) {
      pa.k = k;
      pa.adj = false;
      const bool col = (k % 2) == 1;
      const int N = col ? d.M1 : d.M2;
      if (k <= L) {
        if (col) f2_pass_len<true, F2P_MID>(N, dp, grid, pa);
        else f2_pass_len<false, F2P_MID>(N, dp, grid, pa);
      } else {
        if (col) f2_pass_len<true, F2P_TURN>(N, dp, grid, pa);
        else f2_pass_len<false, F2P_TURN>(N, dp, grid, pa);
      }
      pa.in_scale = 1.f;
    }
    // adjoint middle passes k = L..2
    for (int k = L; k >= 2; --k) {
      pa.k = k;
      pa.adj = true;
      if ((k % 2) == 1) f2_pass_len<true, F2P_MID>(d.M1, dp, grid, pa);
      else f2_pass_len<false, F2P_MID>(d.M2, dp, grid, pa);
    }
    // update (+ next first pass); the columns outside the support are cleared
    // for the next iteration (the update pass never reads them)
    pa.next = it + 1 < d.iters;
    pa.s_prev = s_cur;
    const float un = f2_pass_len<true, F2P_LAST>(d.M1, dp, grid, pa);
    if (pa.next) f2_clear_outside(d, grid);
    if (d.op == F2_SPEC) {
      // normalisation of the new iterate: its first-pass image is unnormalised,
      // the next pass scales the grid on load
      const double nsum = block_sum_t<kF2Threads, double>((double)un, redd);
      pa.s_prev = (float)(1.0 / sqrt(nsum));
      pa.in_scale = pa.s_prev;
    }
    __syncthreads();
  }
  // x0 = sqrt(sum(y) / (m c)) u / ||u|| (spectral); the result checked for NaN / Inf
  const float s = d.op == F2_SPEC ? scale_out * pa.s_prev : 1.f;
  bool bad = false;
  for (int e = threadIdx.x; e < d.N1 * d.N2; e += kF2Threads) {
    const float2 v = cscale(d.x[e], s);
    if (d.op == F2_SPEC) d.x[e] = v;
    bad |= !finite2(v);
  }
  flag_nonfinite(d.nf, bad);
}

// Grid layout of the LDS-resident path: both lengths in {16, ..., 256} and
// the padded grid within the LDS budget.
bool f2_layout(int M1, int M2, int* ldr, int* pad2) {
  auto ok_len = [](int n) { return n == 16 || n == 32 || n == 64 || n == 96 || n == 128 || n == 192 || n == 256; };
  if (!ok_len(M1) || !ok_len(M2)) return false;
  const bool r8 = M2 >= 32 && (M2 % 3) != 0;  // radix-8-first row lengths pad one slot every 8
  *pad2 = r8 ? 3 : 0;
  *ldr = r8 ? M2 + M2 / 8 : M2;
  return (size_t)M1 * (size_t)(*ldr) * sizeof(float2) <= (size_t)kF2GridBytes;
}

bool f2_shape_fits(int M1, int M2) {
  int a, b;
  return f2_layout(M1, M2, &a, &b);
}

size_t f2_grid_bytes(int M1, int M2) {
  int ldr, pad;
  return f2_layout(M1, M2, &ldr, &pad) ? (size_t)M1 * ldr * sizeof(float2) : 0;
}

}  // namespace

// For GD the LDS-resident solver is opt-in (SR_LDS_RESIDENT=1).  Measured
// against the level launches (300 GD steps): 512 problems on 64 x 64 grids,
// L = 2: 12.2 ms against 13.9 ms; 256 problems on 128 x 128 grids: 29.4
// against 26.4 ms (one workgroup per CU); 1024 problems on 64 x 32 grids,
// L = 1: 12.2 against 9.2 ms (too little work per workgroup).  Not a win
// often enough to be the default there.  For the power iteration it is the
// default (SR_LDS_RESIDENT=0 turns it off): on 256 uneven problems, 100
// iterations, the small ones here beside the level launches of the others
// take 26.6 ms against 28.1 ms with every problem on the levels.
bool fused2d_enabled(bool by_default) {
  const char* e = std::getenv("SR_LDS_RESIDENT");
  if (e == nullptr || *e == '\0') return by_default;
  return std::atoi(e) != 0;
}

bool fused2d_supported(const Geo& g) {
  return g.ndim == 2 && g.L >= 1 && !g.cropped() && f2_shape_fits(g.M1, g.M2);
}

static sr_status f2_launch(sr_plan_s* p, const std::vector<F2Desc>& descs, size_t lds, hipStream_t s) {
  if (descs.empty()) return SR_OK;
  const size_t bytes = descs.size() * sizeof(F2Desc);
  if (p->f2_desc_cap < descs.size()) {
    if (p->f2_descs) {
      // launches already queued (on either of the plan's streams) may still read the old ones
      if (hipError_t w = hipStreamSynchronize(p->stream); w != hipSuccess) return hip_fail(w, "stream wait");
      if (p->aux_stream != nullptr)
        if (hipError_t w = hipStreamSynchronize(p->aux_stream); w != hipSuccess) return hip_fail(w, "stream wait");
      (void)hipFree(p->f2_descs);
    }
    p->f2_descs = nullptr;
    hipError_t e = hipMalloc(&p->f2_descs, bytes);
    if (e != hipSuccess) return fail(SR_E_NOMEM, "descriptor allocation failed");
    p->f2_desc_cap = descs.size();
  }
  // the plan keeps the host copy alive while the upload is in flight
  std::vector<unsigned char>& host = p->f2_host;
  host.resize(bytes);
  std::memcpy(host.data(), descs.data(), bytes);
  hipError_t e = hipMemcpyAsync(p->f2_descs, host.data(), bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "descriptor upload");
  static bool raised = false;
  if (!raised) {
    e = hipFuncSetAttribute((const void*)fused2d_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, kF2GridBytes);
    if (e != hipSuccess) return hip_fail(e, "LDS attribute");
    raised = true;
  }
  hipLaunchKernelGGL(fused2d_kernel, dim3((unsigned)descs.size()), dim3(kF2Threads), lds, s,
                     (const F2Desc*)p->f2_descs);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "LDS-resident solver launch");
  return SR_OK;
}

static F2Desc f2_desc(const sr_plan_s* p, size_t i, int op, const float* y, float2* x, int iters) {
  const Geo& g = p->geo[i];
  F2Desc d{};
  f2_layout(g.M1, g.M2, &d.ldr, &d.pad2);
  d.M1 = g.M1;
  d.M2 = g.M2;
  d.N1 = g.N1;
  d.N2 = g.N2;
  d.o1 = g.o1;
  d.o2 = g.o2;
  d.L = g.L;
  d.th = p->theta + g.th_off;
  d.eph = p->use_table ? p->eph + g.th_off : nullptr;
  d.y = y + p->yoff[i];
  d.x = x + p->xoff[i];
  d.tw0 = p->twiddles(g.M1, 0);
  d.tw1 = p->twiddles(g.M2, 0);
  d.inv_m = 1.f / (float)g.m;  // (not cropped: m is the grid size)
  d.iters = iters;
  d.op = op;
  d.loss = p->loss;
  d.loss_eps = p->loss_eps;
  d.nf = p->sync + 2;
  return d;
}

// GD on the listed problems (indices into the plan), whole solve in one launch.
sr_status fused2d_gd(sr_plan_s* p, const std::vector<int>& which, const float* y, float2* x, int iters,
                     const float* eta, hipStream_t s) {
  std::vector<F2Desc> descs;
  size_t lds = 0;
  for (int i : which) {
    F2Desc d = f2_desc(p, i, F2_GD, y, x, iters);
    d.step = eta[i] / (float)p->geo[i].m;
    lds = std::max(lds, f2_grid_bytes(d.M1, d.M2));
    descs.push_back(d);
  }
  return f2_launch(p, descs, lds, s);
}

// Spectral initialisation of the listed problems (c = 1/m).
sr_status fused2d_spectral(sr_plan_s* p, const std::vector<int>& which, const float* y, const float2* v0, int iters,
                           float lam, float2* x0, hipStream_t s) {
  std::vector<F2Desc> descs;
  size_t lds = 0;
  for (int i : which) {
    F2Desc d = f2_desc(p, i, F2_SPEC, y, x0, iters);
    d.v0 = v0 + p->xoff[i];
    d.step = 1.f;  // 1 / (m c) with c = 1/m
    d.lam = lam;
    lds = std::max(lds, f2_grid_bytes(d.M1, d.M2));
    descs.push_back(d);
  }
  return f2_launch(p, descs, lds, s);
}

}  // namespace sr
