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
#include "loss.hpp"

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
  MID_PHASE_GT = 9,         // gth += Im(conj(v) save), v <- D v     (adjoint VJP)
  MID_GD_POIS = 10          // v <- (1 - y/(|v|^2 + eps)) v, Poisson loss partials
};
// The reverse-mode mid operations (phase diagonal with a saved intermediate).
constexpr bool mid_rev_phase(int mid) { return mid >= MID_PHASE_SAVE && mid <= MID_PHASE_GT; }

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
  const float2* tw;   // thread-order twiddle table of the default thread shape
  const float2* tw_n; // ... of the length's narrow or wide thread shape (where it has one)
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
  const float* y;        // measurements on the window (MID_GD, MID_GD_POIS, MID_SPEC)
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
  // measurement window: grid rows [win_lo0, win_hi0) x columns [win_lo1,
  // win_hi1), stored row-major with row length win_ld.  y, z_out, y_out (and
  // the input of the adjoint's first pass) live on the window; the residual
  // and the spectral weight are zero outside it.
  int win_lo0, win_hi0, win_lo1, win_hi1;
  long long win_ld;
  int crop;  // nonzero when the window is smaller than the grid (host: picks the window-aware kernels)
  float loss_eps;  // Poisson loss guard (MID_GD_POIS)
  // stacked problems: one launch runs this pass for `stack` problems of one
  // geometry; ntr counts the transforms of all of them, ntr_p those of one,
  // and problem s's data sits s * s_<buffer> elements after problem 0's
  int stack, ntr_p;
  int s_in, s_out, s_out2, s_win, s_th, s_save, s_gth, s_xin;
  const float* step_v;  // GD update of a stack: each problem's step (nullable: `step` for all)
  // non-finite flag (nullable): the final update of a solve (POST_GD,
  // POST_SPEC) stores 1 here when an updated iterate entry is NaN or Inf
  unsigned* nf;
};

// 1/sqrt of the sum of the previous iterate's squared-norm partials: strided
// per-thread sums, then a fixed-order workgroup reduction in float64, so
// every thread (and every workgroup of the pass) gets the same value.
template <int NTHREADS>
__device__ __forceinline__ float inv_norm_from_partials(const float* part, int n) {
  __shared__ double redd[NTHREADS / 64 > 0 ? NTHREADS / 64 : 1];
  double acc = 0.0;
  for (int i = (int)threadIdx.x; i < n; i += NTHREADS) acc += (double)part[i];
  return (float)(1.0 / sqrt(block_sum_t<NTHREADS, double>(acc, redd)));
}

// One tile (B transforms) of a fused pass.  `lds` holds 2*B*N complex
// elements, `red` one float per thread.  part_in/npart/part_out override the
// partial-sum pointers of `a` (persistent kernels alternate them per
// iteration); partial sums are written at index `tile`.  TAB selects the
// phase source: exp(i theta) tables (ep_*) or the phases themselves (th_*,
// evaluated with sincos).
//
// Every global load the tile needs (input, phases, measurements, twiddles,
// the previous iterate) is issued up front, so a pass costs one memory
// round trip plus its arithmetic, not one round trip per stage.  Loads and
// stores go through buffer resources: lanes outside a window (the zero-padded
// rows/columns, transforms past ntr) read zeros and drop their writes.
template <int N, int B, bool COL, int PRE, int MID, bool FFT2, bool INV1, bool INV2, int POST, bool DB = true,
          int EV = 0, bool TAB = false, bool WIN = false>
__device__ __forceinline__ void pass_tile(const PassArgs& a, int tile, float2* lds, float* red, const float* part_in,
                                          int npart, float* part_out) {
  using T = TileV<N, B, COL, DB, EV>;
  constexpr int E = T::E;
  constexpr bool MID_PH = (MID == MID_PHASE || MID == MID_PHASE_CONJ || mid_rev_phase(MID));
  constexpr bool MID_SAVED = (MID == MID_PHASE_CONJ_GT || MID == MID_PHASE_GT);
  constexpr bool MID_Y = (MID == MID_GD || MID == MID_GD_POIS || MID == MID_SPEC);
  constexpr bool POST_PH = (POST != POST_STORE);
  constexpr bool POST_X = (POST == POST_GD || POST == POST_SPEC || POST == POST_GD_FWD || POST == POST_SPEC_FWD);
  constexpr bool POST_FWD = (POST == POST_GD_FWD || POST == POST_SPEC_FWD);
  constexpr bool POST_IS_GD = (POST == POST_GD || POST == POST_GD_FWD);
  constexpr bool POST_IS_SPEC = (POST == POST_SPEC || POST == POST_SPEC_FWD);
  int t = T::thread_t();
  const int bl = T::thread_b();
  const int tb = tile * B + bl;  // transform index (over every problem of a stack)
  const bool active = tb < a.ntr;
  int b = tb, sp = 0;            // this lane's transform within its problem, and the problem
  if (a.stack > 1) {
    sp = tb / a.ntr_p;
    b = tb - sp * a.ntr_p;
  }
  int gb = a.tr_lo + b;  // grid coordinate of this transform
  const int gld = (int)a.grid_ld, ild = (int)a.in_ld, old = (int)a.out_ld;
  // the lane's problem's offset in each buffer (zero without a stack)
  const int o_in = sp * a.s_in, o_out = sp * a.s_out, o_out2 = sp * a.s_out2, o_win = sp * a.s_win;
  const int o_th = sp * a.s_th, o_sv = sp * a.s_save, o_gt = sp * a.s_gth, o_xin = sp * a.s_xin;

  // element offsets: grid position, input and output buffer positions
  auto gidx = [&](int k) -> int { return COL ? k * gld + gb : gb * gld + k; };
  auto in_addr = [&](int k) -> int { return o_in + (COL ? (k - a.in_lo) * ild + b : b * ild + (k - a.in_lo)); };
  auto out_rel = [&](int k) -> int { return COL ? (k - a.out_lo) * old + b : b * old + (k - a.out_lo); };
  auto out_addr = [&](int k) -> int { return o_out + out_rel(k); };
  auto in_win = [&](int k) { return active && k >= a.in_lo && k < a.in_hi; };
  auto out_win = [&](int k) { return active && k >= a.out_lo && k < a.out_hi; };
  // measurement window: membership and index of grid element k of this
  // transform (the transform's own coordinate is tested once; the index is
  // affine in k).  Kernels built without WIN take the window to be the whole
  // grid (no trimming), where membership is `active` and the index is gidx.
  const int wld = (int)a.win_ld;
  const bool m_lane =
      WIN ? active && (COL ? (gb >= a.win_lo1 && gb < a.win_hi1) : (gb >= a.win_lo0 && gb < a.win_hi0)) : active;
  const int m_klo = COL ? a.win_lo0 : a.win_lo1;
  const int m_khi = COL ? a.win_hi0 : a.win_hi1;
  const int m_base = COL ? (gb - a.win_lo1) - a.win_lo0 * wld : (gb - a.win_lo0) * wld - a.win_lo1;
  auto m_in = [&](int k) { return WIN ? m_lane && k >= m_klo && k < m_khi : active; };
  auto m_idx = [&](int k) -> int { return o_win + (WIN ? (COL ? m_base + k * wld : m_base + k) : gidx(k)); };
  // the adjoint's first pass ([F_a^H] alone) reads its input on the window
  constexpr bool IN_WIN = WIN && (PRE == PRE_NONE && MID == MID_NONE && !FFT2 && INV1 && POST == POST_STORE);

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
  T::load_twiddles(w, EV ? a.tw_n : a.tw, t);
  const Rsrc r_in = rsrc(a.in);
  const Rsrc r_out = rsrc(a.out);
  const Rsrc r_pre = TAB ? rsrc(a.ep_pre) : rsrc(a.th_pre);
  const Rsrc r_mid = TAB ? rsrc(a.ep_mid) : rsrc(a.th_mid);
  const Rsrc r_post = TAB ? rsrc(a.ep_post) : rsrc(a.th_post);
  const Rsrc r_y = rsrc(a.y);
  const Rsrc r_save = rsrc(a.save);
  const Rsrc r_gth = rsrc(a.gth);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int k = T::elem(t, j);
    const bool iw = in_win(k);
    const int g = gidx(k) + o_th;  // phase index
    if constexpr (IN_WIN) v[j] = ld2(r_in, off8(m_in(k), m_idx(k) - o_win + o_in));
    else v[j] = ld2(r_in, off8(iw, in_addr(k)));
    if constexpr (PRE == PRE_PHASE) {
      if constexpr (TAB) dp[j] = ld2(r_pre, off8(iw, g));
      else dp[j].x = ld1(r_pre, off4(iw, g));
    }
    if constexpr (MID_PH) {
      if constexpr (TAB) dm[j] = ld2(r_mid, off8(active, g));
      else dm[j].x = ld1(r_mid, off4(active, g));
    }
    if constexpr (MID_Y) yv[j] = ld1(r_y, off4(m_in(k), m_idx(k)));
    if constexpr (MID_SAVED) {
      sv[j] = ld2(r_save, off8(active, g - o_th + o_sv));
      gt[j] = ld1(r_gth, off4(active, g - o_th + o_gt));
    }
    if constexpr (MID != MID_STORE) {
      const bool ow = out_win(k);
      if constexpr (POST_PH) {
        if constexpr (TAB) dq[j] = ld2(r_post, off8(ow, g));
        else dq[j].x = ld1(r_post, off4(ow, g));
      }
      if constexpr (POST_X) xo[j] = ld2(r_out, off8(ow, out_addr(k)));
      if constexpr (POST == POST_PHASE_CONJ_GT) {
        xo[j] = ld2(rsrc(a.xin), off8(ow, o_xin + out_rel(k)));
        gt[j] = ld1(r_gth, off4(ow, g - o_th + o_gt));
      }
    }
  }
  // phases -> diagonal entries where no table was given (the sixteen-
  // element shape forms the mid and post entries where they are used, so
  // that only the phases stay live across the first transform)
  constexpr bool LATE_PH = !TAB && E >= 16;
  if constexpr (!TAB) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      if constexpr (PRE == PRE_PHASE) dp[j] = phase_turns(dp[j].x);
      if constexpr (MID_PH && !LATE_PH) dm[j] = phase_turns(dm[j].x);
      if constexpr (POST_PH && !LATE_PH) dq[j] = phase_turns(dq[j].x);
    }
  }
  auto Dm = [&](int j) -> float2 {
    if constexpr (LATE_PH) return phase_turns(dm[j].x);
    else return dm[j];
  };
  auto Dq = [&](int j) -> float2 {
    if constexpr (LATE_PH) return phase_turns(dq[j].x);
    else return dq[j];
  };

  float s_pre = a.scale_pre;
  float s_prev = 1.f;  // 1/||u_prev|| for the spectral update
  if constexpr (PRE == PRE_PHASE || POST_IS_SPEC) {  // the only shapes that take the previous norm
    if (part_in != nullptr) {
      // a stack keeps each problem's partials together (npart apiece), and
      // a pass that reads them has whole problems in each tile
      const float* pin = a.stack > 1 ? part_in + (tile * B / a.ntr_p) * npart : part_in;
      s_prev = inv_norm_from_partials<T::THREADS>(pin, npart);
      if (PRE == PRE_PHASE) s_pre *= s_prev;
    }
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
      const float2 d = cscale(Dm(j), a.scale_mid);
      v[j] = (MID == MID_PHASE_CONJ) ? cmulc(v[j], d) : cmul(v[j], d);
    }
  } else if constexpr (mid_rev_phase(MID)) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      const unsigned go8 = off8(active, gidx(k) + o_sv), go4 = off4(active, gidx(k) + o_gt);
      const float2 u = cscale(v[j], a.scale_mid);
      if constexpr (MID == MID_PHASE_SAVE) {
        v[j] = cmul(u, Dm(j));
        st2(r_save, go8, v[j]);
      } else if constexpr (MID == MID_PHASE_CONJ_SAVE) {
        v[j] = cmulc(u, Dm(j));
        st2(r_save, go8, v[j]);
      } else if constexpr (MID == MID_PHASE_CONJ_GT) {
        // Im(u conj(s)) = u.y s.x - u.x s.y
        st1(r_gth, go4, gt[j] + (u.y * sv[j].x - u.x * sv[j].y));
        v[j] = cmulc(u, Dm(j));
      } else {  // MID_PHASE_GT: Im(conj(u) s) = u.x s.y - u.y s.x
        st1(r_gth, go4, gt[j] + (u.x * sv[j].y - u.y * sv[j].x));
        v[j] = cmul(u, Dm(j));
      }
    }
  } else if constexpr (MID == MID_GD) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const bool in = m_in(T::elem(t, j));
      float2 z = cscale(v[j], a.scale_mid);
      float d = in ? cabs2(z) - yv[j] : 0.f;  // zero residual outside the measurement window
      acc += d * d;
      v[j] = cscale(z, d);
    }
  } else if constexpr (MID == MID_GD_POIS) {
    float z2[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const bool in = m_in(T::elem(t, j));
      float2 z = cscale(v[j], a.scale_mid);
      z2[j] = cabs2(z);
      v[j] = cscale(z, in ? poisson_weight(z2[j], yv[j], a.loss_eps) : 0.f);
    }
    if (part_out != nullptr) {  // the logarithms only for a loss trace
#pragma unroll
      for (int j = 0; j < E; ++j)
        acc += m_in(T::elem(t, j)) ? poisson_term(z2[j], yv[j], a.loss_eps) : 0.f;
    }
  } else if constexpr (MID == MID_SPEC) {
    const float ybar = (float)(a.ysum[active ? sp : 0] * (double)a.inv_m);  // the problem's sum(y) (a stack: one each)
#pragma unroll
    for (int j = 0; j < E; ++j) {
      float2 z = cscale(v[j], a.scale_mid);
      float wgt = a.lam;
      if (yv[j] > 0.f) wgt = fmaxf(1.f - ybar / yv[j], a.lam);
      v[j] = cscale(z, m_in(T::elem(t, j)) ? wgt : 0.f);
    }
  } else if constexpr (MID == MID_STORE) {
    const Rsrc r_z = rsrc(a.z_out), r_yo = rsrc(a.y_out);
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      float2 z = cscale(v[j], a.scale_mid);
      if (a.z_out) st2(r_z, off8(m_in(k), m_idx(k)), z);
      if (a.y_out) st1(r_yo, off4(m_in(k), m_idx(k)), cabs2(z));
    }
  }

  // ---- second transform, post-diagonal, update, store
  if constexpr (FFT2) T::template fft<INV2>(v, lds, ph, w, t, bl);
  if constexpr (E >= 16) {
    // the sixteen-element shape recomputes its store addresses here rather
    // than keeping the load phase's ones live (in scratch) across the
    // transforms: the lane coordinates are marked as changed (no code)
    asm volatile("" : "+v"(t), "+v"(b), "+v"(gb));
  }

  if constexpr (MID != MID_STORE) {
    constexpr bool CHECK = (POST == POST_GD || POST == POST_SPEC);  // the last update of a solve
    bool bad = false;
    float step = a.step;
    if constexpr (POST_IS_GD) {
      if (a.step_v != nullptr && active) step = a.step_v[sp];
    }
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      const bool ow = out_win(k);
      float2 val = cscale(v[j], a.scale_out);
      float2 qj = make_float2(1.f, 0.f);
      if constexpr (POST_PH) qj = Dq(j);
      if constexpr (POST == POST_PHASE_CONJ_GT) {
        const float2 u1 = cmul(xo[j], qj);  // u_1 = D_1 U x at this position
        st1(r_gth, off4(ow, gidx(k) + o_gt), gt[j] + (val.y * u1.x - val.x * u1.y));
      }
      if constexpr (POST_PH) val = cmulc(val, qj);
      if constexpr (POST_IS_GD) {
        val = make_float2(xo[j].x - step * val.x, xo[j].y - step * val.y);
      } else if constexpr (POST_IS_SPEC) {
        val = make_float2(s_prev * (a.step * val.x - a.two_lam * xo[j].x),
                          s_prev * (a.step * val.y - a.two_lam * xo[j].y));
        acc += ow ? cabs2(val) : 0.f;
      }
      st2(r_out, off8(ow, out_addr(k)), val);
      if constexpr (CHECK) bad |= ow && !finite2(val);
      if constexpr (POST_FWD) v[j] = ow ? cmul(val, qj) : make_float2(0.f, 0.f);  // zero outside the support
    }
    if constexpr (CHECK) flag_nonfinite(a.nf, bad);
  }

  if constexpr (POST_FWD) {
    T::template fft<false>(v, lds, ph, w, t, bl);
    const float s1 = a.scale_out;  // 1/sqrt(M1) for both transforms of this column pass
    const Rsrc r_o2 = rsrc(a.out2);
    const int o2ld = (int)a.out2_ld;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int k = T::elem(t, j);
      st2(r_o2, off8(active, o_out2 + k * o2ld + b), cscale(v[j], s1));
    }
  }

  if constexpr (MID == MID_GD || MID == MID_GD_POIS || POST_IS_SPEC) {
    if (part_out != nullptr) {
      float sum = block_sum<T::THREADS>(acc, red);
      if (threadIdx.x == 0) part_out[tile] = sum;
    }
  }
}

// Whether a pass shape reads any phase diagonal.
template <int PRE, int MID, int POST>
constexpr bool pass_has_phase() {
  return PRE == PRE_PHASE || MID == MID_PHASE || MID == MID_PHASE_CONJ || mid_rev_phase(MID) || POST != POST_STORE;
}

// pass_tile with the phase source picked at run time (the tables are set
// for every diagonal of a pass or for none), window-aware so that it serves
// every geometry.
template <int N, int B, bool COL, int PRE, int MID, bool FFT2, bool INV1, bool INV2, int POST, int EV = 0>
__device__ __forceinline__ void pass_tile_rt(const PassArgs& a, int tile, float2* lds, float* red, const float* part_in,
                                             int npart, float* part_out) {
  if constexpr (pass_has_phase<PRE, MID, POST>()) {
    if (a.ep_pre != nullptr || a.ep_mid != nullptr || a.ep_post != nullptr) {
      pass_tile<N, B, COL, PRE, MID, FFT2, INV1, INV2, POST, true, EV, true, true>(a, tile, lds, red, part_in, npart,
                                                                                  part_out);
      return;
    }
  }
  pass_tile<N, B, COL, PRE, MID, FFT2, INV1, INV2, POST, true, EV, false, true>(a, tile, lds, red, part_in, npart,
                                                                               part_out);
}

template <int N, int B, bool COL, int PRE, int MID, bool FFT2, bool INV1, bool INV2, int POST, bool DB = true,
          int EV = 0, bool TAB = false, bool WIN = false>
__global__ void __launch_bounds__((TileV<N, B, COL, DB, EV>::THREADS)) pass_kernel(const PassArgs a) {
  extern __shared__ float2 lds[];
  __shared__ float red[TileV<N, B, COL, DB, EV>::THREADS];
  pass_tile<N, B, COL, PRE, MID, FFT2, INV1, INV2, POST, DB, EV, TAB, WIN>(a, xcd_tile(blockIdx.x, gridDim.x), lds,
                                                                            red, a.part_in, a.npart, a.part_out);
}

}  // namespace sr
