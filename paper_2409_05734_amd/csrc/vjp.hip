// Reverse-mode derivatives of the structured operator with respect to the
// signal and to the phases theta_l of the diagonals D_l (section III, Eq. (5)),
// in PyTorch's complex-gradient convention (dL/dRe + i dL/dIm).
//
// For z = A x with u_l = D_l w_{l-1}, w_l = F u_l (w_0 = U x):
//   ubar_l = F^H wbar_l,  thetabar_l += Im(ubar_l conj(u_l)),
//   wbar_{l-1} = D_l^* ubar_l,  xbar = U^H wbar_0 = A^H zbar.
// For v = A^H r with t_l = F^H s_l, q_l = D_l^* t_l (s_L = r, s_{l-1} = q_l):
//   qbar_1 = U vbar,  thetabar_l += Im(conj(qbar_l) q_l),
//   qbar_{l+1} = F D_l qbar_l,  rbar = A vbar.
// The intermediates u_l / q_l are recomputed inside the call (one grid buffer
// per layer for the current problem) rather than kept from an earlier call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "fft_core.hpp"
#include "fused1d.hpp"
#include "schedule.hpp"

namespace sr {

namespace {

// gth_1[support] += Im(conj(gv) v) for the adjoint derivative's first layer,
// for P stacked problems (problem s: gv, v at s n, gth at s gth_stride)
__global__ void gth_support_kernel(const float2* __restrict__ gv, const float2* __restrict__ v, float* gth, int N1,
                                   int N2, int o1, int o2, long long M2, int P, long long gth_stride) {
  const long long n = (long long)N1 * N2;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n * P; e += (long long)gridDim.x * blockDim.x) {
    const long long s = e / n, l = e - s * n;
    const int i = (int)(l / N2), j = (int)(l % N2);
    const float2 a = gv[e], b = v[e];
    gth[s * gth_stride + (long long)(o1 + i) * M2 + (o2 + j)] += a.x * b.y - a.y * b.x;
  }
}

// gth[e] += sum over the stack of part[s * len + e], added in problem order
// (the order of a problem-by-problem loop)
__global__ void gth_reduce_kernel(const float* __restrict__ part, float* gth, long long len, int P) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < len; e += (long long)gridDim.x * blockDim.x) {
    float acc = gth[e];
    for (int s = 0; s < P; ++s) acc += part[(long long)s * len + e];
    gth[e] = acc;
  }
}

sr_status ensure_vjp_buf(sr_plan_s* p, int P = 1) {
  size_t need = 0;
  for (const Geo& g : p->geo)
    if (g.ndim == 2) need = std::max(need, (size_t)P * ((size_t)std::max(g.L - 1, 1) * (size_t)g.mg + (size_t)g.n));
  if (need <= p->vjp_elems) return SR_OK;
  if (p->vjp_buf) {
    // queued work may still use the old buffer
    if (hipError_t w = hipStreamSynchronize(p->stream); w != hipSuccess) return hip_fail(w, "stream wait");
    (void)hipFree(p->vjp_buf);
    p->vjp_buf = nullptr;
    p->vjp_elems = 0;
  }
  hipError_t e = hipMalloc(&p->vjp_buf, need * sizeof(float2));
  if (e != hipSuccess) return fail(SR_E_NOMEM, "derivative workspace allocation failed");
  p->vjp_elems = need;
  return SR_OK;
}

// save buffer of layer k (k = 2..L) and an n-sized scratch after them (for
// a stack: P grids per layer, then P signals)
float2* save_of(sr_plan_s* p, const Geo& g, int k) { return p->vjp_buf + (size_t)(k - 2) * p->stk.P * g.mg; }
float2* nscratch(sr_plan_s* p, const Geo& g) {
  return p->vjp_buf + (size_t)std::max(g.L - 1, 1) * p->stk.P * g.mg;
}

// phase cotangents of layer l: the caller's array, or, for a stack sharing
// its phases, problem 0's block of the per-problem scratch
float* gth_of(const sr_plan_s* p, const Geo& g, float* gtheta, int l) {
  if (p->stk.P > 1 && p->stk.th_stride == 0) return p->stk_gth + (int64_t)(l - 1) * g.mg;
  return gtheta + g.th_off + (int64_t)(l - 1) * g.mg;
}

sr_status fused1d_vjp(sr_plan_s* p, const Geo& g, int op, Fused1DArgs a) {
  a.n = g.N1;
  a.m = g.M1;
  a.L = g.L;
  a.off = g.o1;
  a.mw = g.W1;
  a.moff = g.c1;
  a.theta = p->theta_l(g, 1);
  a.tw = p->twiddles(g.M1, 1) ? p->twiddles(g.M1, 1) : p->twiddles(g.M1, 0);  // the 1D kernels' shape
  hipError_t e = launch_fused1d(g.M1, op, a, p->stream);
  if (e != hipSuccess) return hip_fail(e, "fused 1D derivative launch");
  return SR_OK;
}

#define VJ_CHECK(st)            \
  do {                          \
    sr_status s_ = (st);        \
    if (s_ != SR_OK) return s_; \
  } while (0)

// Forward passes 1..L on x (saving u_k, k >= 2), or with phase cotangents
// accumulated (kind_mid = PK_MID_FWD_GT).  Returns the result buffer.
sr_status fwd_passes(sr_plan_s* p, const Geo& g, const float2* x, int kind_mid, float* gtheta, float2** cur_out) {
  float2* bufs[2] = {p->bufA, p->bufB};
  int which = 0;
  {
    PassArgs a = base_args(p, g, 1);
    a.in = x;
    a.in_ld = g.N2;
    a.in_lo = g.o1;
    a.in_hi = g.o1 + g.N1;
    a.ntr = g.N2;
    a.tr_lo = g.o2;
    a.th_pre = p->theta_l(g, 1);
    a.out = bufs[which];
    a.out_ld = g.N2;
    a.out_lo = 0;
    a.out_hi = g.M1;
    a.scale_out = 1.f / std::sqrt((float)g.M1);
    VJ_CHECK(launch(p, g, 1, PK_FIRST_FWD, a));
  }
  for (int k = 2; k <= g.L; ++k) {
    PassArgs a = base_args(p, g, k);
    set_in(a, g, k, bufs[which]);
    out_full(a, g, k, bufs[which ^ 1]);
    a.th_mid = p->theta_l(g, k);
    const float s = 1.f / std::sqrt((float)pass_len(g, k));
    a.scale_mid = s;
    a.scale_out = s;
    a.save = save_of(p, g, k);
    if (kind_mid == PK_MID_FWD_GT) a.gth = gth_of(p, g, gtheta, k);
    VJ_CHECK(launch(p, g, k, kind_mid, a));
    which ^= 1;
  }
  *cur_out = bufs[which];
  return SR_OK;
}

// Adjoint passes from r (full grid): first [F^H], then mids of kind kind_mid
// (save q_k or accumulate phase cotangents), then the last pass of kind
// kind_last into x_out.
sr_status adj_passes(sr_plan_s* p, const Geo& g, const float2* r, int kind_mid, int kind_last, float* gtheta,
                     const float2* xin, float2* x_out) {
  const int kt = g.L + 1;
  float2* cur = p->bufA;
  float2* other = p->bufB;
  {
    PassArgs a = base_args(p, g, kt);
    in_full(a, g, kt, r);
      set_out(a, g, kt, cur);
    a.scale_out = 1.f / std::sqrt((float)pass_len(g, kt));
    VJ_CHECK(launch(p, g, kt, PK_FIRST_ADJ, a));
  }
  for (int k = g.L; k >= 2; --k) {
    PassArgs a = base_args(p, g, k);
    in_full(a, g, k, cur);
    set_out(a, g, k, other);
    a.th_mid = p->theta_l(g, k);
    const float s = 1.f / std::sqrt((float)pass_len(g, k));
    a.scale_mid = s;
    a.scale_out = s;
    a.save = save_of(p, g, k);
    if (kind_mid == PK_MID_ADJ_GT) a.gth = gth_of(p, g, gtheta, k);
    VJ_CHECK(launch(p, g, k, kind_mid, a));
    std::swap(cur, other);
  }
  PassArgs a = base_args(p, g, 1);
  a.in = cur;
  a.in_ld = g.N2;
  a.in_lo = 0;
  a.in_hi = g.M1;
  a.ntr = g.N2;
  a.tr_lo = g.o2;
  a.out = x_out;
  a.out_ld = g.N2;
  a.out_lo = g.o1;
  a.out_hi = g.o1 + g.N1;
  a.th_post = p->theta_l(g, 1);
  a.scale_out = 1.f / std::sqrt((float)g.M1);
  if (kind_last == PK_LAST_ADJ_GT) {
    a.gth = gth_of(p, g, gtheta, 1);
    a.xin = xin;
  }
  return launch(p, g, 1, kind_last, a);
}

}  // namespace

namespace {

// Stack set-up shared by both derivatives: buffers, the registered
// per-problem strides of the intermediates and of the phase cotangents, and
// the zeroed per-problem scratch when the stack shares its phases.
sr_status stack_vjp_setup(sr_plan_s* p, int P, float* gtheta) {
  const Geo& g = p->geo[0];
  for (int k = 2; k <= g.L; ++k) p->stk.add(save_of(p, g, k), g.mg, sizeof(float2), (int)g.mg);
  p->stk.add(nscratch(p, g), g.n, sizeof(float2), (int)g.n);
  const size_t block = (size_t)g.L * g.mg;
  if (p->stk.th_stride == 0) {
    const size_t need = (size_t)P * block;
    if (need > p->stk_gth_elems) {
      if (p->stk_gth) {
        // queued work may still use the old scratch
        if (hipError_t w = hipStreamSynchronize(p->stream); w != hipSuccess) return hip_fail(w, "stream wait");
        (void)hipFree(p->stk_gth);
        p->stk_gth = nullptr;
        p->stk_gth_elems = 0;
      }
      if (hipMalloc(&p->stk_gth, need * sizeof(float)) != hipSuccess)
        return fail(SR_E_NOMEM, "stacked derivative workspace allocation failed");
      p->stk_gth_elems = need;
    }
    hipError_t e = hipMemsetAsync(p->stk_gth, 0, need * sizeof(float), p->stream);
    if (e != hipSuccess) return hip_fail(e, "stacked derivative workspace clear");
    p->stk.add(p->stk_gth, block, sizeof(float), (int)block);
  } else {
    p->stk.add(gtheta + g.th_off, block, sizeof(float), p->stk.th_stride);
  }
  return SR_OK;
}

// a stack sharing its phases: add the per-problem cotangents in problem order
sr_status stack_vjp_finish(sr_plan_s* p, int P, float* gtheta) {
  if (p->stk.th_stride != 0) return SR_OK;
  const Geo& g = p->geo[0];
  const long long len = (long long)g.L * g.mg;
  const int groups = (int)std::min<long long>((len + 255) / 256, 2048);
  hipLaunchKernelGGL(gth_reduce_kernel, dim3(groups), dim3(256), 0, p->stream, p->stk_gth, gtheta + g.th_off, len, P);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SR_OK : hip_fail(e, "gth_reduce");
}

sr_status vjp_forward_stacked(sr_plan_s* p, int P, int ths, const float2* x, const float2* gz, float2* gx,
                              float* gtheta) {
  const Geo& g = p->geo[0];
  VJ_CHECK(ensure_stack_bufs(p, 2 * (size_t)P * g.mg));
  VJ_CHECK(ensure_vjp_buf(p, P));
  StackScope sc(p, P, ths);
  VJ_CHECK(stack_vjp_setup(p, P, gtheta));
  p->stk.add(x, g.n, sizeof(float2), (int)g.n);
  p->stk.add(gz, g.m, sizeof(float2), (int)g.m);
  if (gx) p->stk.add(gx, g.n, sizeof(float2), (int)g.n);
  float2* gxi = gx ? gx : nscratch(p, g);
  float2* cur = nullptr;
  if (g.L >= 2) VJ_CHECK(fwd_passes(p, g, x, PK_MID_FWD_SAVE, gtheta, &cur));
  VJ_CHECK(adj_passes(p, g, gz, PK_MID_ADJ_GT, PK_LAST_ADJ_GT, gtheta, x, gxi));
  return stack_vjp_finish(p, P, gtheta);
}

sr_status vjp_adjoint_stacked(sr_plan_s* p, int P, int ths, const float2* r, const float2* gv, float2* gr,
                              float* gtheta) {
  const Geo& g = p->geo[0];
  VJ_CHECK(ensure_stack_bufs(p, 2 * (size_t)P * g.mg));
  VJ_CHECK(ensure_vjp_buf(p, P));
  StackScope sc(p, P, ths);
  VJ_CHECK(stack_vjp_setup(p, P, gtheta));
  p->stk.add(r, g.m, sizeof(float2), (int)g.m);
  p->stk.add(gv, g.n, sizeof(float2), (int)g.n);
  if (gr) p->stk.add(gr, g.m, sizeof(float2), (int)g.m);
  float2* v = nscratch(p, g);
  VJ_CHECK(adj_passes(p, g, r, PK_MID_ADJ_SAVE, PK_LAST_ADJ, gtheta, nullptr, v));
  {
    const long long n = g.n * P;
    const int groups = (int)std::min<long long>((n + 255) / 256, 1024);
    int sg = 0;
    p->stk.stride_of(gth_of(p, g, gtheta, 1), &sg);
    hipLaunchKernelGGL(gth_support_kernel, dim3(groups), dim3(256), 0, p->stream, gv, v, gth_of(p, g, gtheta, 1),
                       g.N1, g.N2, g.o1, g.o2, (long long)g.M2, P, (long long)sg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gth_support");
  }
  float2* cur = nullptr;
  VJ_CHECK(fwd_passes(p, g, gv, PK_MID_FWD_GT, gtheta, &cur));
  if (gr != nullptr) {
    const int k = g.L + 1;
    PassArgs a = base_args(p, g, k);
    set_in(a, g, k, cur);
    a.scale_mid = 1.f / std::sqrt((float)pass_len(g, k));
    a.z_out = gr;
    VJ_CHECK(launch(p, g, k, PK_LAST_STORE, a));
  }
  return stack_vjp_finish(p, P, gtheta);
}

}  // namespace

// ------------------------------------------------ on the batched levels
// Both products for the 2D problems of a batched plan, one launch per pass
// level over all of them: each problem's passes are recorded with its own
// ping-pong buffers and its own saved intermediates, and (the problems'
// phase blocks being disjoint, so no two tiles of a level add into the same
// cotangent) its own slice of the phase cotangents.  The adjoint product's
// first-layer term between its two halves is one small launch per problem.

struct LevelLists;
LevelLists* level_lists_new();
void level_lists_delete(LevelLists* l);
sr_status level_lists_build(sr_plan_s* p, const std::vector<std::vector<PassRecord>>& recs, LevelLists* l);
sr_status level_lists_run(sr_plan_s* p, const LevelLists* l);
sr_status level_bufs_alloc(sr_plan_s* p);

struct VjpBatchState {
  std::string key[2];
  LevelLists* lists[3] = {nullptr, nullptr, nullptr};  // A's product; A^H's two halves
  float2* save = nullptr;                               // per problem: its saved grids and an n-sized scratch
  std::vector<size_t> save_off;
  ~VjpBatchState() {
    for (LevelLists* l : lists)
      if (l) level_lists_delete(l);
    if (save) (void)hipFree(save);
  }
};

void destroy_vjp_batch_state(VjpBatchState* s) { delete s; }

namespace {

// the 2D problems the levels take, if there are at least two and their phase
// blocks are pairwise disjoint
std::vector<int> vjp_level_problems(const sr_plan_s* p) {
  std::vector<int> lvl;
  const bool want = p->schedule == SR_SCHED_BATCHED || (p->schedule == SR_SCHED_AUTO && p->geo.size() >= 8);
  if (!want) return lvl;
  for (size_t i = 0; i < p->geo.size(); ++i)
    if (batch_level_capable(p->geo[i])) lvl.push_back((int)i);
  if (lvl.size() < 2) return {};
  std::vector<std::pair<int64_t, int64_t>> iv;
  for (int i : lvl) iv.push_back({p->geo[i].th_off, p->geo[i].th_off + (int64_t)p->geo[i].L * p->geo[i].mg});
  std::sort(iv.begin(), iv.end());
  for (size_t k = 1; k < iv.size(); ++k)
    if (iv[k].first < iv[k - 1].second) return {};
  return lvl;
}

sr_status vjp_batch_prepare(sr_plan_s* p, VjpBatchState** out) {
  VJ_CHECK(level_bufs_alloc(p));
  VjpBatchState* st = p->vjp_batch;
  if (st == nullptr) {
    // built completely before the plan refers to it: a failed allocation
    // leaves no half-made state behind for the next call to reuse
    st = new VjpBatchState();
    size_t elems = 0;
    st->save_off.assign(p->geo.size(), 0);
    for (size_t i = 0; i < p->geo.size(); ++i) {
      const Geo& g = p->geo[i];
      st->save_off[i] = elems;
      if (batch_level_capable(g)) elems += (size_t)std::max(g.L - 1, 1) * g.mg + (size_t)g.n;
    }
    if (hipMalloc(&st->save, std::max<size_t>(elems, 1) * sizeof(float2)) != hipSuccess) {
      st->save = nullptr;
      delete st;
      return fail(SR_E_NOMEM, "batched derivative workspace allocation failed");
    }
    for (LevelLists*& l : st->lists) l = level_lists_new();
    p->vjp_batch = st;
  }
  *out = st;
  return SR_OK;
}

// Points the plan's pass buffers and derivative scratch at problem i's own.
struct ProblemBuffers {
  sr_plan_s* p;
  float2 *a0, *b0, *v0;
  ProblemBuffers(sr_plan_s* pl, const VjpBatchState* st, int i)
      : p(pl), a0(pl->bufA), b0(pl->bufB), v0(pl->vjp_buf) {
    const Geo& g = p->geo[i];
    p->bufA = p->lvl_bufs + p->lvl_off[i];
    p->bufB = p->lvl_bufs + p->lvl_off[i] + g.mg;
    p->vjp_buf = st->save + st->save_off[i];
  }
  ~ProblemBuffers() {
    p->bufA = a0;
    p->bufB = b0;
    p->vjp_buf = v0;
  }
};

std::string vjp_key(const std::vector<int>& lvl, std::initializer_list<const void*> ptrs) {
  std::string k;
  for (const void* q : ptrs) k += ptr_key(q) + ":";
  for (int i : lvl) k += std::to_string(i) + ",";
  return k;
}

sr_status vjp_forward_levels(sr_plan_s* p, const std::vector<int>& lvl, const float2* x, const float2* gz,
                             float2* gx, float* gtheta) {
  VjpBatchState* st = nullptr;
  VJ_CHECK(vjp_batch_prepare(p, &st));
  const std::string key = vjp_key(lvl, {x, gz, gx, gtheta});
  if (st->key[0] != key) {
    st->key[0].clear();
    std::vector<std::vector<PassRecord>> recs(p->geo.size());
    sr_status status = SR_OK;
    for (int i : lvl) {
      const Geo& g = p->geo[i];
      ProblemBuffers pb(p, st, i);
      const float2* xi = x + p->xoff[i];
      float2* gxi = gx ? gx + p->xoff[i] : nscratch(p, g);
      g_recording = &recs[i];
      float2* cur = nullptr;
      if (g.L >= 2) status = fwd_passes(p, g, xi, PK_MID_FWD_SAVE, gtheta, &cur);
      if (status == SR_OK) status = adj_passes(p, g, gz + p->yoff[i], PK_MID_ADJ_GT, PK_LAST_ADJ_GT, gtheta, xi, gxi);
      g_recording = nullptr;
      if (status != SR_OK) return status;
    }
    VJ_CHECK(level_lists_build(p, recs, st->lists[0]));
    st->key[0] = key;
  }
  return level_lists_run(p, st->lists[0]);
}

sr_status vjp_adjoint_levels(sr_plan_s* p, const std::vector<int>& lvl, const float2* r, const float2* gv,
                             float2* gr, float* gtheta) {
  VjpBatchState* st = nullptr;
  VJ_CHECK(vjp_batch_prepare(p, &st));
  const std::string key = vjp_key(lvl, {r, gv, gr, gtheta});
  if (st->key[1] != key) {
    st->key[1].clear();
    std::vector<std::vector<PassRecord>> ra(p->geo.size()), rb(p->geo.size());
    sr_status status = SR_OK;
    for (int i : lvl) {
      const Geo& g = p->geo[i];
      ProblemBuffers pb(p, st, i);
      g_recording = &ra[i];
      status = adj_passes(p, g, r + p->yoff[i], PK_MID_ADJ_SAVE, PK_LAST_ADJ, gtheta, nullptr, nscratch(p, g));
      g_recording = &rb[i];
      float2* cur = nullptr;
      if (status == SR_OK) status = fwd_passes(p, g, gv + p->xoff[i], PK_MID_FWD_GT, gtheta, &cur);
      if (status == SR_OK && gr != nullptr) {
        const int k = g.L + 1;
        PassArgs a = base_args(p, g, k);
        set_in(a, g, k, cur);
        a.scale_mid = 1.f / std::sqrt((float)pass_len(g, k));
        a.z_out = gr + p->yoff[i];
        status = launch(p, g, k, PK_LAST_STORE, a);
      }
      g_recording = nullptr;
      if (status != SR_OK) return status;
    }
    VJ_CHECK(level_lists_build(p, ra, st->lists[1]));
    VJ_CHECK(level_lists_build(p, rb, st->lists[2]));
    st->key[1] = key;
  }
  VJ_CHECK(level_lists_run(p, st->lists[1]));
  // first layer: gth_1 += Im(conj(gv) v) on each problem's support
  for (int i : lvl) {
    const Geo& g = p->geo[i];
    const float2* v = st->save + st->save_off[i] + (size_t)std::max(g.L - 1, 1) * g.mg;  // the problem's scratch
    const long long n = g.n;
    const int groups = (int)std::min<long long>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(gth_support_kernel, dim3(groups), dim3(256), 0, p->stream, gv + p->xoff[i], v,
                       gtheta + g.th_off, g.N1, g.N2, g.o1, g.o2, (long long)g.M2, 1, 0LL);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "gth_support");
  }
  return level_lists_run(p, st->lists[2]);
}

}  // namespace

sr_status vjp_forward(sr_plan_s* p, const float2* x, const float2* gz, float2* gx, float* gtheta) {
  {
    int ths = 0;
    const int P = stack_size(p, &ths);
    if (P > 1) return vjp_forward_stacked(p, P, ths, x, gz, gx, gtheta);
  }
  const std::vector<int> lvl = vjp_level_problems(p);
  std::vector<char> done(p->geo.size(), 0);
  if (!lvl.empty()) {
    VJ_CHECK(vjp_forward_levels(p, lvl, x, gz, gx, gtheta));
    for (int i : lvl) done[i] = 1;
  }
  VJ_CHECK(ensure_vjp_buf(p));
  for (size_t i = 0; i < p->geo.size(); ++i) {
    if (done[i]) continue;
    const Geo& g = p->geo[i];
    const float2* xi = x + p->xoff[i];
    const float2* gzi = gz + p->yoff[i];
    if (g.ndim == 1) {
      Fused1DArgs a{};
      a.x_in = xi;
      a.r_in = gzi;
      a.x_out = gx ? gx + p->xoff[i] : nullptr;
      a.gth = gtheta + g.th_off;
      VJ_CHECK(fused1d_vjp(p, g, F1_FWD_VJP, a));
      continue;
    }
    float2* gxi = gx ? gx + p->xoff[i] : nscratch(p, g);
    float2* cur = nullptr;
    if (g.L >= 2) VJ_CHECK(fwd_passes(p, g, xi, PK_MID_FWD_SAVE, gtheta, &cur));
    VJ_CHECK(adj_passes(p, g, gzi, PK_MID_ADJ_GT, PK_LAST_ADJ_GT, gtheta, xi, gxi));
  }
  return SR_OK;
}

sr_status vjp_adjoint(sr_plan_s* p, const float2* r, const float2* gv, float2* gr, float* gtheta) {
  {
    int ths = 0;
    const int P = stack_size(p, &ths);
    if (P > 1) return vjp_adjoint_stacked(p, P, ths, r, gv, gr, gtheta);
  }
  const std::vector<int> lvl = vjp_level_problems(p);
  std::vector<char> done(p->geo.size(), 0);
  if (!lvl.empty()) {
    VJ_CHECK(vjp_adjoint_levels(p, lvl, r, gv, gr, gtheta));
    for (int i : lvl) done[i] = 1;
  }
  VJ_CHECK(ensure_vjp_buf(p));
  for (size_t i = 0; i < p->geo.size(); ++i) {
    if (done[i]) continue;
    const Geo& g = p->geo[i];
    const float2* ri = r + p->yoff[i];
    const float2* gvi = gv + p->xoff[i];
    if (g.ndim == 1) {
      Fused1DArgs a{};
      a.r_in = ri;
      a.x_in = gvi;
      a.z_out = gr ? gr + p->yoff[i] : nullptr;
      a.gth = gtheta + g.th_off;
      VJ_CHECK(fused1d_vjp(p, g, F1_ADJ_VJP, a));
      continue;
    }
    // recompute q_k (k >= 2) and v = A^H r
    float2* v = nscratch(p, g);
    VJ_CHECK(adj_passes(p, g, ri, PK_MID_ADJ_SAVE, PK_LAST_ADJ, gtheta, nullptr, v));
    // first layer: gth_1 += Im(conj(gv) v) on the support
    {
      const long long n = g.n;
      const int groups = (int)std::min<long long>((n + 255) / 256, 1024);
      hipLaunchKernelGGL(gth_support_kernel, dim3(groups), dim3(256), 0, p->stream, gvi, v, gth_of(p, g, gtheta, 1),
                         g.N1, g.N2, g.o1, g.o2, (long long)g.M2, 1, 0LL);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_fail(e, "gth_support");
    }
    // forward passes on gv with the cotangents of layers 2..L, then A gv
    float2* cur = nullptr;
    VJ_CHECK(fwd_passes(p, g, gvi, PK_MID_FWD_GT, gtheta, &cur));
    if (gr != nullptr) {
      const int k = g.L + 1;
      PassArgs a = base_args(p, g, k);
      set_in(a, g, k, cur);
      a.scale_mid = 1.f / std::sqrt((float)pass_len(g, k));
      a.z_out = gr + p->yoff[i];
      VJ_CHECK(launch(p, g, k, PK_LAST_STORE, a));
    }
  }
  return SR_OK;
}

}  // namespace sr

namespace sr {

// ------------------------------------------- GD-step and intensity derivatives
// One GD step (section II-B.1, Eq. (2)): z = A x, r = (|z|^2 - y) z,
// x+ = x - (eta/m) A^H r.  Given the cotangent xbar+ of x+ (PyTorch's
// convention), the reverse step is
//   vbar = -(eta/m) xbar+,   (rbar, thetabar) from the derivative of A^H r,
//   zbar = (2|z|^2 - y) rbar + z^2 conj(rbar),   ybar += -Re(conj(rbar) z),
//   (xbar_A, thetabar) from the derivative of A x,   xbar = xbar+ + xbar_A,
// with z recomputed from x (nothing of the forward step is kept but x).
// The intensities y = |A x|^2 (Eq. (1)) have zbar = 2 ybar z.
namespace {

// problem b = blockIdx.y covers [off[b], off[b + 1]) of a concatenated array
#define SR_PROBLEM_RANGE(off)                                                                     \
  const long long lo_ = (off)[blockIdx.y], hi_ = (off)[blockIdx.y + 1];                          \
  for (long long e = lo_ + blockIdx.x * (long long)blockDim.x + threadIdx.x; e < hi_;            \
       e += (long long)gridDim.x * blockDim.x)

// r = (|z|^2 - y) z   (the l2 residual of the GD step)
__global__ void step_resid_kernel(const float2* __restrict__ z, const float* __restrict__ y, float2* __restrict__ r,
                                  const int64_t* __restrict__ yoff) {
  SR_PROBLEM_RANGE(yoff) {
    const float2 zz = z[e];
    r[e] = cscale(zz, cabs2(zz) - y[e]);
  }
}

// out = s_b * in over problem b's signal (s_b = -eta_b / m_b)
__global__ void step_scale_kernel(const float2* __restrict__ in, const float* __restrict__ s, float2* __restrict__ out,
                                  const int64_t* __restrict__ xoff) {
  const float sb = s[blockIdx.y];
  SR_PROBLEM_RANGE(xoff) out[e] = cscale(in[e], sb);
}

// rbar -> zbar = (2|z|^2 - y) rbar + z^2 conj(rbar) in place; gy += -Re(conj(rbar) z)
__global__ void step_zbar_kernel(const float2* __restrict__ z, const float* __restrict__ y, float2* __restrict__ rz,
                                 float* __restrict__ gy, const int64_t* __restrict__ yoff) {
  SR_PROBLEM_RANGE(yoff) {
    const float2 zz = z[e], rb = rz[e];
    const float a = 2.f * cabs2(zz) - y[e];
    const float2 z2 = cmul(zz, zz);
    rz[e] = make_float2(a * rb.x + z2.x * rb.x + z2.y * rb.y, a * rb.y + z2.y * rb.x - z2.x * rb.y);
    if (gy != nullptr) gy[e] -= rb.x * zz.x + rb.y * zz.y;
  }
}

// out = a + b
__global__ void step_add_kernel(const float2* __restrict__ a, const float2* __restrict__ b, float2* __restrict__ out,
                                long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    out[e] = cadd(a[e], b[e]);
}

// z <- 2 gy z   (cotangent of z from that of y = |z|^2)
__global__ void intensity_bar_kernel(float2* __restrict__ z, const float* __restrict__ gy, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    z[e] = cscale(z[e], 2.f * gy[e]);
}

#undef SR_PROBLEM_RANGE

dim3 range_grid(const sr_plan_s* p, bool meas) {
  int64_t longest = 0;
  for (const Geo& g : p->geo) longest = std::max(longest, meas ? g.m : g.n);
  return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((longest + 255) / 256, 512)), (unsigned)p->geo.size());
}

dim3 flat_grid(long long n) { return dim3((unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 4096))); }

// The temporaries (3 measurement-layout arrays, 2 signal-layout ones) and the
// device offset table, allocated once per plan.
sr_status step_bufs(sr_plan_s* p) {
  if (p->gstep_buf != nullptr) return SR_OK;
  const size_t m = (size_t)p->yoff.back(), n = (size_t)p->xoff.back(), np = p->geo.size();
  float2* buf = nullptr;
  if (hipMalloc(&buf, (3 * m + 2 * n) * sizeof(float2)) != hipSuccess)
    return fail(SR_E_NOMEM, "GD-step derivative workspace allocation failed");
  int64_t* off = nullptr;
  if (hipMalloc(&off, 2 * (np + 1) * sizeof(int64_t)) != hipSuccess) {
    (void)hipFree(buf);
    return fail(SR_E_NOMEM, "offset table allocation failed");
  }
  float* sc = nullptr;
  if (hipMalloc(&sc, np * sizeof(float)) != hipSuccess) {
    (void)hipFree(buf);
    (void)hipFree(off);
    return fail(SR_E_NOMEM, "step table allocation failed");
  }
  // the plan's offset vectors live as long as the plan: an ordered copy
  hipError_t e = hipMemcpyAsync(off, p->xoff.data(), (np + 1) * sizeof(int64_t), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(off + np + 1, p->yoff.data(), (np + 1) * sizeof(int64_t), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    (void)hipFree(buf);
    (void)hipFree(off);
    (void)hipFree(sc);
    return hip_fail(e, "offset table upload");
  }
  p->gstep_buf = buf;
  p->d_off = off;
  p->d_scale = sc;
  return SR_OK;
}

}  // namespace

sr_status gd_step_vjp(sr_plan_s* p, const float* y, const float2* x, const float* eta_host, const float2* gxn,
                      float2* gx, float* gy, float* gtheta) {
  VJ_CHECK(step_bufs(p));
  const size_t m = (size_t)p->yoff.back(), n = (size_t)p->xoff.back(), np = p->geo.size();
  float2* z = p->gstep_buf;
  float2* r = z + m;
  float2* rz = r + m;     // rbar, then zbar
  float2* vbar = rz + m;  // -(eta/m) xbar+
  float2* gxa = vbar + n; // A^H zbar
  const int64_t* xoff = p->d_off;
  const int64_t* yoff = p->d_off + np + 1;
  std::vector<float> s(np);
  for (size_t i = 0; i < np; ++i) s[i] = -eta_host[i] / (float)p->geo[i].m;
  VJ_CHECK(put_floats(p, p->d_scale, s.data(), (int)np));
  // recompute z = A x and r
  VJ_CHECK(sr_forward(p, x, z, nullptr));
  hipLaunchKernelGGL(step_resid_kernel, range_grid(p, true), dim3(256), 0, p->stream, z, y, r, yoff);
  hipLaunchKernelGGL(step_scale_kernel, range_grid(p, false), dim3(256), 0, p->stream, gxn, p->d_scale, vbar, xoff);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return hip_fail(e, "GD-step derivative kernels");
  // through A^H r: rbar and the phase terms of the adjoint
  VJ_CHECK(vjp_adjoint(p, r, vbar, rz, gtheta));
  hipLaunchKernelGGL(step_zbar_kernel, range_grid(p, true), dim3(256), 0, p->stream, z, y, rz, gy, yoff);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return hip_fail(e, "GD-step derivative kernels");
  // through z = A x: the signal cotangent and the phase terms of the forward operator
  VJ_CHECK(vjp_forward(p, x, rz, gxa, gtheta));
  hipLaunchKernelGGL(step_add_kernel, flat_grid((long long)n), dim3(256), 0, p->stream, gxn, gxa, gx, (long long)n);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return hip_fail(e, "GD-step derivative kernels");
  return SR_OK;
}

sr_status intensity_vjp(sr_plan_s* p, const float2* x, const float* gy, float2* gx, float* gtheta) {
  VJ_CHECK(step_bufs(p));
  const size_t m = (size_t)p->yoff.back();
  float2* z = p->gstep_buf;
  VJ_CHECK(sr_forward(p, x, z, nullptr));
  hipLaunchKernelGGL(intensity_bar_kernel, flat_grid((long long)m), dim3(256), 0, p->stream, z, gy, (long long)m);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return hip_fail(e, "intensity derivative kernel");
  return vjp_forward(p, x, z, gx, gtheta);
}

}  // namespace sr
