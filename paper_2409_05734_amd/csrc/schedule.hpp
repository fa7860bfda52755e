// Pass scheduling helpers shared by the operator, solver and derivative
// drivers: axis and length of each fused pass, buffer layouts between passes,
// and the launch hook (with optional recording for the persistent solver).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "launch.hpp"
#include "plan.hpp"

namespace sr {


inline int pass_col(int k) { return (k % 2) == 1; }  // forward pass k (1-based): odd -> axis 0
inline int pass_len(const Geo& g, int k) { return pass_col(k) ? g.M1 : g.M2; }

// The tile a pass other than [F D F] / [F^H D^* F^H] runs (the passes that
// write or read per-tile partial sums are among them): the tuner's choice,
// or the length's default where that choice is the wide shape, which only
// those two column passes have (launch_pass falls back the same way).
inline int tile_other(const sr_plan_s* p, int N, bool col) {
  int b = p->tile(N, col);
  if (b <= 0 || (b & kWide)) b = default_tile(N, col);
  return b;
}

inline PassArgs base_args(const sr_plan_s* p, const Geo& g, int k) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.grid_ld = g.M2;
  a.tw = p->twiddles(pass_len(g, k), 0);
  // the length's other thread shape: narrow, or wide (no length has both)
  a.tw_n = p->twiddles(pass_len(g, k), 1) ? p->twiddles(pass_len(g, k), 1) : p->twiddles(pass_len(g, k), 2);
  a.scale_pre = 1.f;
  a.scale_mid = 1.f;
  a.scale_out = 1.f;
  a.inv_m = 1.f / (float)g.m;
  a.win_lo0 = g.c1;
  a.win_hi0 = g.c1 + g.W1;
  a.win_lo1 = g.c2;
  a.win_hi1 = g.c2 + g.W2;
  a.win_ld = g.W2;
  a.crop = g.cropped() ? 1 : 0;
  a.loss_eps = p->loss_eps;
  a.nf = p->sync + 2;
  return a;
}

// Buffer layouts between passes.  "Compact" buffers hold only the N2 support
// columns (M1 x N2, row-major); "full" buffers hold the whole M1 x M2 grid.
// The output of forward pass 1 and the input of the last adjoint pass are
// compact; every other intermediate is full.

// Row-mode input from a compact buffer (pass 2 reads the output of pass 1).
inline void in_compact(PassArgs& a, const Geo& g, const float2* buf) {
  a.in = buf;
  a.in_ld = g.N2;
  a.in_lo = g.o2;
  a.in_hi = g.o2 + g.N2;
  a.ntr = g.M1;
  a.tr_lo = 0;
}

// Input from a full grid buffer, for a pass on the axis of forward pass k.
inline void in_full(PassArgs& a, const Geo& g, int k, const float2* buf) {
  a.in = buf;
  a.in_ld = g.M2;
  a.in_lo = 0;
  a.in_hi = pass_len(g, k);
  a.ntr = pass_col(k) ? g.M2 : g.M1;
  a.tr_lo = 0;
}

// Input of forward pass k >= 2 (the output of pass k-1).
inline void set_in(PassArgs& a, const Geo& g, int k, const float2* buf) {
  if (k == 2) in_compact(a, g, buf);
  else in_full(a, g, k, buf);
}

// Output of a pass on the axis of pass k: compact for k == 2, full otherwise.
inline void set_out(PassArgs& a, const Geo& g, int k, float2* buf) {
  a.out = buf;
  if (k == 2) {
    a.out_ld = g.N2;
    a.out_lo = g.o2;
    a.out_hi = g.o2 + g.N2;
  } else {
    a.out_ld = g.M2;
    a.out_lo = 0;
    a.out_hi = pass_len(g, k);
  }
}

inline void out_full(PassArgs& a, const Geo& g, int k, float2* buf) {
  a.out = buf;
  a.out_ld = g.M2;
  a.out_lo = 0;
  a.out_hi = pass_len(g, k);
}

// Problems of one 2D geometry whose phase blocks are equal (shared masks) or
// evenly spaced without overlap run as a stack: every fused pass is one
// launch for all of them.  Returns the stack size (1: the plan does not
// qualify) and the spacing of the phase blocks.  SR_STACK=0 turns it off.
inline int stack_size(const sr_plan_s* p, int* th_stride) {
  const size_t np = p->geo.size();
  if (p->kind != SR_STRUCTURED || np < 2 || p->schedule == SR_SCHED_LOOP) return 1;
  const char* env = std::getenv("SR_STACK");
  if (env != nullptr && std::atoi(env) == 0) return 1;
  const Geo& g0 = p->geo[0];
  if (g0.ndim != 2) return 1;
  const int64_t d = p->geo[1].th_off - g0.th_off;
  const int64_t block = (int64_t)g0.L * g0.mg;
  if (d < 0 || (d != 0 && d < block)) return 1;
  for (size_t i = 0; i < np; ++i) {
    const Geo& g = p->geo[i];
    if (g.ndim != 2 || g.N1 != g0.N1 || g.N2 != g0.N2 || g.M1 != g0.M1 || g.M2 != g0.M2 || g.W1 != g0.W1 ||
        g.W2 != g0.W2 || g.L != g0.L || g.th_off != g0.th_off + (int64_t)i * d)
      return 1;
  }
  // every offset inside a stacked buffer stays well within 32-bit byte offsets
  const int64_t lim = (int64_t)1 << 26;
  if ((int64_t)np * std::max<int64_t>(block, std::max<int64_t>(g0.mg, d)) >= lim) return 1;
  *th_stride = (int)d;
  return (int)np;
}

// The plan's ping-pong buffers for a stack of P problems (P grids each).
inline sr_status ensure_stack_bufs(sr_plan_s* p, size_t elems) {
  if (elems <= p->stk_elems) return SR_OK;
  if (p->stk_buf) {
    // queued work may still use the old buffer
    if (hipError_t w = hipStreamSynchronize(p->stream); w != hipSuccess) return hip_fail(w, "stream wait");
    (void)hipFree(p->stk_buf);
    p->stk_buf = nullptr;
    p->stk_elems = 0;
  }
  hipError_t e = hipMalloc(&p->stk_buf, elems * sizeof(float2));
  if (e != hipSuccess) return fail(SR_E_NOMEM, "stacked workspace allocation failed");
  p->stk_elems = elems;
  return SR_OK;
}

inline sr_status ensure_stack_parts(sr_plan_s* p, size_t elems) {
  if (elems <= p->stk_part_elems) return SR_OK;
  if (p->stk_part) {
    // queued work may still use the old buffer
    if (hipError_t w = hipStreamSynchronize(p->stream); w != hipSuccess) return hip_fail(w, "stream wait");
    (void)hipFree(p->stk_part);
    p->stk_part = nullptr;
    p->stk_part_elems = 0;
  }
  hipError_t e = hipMalloc(&p->stk_part, elems * sizeof(float));
  if (e != hipSuccess) return fail(SR_E_NOMEM, "stacked partial-sum allocation failed");
  p->stk_part_elems = elems;
  return SR_OK;
}

// Runs a stack for the lifetime of the object: the plan's ping-pong buffers
// are the stacked ones (registered with stride mg), restored afterwards.
struct StackScope {
  sr_plan_s* p;
  float2 *a0, *b0;
  StackScope(sr_plan_s* pl, int P, int th_stride) : p(pl), a0(pl->bufA), b0(pl->bufB) {
    const Geo& g = p->geo[0];
    p->stk.P = P;
    p->stk.th_stride = th_stride;
    p->stk.regions.clear();
    p->bufA = p->stk_buf;
    p->bufB = p->stk_buf + (size_t)P * g.mg;
    p->stk.add(p->bufA, g.mg, sizeof(float2), (int)g.mg);
    p->stk.add(p->bufB, g.mg, sizeof(float2), (int)g.mg);
  }
  ~StackScope() {
    p->bufA = a0;
    p->bufB = b0;
    p->stk = StackState{};
  }
};

// Launch one fused pass, or, while a persistent schedule is being recorded,
// append it to the recording instead.
struct PassRecord {
  int k, kind;
  PassArgs a;
};
inline std::vector<PassRecord>* g_recording = nullptr;

// exp(i theta) table entry parallel to a phase pointer (the table mirrors
// the phase buffer's layout)
inline const float2* table_of(const sr_plan_s* p, const float* th) {
  return th == nullptr ? nullptr : p->eph + (th - p->theta);
}

inline sr_status launch(sr_plan_s* p, const Geo& g, int k, int kind, const PassArgs& a_in) {
  PassArgs a = a_in;
  if (p->use_table) {
    a.ep_pre = table_of(p, a.th_pre);
    a.ep_mid = table_of(p, a.th_mid);
    a.ep_post = table_of(p, a.th_post);
  }
  if (p->stk.P > 1) {  // one launch for the whole stack
    a.stack = p->stk.P;
    a.ntr_p = a.ntr;
    a.ntr *= p->stk.P;
    a.s_th = p->stk.th_stride;
    int sy = 0, sz = 0, syo = 0;
    const StackState& st = p->stk;
    if (!st.stride_of(a.in, &a.s_in) || !st.stride_of(a.out, &a.s_out) || !st.stride_of(a.out2, &a.s_out2) ||
        !st.stride_of(a.save, &a.s_save) || !st.stride_of(a.gth, &a.s_gth) || !st.stride_of(a.xin, &a.s_xin) ||
        !st.stride_of(a.y, &sy) || !st.stride_of(a.z_out, &sz) || !st.stride_of(a.y_out, &syo))
      return fail(SR_E_STATE, "stacked pass: a buffer without a per-problem stride");
    a.s_win = std::max(sy, std::max(sz, syo));  // measurement-shaped buffers share one stride
    a.step_v = p->stk.steps;
    if (a.part_in != nullptr || a.part_out != nullptr) {  // per-problem partial sums: whole problems per tile
      const int bt = tile_other(p, pass_len(g, k), pass_col(k)) & (kSingleBuffer - 1);
      if (a.ntr_p % bt != 0) return fail(SR_E_STATE, "stacked pass with partial sums: a tile spans two problems");
    }
  }
  if (g_recording != nullptr) {
    g_recording->push_back({k, kind, a});
    return SR_OK;
  }
  const int N = pass_len(g, k);
  const bool col = pass_col(k);
  hipError_t e = launch_pass(N, kind, col, p->tile(N, col), a, p->stream);
  if (e != hipSuccess) return hip_fail(e, "pass launch");
  return SR_OK;
}



// ------------------------------------------------------------- graphs
// Solver iterations are captured once into a hipGraph (on a private stream)
// and replayed on the plan's stream: one graph launch per chunk of
// iterations instead of 2L+1 kernel launches per iteration.  Graphs are
// cached by the call's pointers and scalars; SR_GRAPH=0 disables them.

constexpr int kGraphChunk = 50;  // iterations per captured graph (even)
constexpr int kGraphTail = 8;    // a remainder of at least this many steady iterations gets a graph too
constexpr size_t kGraphCacheSize = 8;

inline bool graphs_enabled(const sr_plan_s* p) {
  if (p->schedule == SR_SCHED_LOOP) return false;
  const char* e = std::getenv("SR_GRAPH");
  return e == nullptr || std::atoi(e) != 0;
}

// Destroy the captured graphs whose key starts with `prefix`, once the stream
// has drained: their kernels take device lists that the caller is about to
// free and rebuild, and a later call under the same key must capture anew.
inline sr_status drop_graphs(sr_plan_s* p, const std::string& prefix) {
  auto hit = [&](const std::pair<std::string, hipGraphExec_t>& g) { return g.first.compare(0, prefix.size(), prefix) == 0; };
  if (std::none_of(p->graphs.begin(), p->graphs.end(), hit)) return SR_OK;
  if (hipError_t e = hipStreamSynchronize(p->stream); e != hipSuccess) return hip_fail(e, "stream wait");
  auto keep = std::remove_if(p->graphs.begin(), p->graphs.end(), [&](const auto& g) {
    if (!hit(g)) return false;
    (void)hipGraphExecDestroy(g.second);
    return true;
  });
  p->graphs.erase(keep, p->graphs.end());
  return SR_OK;
}

template <class F>
sr_status launch_captured(sr_plan_s* p, const std::string& key, F&& enqueue) {
  for (auto it = p->graphs.begin(); it != p->graphs.end(); ++it) {
    if (it->first == key) {
      hipGraphExec_t ex = it->second;
      std::rotate(it, it + 1, p->graphs.end());  // most recent last
      {
        hipError_t le = hipGraphLaunch(ex, p->stream);
        if (le != hipSuccess) return hip_fail(le, "hipGraphLaunch");
      }
      return SR_OK;
    }
  }
  hipStream_t user = p->stream;
  p->stream = p->cap_stream;
  hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    p->stream = user;
    return hip_fail(e, "hipStreamBeginCapture");
  }
  sr_status st = enqueue();
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(p->cap_stream, &graph);
  p->stream = user;
  if (st != SR_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  if (p->graphs.size() >= kGraphCacheSize) {
    (void)hipGraphExecDestroy(p->graphs.front().second);
    p->graphs.erase(p->graphs.begin());
  }
  p->graphs.push_back({key, ex});
  e = hipGraphLaunch(ex, p->stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return SR_OK;
}

inline std::string ptr_key(const void* a) {
  char buf[32];
  std::snprintf(buf, sizeof(buf), "%p", a);
  return buf;
}

inline std::string float_key(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return std::to_string(u);
}

}  // namespace sr
