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

inline PassArgs base_args(const sr_plan_s* p, const Geo& g, int k) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.grid_ld = g.M2;
  a.tw = p->twiddles(pass_len(g, k), 0);
  a.tw_n = p->twiddles(pass_len(g, k), 1);
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
constexpr size_t kGraphCacheSize = 8;

inline bool graphs_enabled(const sr_plan_s* p) {
  if (p->schedule == SR_SCHED_LOOP) return false;
  const char* e = std::getenv("SR_GRAPH");
  return e == nullptr || std::atoi(e) != 0;
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
    if (graph) hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  if (p->graphs.size() >= kGraphCacheSize) {
    hipGraphExecDestroy(p->graphs.front().second);
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
