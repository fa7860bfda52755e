// C ABI of libsrpr: plan creation and validation, pass scheduling for the
// structured operator (section III, Eq. (5)), the spectral initialisation
// (section II-B.2, Eq. (3)-(4)) and gradient descent (section II-B.1, Eq. (2)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/sr.h"
#include "fused1d.hpp"
#include "launch.hpp"
#include "persist.hpp"
#include "plan.hpp"
#include "schedule.hpp"

using sr::Geo;

namespace {
thread_local std::string g_last_error;
}

namespace sr {

sr_status fail(sr_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

sr_status hip_fail(hipError_t e, const char* what) {
  return fail(SR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

bool supported_len_2d(int M) {
  switch (M) {
    case 16: case 32: case 64: case 96: case 128: case 192: case 256: case 384: case 512: case 768: case 1024: case 2048:
      return true;
    default:
      return false;
  }
}

bool supported_len_1d(int M) {
  switch (M) {
    case 16: case 32: case 64: case 96: case 128: case 192: case 256: case 384: case 512: case 768: case 1024: case 2048:
    case 4096:
      return true;
    default:
      return false;
  }
}

}  // namespace sr

using namespace sr;

#define SR_HIP(call)                                  \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

#define SR_CHECK(st)                  \
  do {                                \
    sr_status s_ = (st);              \
    if (s_ != SR_OK) return s_;       \
  } while (0)

const float* sr_plan_s::theta_l(const Geo& g, int l) const { return theta + g.th_off + (int64_t)(l - 1) * g.mg; }

// Pass 1, [U, D_1, F_0] on the support columns of x, into the compact bufA.
static sr_status first_pass(sr_plan_s* p, const Geo& g, const float2* x, float in_scale, const float* part_in,
                            int npart) {
  PassArgs a = base_args(p, g, 1);
  a.in = x;
  a.in_ld = g.N2;
  a.in_lo = g.o1;
  a.in_hi = g.o1 + g.N1;
  a.ntr = g.N2;
  a.tr_lo = g.o2;
  a.th_pre = p->theta_l(g, 1);
  a.scale_pre = in_scale;
  a.part_in = part_in;
  a.npart = npart;
  a.out = p->bufA;
  a.out_ld = g.N2;
  a.out_lo = 0;
  a.out_hi = g.M1;
  a.scale_out = 1.f / std::sqrt((float)g.M1);
  return launch(p, g, 1, PK_FIRST_FWD, a);
}

// Passes 2..L from the compact bufA.  Returns the buffer holding the result
// (compact bufA if L == 1, else a full grid).
static sr_status forward_rest(sr_plan_s* p, const Geo& g, float2** cur_out) {
  float2* bufs[2] = {p->bufA, p->bufB};
  int which = 0;
  for (int k = 2; k <= g.L; ++k) {
    PassArgs a = base_args(p, g, k);
    set_in(a, g, k, bufs[which]);
    out_full(a, g, k, bufs[which ^ 1]);
    a.th_mid = p->theta_l(g, k);
    const float s = 1.f / std::sqrt((float)pass_len(g, k));
    a.scale_mid = s;
    a.scale_out = s;
    SR_CHECK(launch(p, g, k, PK_MID_FWD, a));
    which ^= 1;
  }
  *cur_out = bufs[which];
  return SR_OK;
}

// Forward passes 1..L (through D_L's first transform), starting from x.
static sr_status forward_body(sr_plan_s* p, const Geo& g, const float2* x, float in_scale, const float* part_in,
                              int npart, float2** cur_out) {
  SR_CHECK(first_pass(p, g, x, in_scale, part_in, npart));
  return forward_rest(p, g, cur_out);
}

// Adjoint passes L..1 starting from `cur` (layout of the output of pass L+1's
// mirror: compact if L == 1, full otherwise), ending with the column pass that
// applies D_1^*, crops, and performs `last_kind` into x.
static sr_status adjoint_body(sr_plan_s* p, const Geo& g, float2* cur, int last_kind, float2* x, float step,
                              float two_lam, const float* part_in, int npart, float* part_out,
                              float2* out2 = nullptr) {
  float2* other = (cur == p->bufA) ? p->bufB : p->bufA;
  for (int k = g.L; k >= 2; --k) {
    PassArgs a = base_args(p, g, k);
    in_full(a, g, k, cur);
    set_out(a, g, k, other);
    a.th_mid = p->theta_l(g, k);
    const float s = 1.f / std::sqrt((float)pass_len(g, k));
    a.scale_mid = s;
    a.scale_out = s;
    SR_CHECK(launch(p, g, k, PK_MID_ADJ, a));
    std::swap(cur, other);
  }
  PassArgs a = base_args(p, g, 1);
  a.in = cur;
  a.in_ld = g.N2;
  a.in_lo = 0;
  a.in_hi = g.M1;
  a.ntr = g.N2;
  a.tr_lo = g.o2;
  a.out = x;
  a.out_ld = g.N2;
  a.out_lo = g.o1;
  a.out_hi = g.o1 + g.N1;
  a.th_post = p->theta_l(g, 1);
  a.scale_out = 1.f / std::sqrt((float)g.M1);
  a.step = step;
  a.two_lam = two_lam;
  a.part_in = part_in;
  a.npart = npart;
  a.part_out = part_out;
  a.out2 = out2;
  a.out2_ld = g.N2;
  return launch(p, g, 1, last_kind, a);
}

// The turnaround pass (index L+1): from the forward result `cur` through the
// epilogue and back; writes into the other ping-pong buffer.
static sr_status turnaround(sr_plan_s* p, const Geo& g, float2* cur, int kind, const float* y, float lam,
                            const double* ysum, float* part_out, float2** out) {
  const int k = g.L + 1;
  float2* other = (cur == p->bufA) ? p->bufB : p->bufA;
  PassArgs a = base_args(p, g, k);
  set_in(a, g, k, cur);
  set_out(a, g, k, other);
  const float s = 1.f / std::sqrt((float)pass_len(g, k));
  a.scale_mid = s;
  a.scale_out = s;
  a.y = y;
  a.lam = lam;
  a.ysum = ysum;
  a.part_out = part_out;
  SR_CHECK(launch(p, g, k, kind, a));
  *out = other;
  return SR_OK;
}

// --------------------------------------------------------------- 2D drivers

static sr_status forward_2d(sr_plan_s* p, const Geo& g, const float2* x, float2* z, float* y) {
  float2* cur = nullptr;
  SR_CHECK(forward_body(p, g, x, 1.f, nullptr, 0, &cur));
  const int k = g.L + 1;
  PassArgs a = base_args(p, g, k);
  set_in(a, g, k, cur);
  a.scale_mid = 1.f / std::sqrt((float)pass_len(g, k));
  a.z_out = z;
  a.y_out = y;
  return launch(p, g, k, PK_LAST_STORE, a);
}

static sr_status adjoint_2d(sr_plan_s* p, const Geo& g, const float2* r, float2* x) {
  const int k = g.L + 1;
  PassArgs a = base_args(p, g, k);
  in_full(a, g, k, r);
  set_out(a, g, k, p->bufA);
  a.scale_out = 1.f / std::sqrt((float)pass_len(g, k));
  SR_CHECK(launch(p, g, k, PK_FIRST_ADJ, a));
  return adjoint_body(p, g, p->bufA, PK_LAST_ADJ, x, 0.f, 0.f, nullptr, 0, nullptr);
}

// The turnaround pass of a GD iteration for the plan's loss.
static int gd_turn_kind(const sr_plan_s* p) { return p->loss == SR_LOSS_POISSON ? PK_TURN_GD_POIS : PK_TURN_GD; }

static sr_status gd_iter_2d(sr_plan_s* p, const Geo& g, const float* y, float2* x, float step, float* loss_part) {
  float2* cur = nullptr;
  SR_CHECK(forward_body(p, g, x, 1.f, nullptr, 0, &cur));
  float2* back = nullptr;
  SR_CHECK(turnaround(p, g, cur, gd_turn_kind(p), y, 0.f, nullptr, loss_part, &back));
  return adjoint_body(p, g, back, PK_LAST_GD, x, step, 0.f, nullptr, 0, nullptr);
}


// One power iteration with deferred normalisation: the passes run on the
// unnormalised iterate u and the last pass scales by 1/||u|| (A is linear and
// T(y) does not depend on the scale).
static sr_status spec_iter_2d(sr_plan_s* p, const Geo& g, const float* y, float2* u, float lam, float inv_mc,
                              const double* ysum, const float* part_in, int npart_in, float* part_out) {
  float2* cur = nullptr;
  SR_CHECK(forward_body(p, g, u, 1.f, nullptr, 0, &cur));
  float2* back = nullptr;
  SR_CHECK(turnaround(p, g, cur, PK_TURN_SPEC, y, lam, ysum, nullptr, &back));
  return adjoint_body(p, g, back, PK_LAST_SPEC, u, inv_mc, 2.f * lam, part_in, npart_in, part_out);
}

// Steady-state iterations: passes 2..L, the turnaround and the adjoint
// passes, then the update fused with the next iteration's pass 1 (writing the
// compact bufA the next pass 2 reads).  `last` selects the plain update for
// the final iteration.  2L launches per iteration instead of 2L+1.
static sr_status gd_steady(sr_plan_s* p, const Geo& g, const float* y, float2* x, float step, float* loss_part,
                           bool last) {
  float2* cur = nullptr;
  SR_CHECK(forward_rest(p, g, &cur));
  float2* back = nullptr;
  SR_CHECK(turnaround(p, g, cur, gd_turn_kind(p), y, 0.f, nullptr, loss_part, &back));
  return adjoint_body(p, g, back, last ? PK_LAST_GD : PK_LAST_GD_FWD, x, step, 0.f, nullptr, 0, nullptr,
                      last ? nullptr : p->bufA);
}

static sr_status spec_steady(sr_plan_s* p, const Geo& g, const float* y, float2* u, float lam, float inv_mc,
                             const double* ysum, const float* part_in, int npart_in, float* part_out, bool last) {
  float2* cur = nullptr;
  SR_CHECK(forward_rest(p, g, &cur));
  float2* back = nullptr;
  SR_CHECK(turnaround(p, g, cur, PK_TURN_SPEC, y, lam, ysum, nullptr, &back));
  return adjoint_body(p, g, back, last ? PK_LAST_SPEC : PK_LAST_SPEC_FWD, u, inv_mc, 2.f * lam, part_in, npart_in,
                      part_out, last ? nullptr : p->bufA);
}

namespace sr {
// Entry points for the batched schedule, which records these pass sequences.
sr_status gd_first_pass_public(sr_plan_s* p, const Geo& g, const float2* x) { return first_pass(p, g, x, 1.f, nullptr, 0); }
sr_status gd_steady_public(sr_plan_s* p, const Geo& g, const float* y, float2* x, float step, bool last,
                           float* loss_part) {
  return gd_steady(p, g, y, x, step, loss_part, last);
}
sr_status forward_2d_public(sr_plan_s* p, const Geo& g, const float2* x, float2* z, float* y) {
  return forward_2d(p, g, x, z, y);
}
sr_status adjoint_2d_public(sr_plan_s* p, const Geo& g, const float2* r, float2* x) { return adjoint_2d(p, g, r, x); }
sr_status spec_steady_public(sr_plan_s* p, const Geo& g, const float* y, float2* u, float lam, float inv_mc,
                             const double* ysum, const float* part_in, int npart_in, float* part_out, bool last) {
  return spec_steady(p, g, y, u, lam, inv_mc, ysum, part_in, npart_in, part_out, last);
}
}  // namespace sr

static int last_pass_groups(const sr_plan_s* p, const Geo& g) {
  return pass_groups(g.M1, true, tile_other(p, g.M1, true), g.N2);
}
static int turn_groups(const sr_plan_s* p, const Geo& g) {
  const int k = g.L + 1;
  const int ntr = (k == 2) ? g.M1 : (pass_col(k) ? g.M2 : g.M1);
  const int N = pass_len(g, k);
  return pass_groups(N, pass_col(k), tile_other(p, N, pass_col(k)), ntr);
}

// ------------------------------------------------------------------ tuner
// Picks the tile width of every (FFT length, mode) a plan uses by timing the
// steady-state GD iteration of each 2D problem shape for every combination of
// the compiled column- and row-tile widths and phase sources (on zeroed
// stand-in data in the plan's spare buffers; best of three runs), keeping the
// fastest.  A plan that runs as a stack is timed as a stack: there the
// bandwidth of the wider tiles beats the latency of the narrower ones that a
// single problem prefers.  SR_TUNE=0 keeps the defaults;
// SR_TUNE_CACHE=<file> reuses and records decisions across processes.

static std::string tune_key(const Geo& g) {
  return std::to_string(g.M1) + "x" + std::to_string(g.M2) + ":" + std::to_string(g.N1) + "x" +
         std::to_string(g.N2) + ":L" + std::to_string(g.L);
}

static bool tune_cache_lookup(const char* path, const std::string& key, int* cb, int* rb, int* tb) {
  if (path == nullptr) return false;
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return false;
  char k[128];
  int c = 0, r = 0, t = 0;
  bool found = false;
  while (std::fscanf(f, "%127s %d %d %d", k, &c, &r, &t) == 4)
    if (key == k) {
      *cb = c;
      *rb = r;
      *tb = t;
      found = true;
    }
  std::fclose(f);
  return found;
}

static void tune_cache_store(const char* path, const std::string& key, int cb, int rb, int tb) {
  if (path == nullptr) return;
  FILE* f = std::fopen(path, "a");
  if (f == nullptr) return;
  std::fprintf(f, "%s %d %d %d\n", key.c_str(), cb, rb, tb);
  std::fclose(f);
}

// SR_TUNE_FORCE="c,r,t" pins the column tile, row tile and phase-table
// choice for every shape (options a length does not offer fall back to its
// default); used to exercise every compiled variant.
static bool tile_offered(int N, bool col, int b) {
  int o[16];
  const int n = tile_options(N, col, o, 16);
  for (int i = 0; i < n; ++i)
    if (o[i] == b) return true;
  return false;
}

static bool stack_spectral_ok(const sr_plan_s* p, const Geo& g);
static bool stack_trace_ok(const sr_plan_s* p, const Geo& g);

static sr_status tune_plan(sr_plan_s* p) {
  const char* force = std::getenv("SR_TUNE_FORCE");
  if (force != nullptr) {
    int c = 0, r = 0, t = 0;
    if (std::sscanf(force, "%d,%d,%d", &c, &r, &t) == 3) {
      for (const Geo& g : p->geo) {
        if (g.ndim != 2) continue;
        p->tiles[{g.M1, 1}] = tile_offered(g.M1, true, c) ? c : default_tile(g.M1, true);
        p->tiles[{g.M2, 0}] = tile_offered(g.M2, false, r) ? r : default_tile(g.M2, false);
      }
      p->use_table = t != 0;
      return SR_OK;
    }
  }
  const char* env = std::getenv("SR_TUNE");
  if (env != nullptr && std::atoi(env) == 0) return SR_OK;
  const char* cache = std::getenv("SR_TUNE_CACHE");
  // a plan that runs as a stack is timed as one (up to 2^23 grid points:
  // enough to fill the GPU), on zeroed stand-ins of that many problems
  int ths = 0;
  const int P_all = stack_size(p, &ths);
  const int P = P_all > 1 ? std::max(2, std::min<int>(P_all, (int)((1 << 23) / p->geo[0].mg))) : 1;
  float2* st_x = nullptr;
  float* st_y = nullptr;
  if (P > 1) {
    const Geo& g = p->geo[0];
    SR_CHECK(ensure_stack_bufs(p, 2 * (size_t)P * g.mg));
    SR_HIP(hipMalloc(&st_x, sizeof(float2) * g.n * P));
    SR_HIP(hipMalloc(&st_y, sizeof(float) * g.m * P));
    SR_HIP(hipMemsetAsync(st_x, 0, sizeof(float2) * g.n * P, p->stream));
    SR_HIP(hipMemsetAsync(st_y, 0, sizeof(float) * g.m * P, p->stream));
  }
  struct Standins {  // released once the timings are done
    sr_plan_s* p;
    float2* x;
    float* y;
    ~Standins() {
      if (x == nullptr && y == nullptr) return;
      (void)hipStreamSynchronize(p->stream);  // (a failure surfaces at the next call)
      if (x) (void)hipFree(x);
      if (y) (void)hipFree(y);
    }
  } standins{p, st_x, st_y};
  std::vector<std::string> done;
  for (const Geo& g : p->geo) {
    if (g.ndim != 2) continue;
    const std::string key = tune_key(g) + (P > 1 ? ":stack" + std::to_string(P) : std::string());
    if (std::find(done.begin(), done.end(), key) != done.end()) continue;
    done.push_back(key);
    if (p->tiles.count({g.M1, 1}) && p->tiles.count({g.M2, 0})) continue;  // decided by an earlier shape
    int cb = 0, rb = 0, tb = 0;
    if (!tune_cache_lookup(cache, key, &cb, &rb, &tb)) {
      int copt[16], ropt[16];
      const int nc = tile_options(g.M1, true, copt, 16);
      const int nr = tile_options(g.M2, false, ropt, 16);
      float best = 1e30f;
      bool best_whole_found = false;
      hipEvent_t e0, e1;
      SR_HIP(hipEventCreate(&e0));
      SR_HIP(hipEventCreate(&e1));
      float2* x = P > 1 ? st_x : p->bufC;
      const float* y = P > 1 ? st_y : (const float*)p->bufD;
      std::unique_ptr<StackScope> scope;
      if (P > 1) {
        scope.reset(new StackScope(p, P, ths));
        p->stk.add(x, g.n, sizeof(float2), (int)g.n);
        p->stk.add(y, g.m, sizeof(float), (int)g.m);
      }
      const char* tab_env = std::getenv("SR_PHASE_TABLE");
      const int tab_lo = tab_env ? std::atoi(tab_env) : 0;
      const int tab_hi = tab_env ? std::atoi(tab_env) : 1;
      for (int tab = tab_lo; tab <= tab_hi; ++tab)
      for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nr; ++j) {
          p->use_table = tab != 0;
          p->tiles[{g.M1, 1}] = copt[i];
          p->tiles[{g.M2, 0}] = ropt[j];
          // the steady-state iteration the solvers run (update fused with the next first pass)
          SR_CHECK(first_pass(p, g, x, 1.f, nullptr, 0));
          for (int w = 0; w < 3; ++w) SR_CHECK(gd_steady(p, g, y, x, 0.f, nullptr, false));
          float ms = 1e30f;  // best of three timed runs (one run is noisy at microsecond scale)
          for (int rep = 0; rep < 3; ++rep) {
            SR_HIP(hipEventRecord(e0, p->stream));
            for (int w = 0; w < 8; ++w) SR_CHECK(gd_steady(p, g, y, x, 0.f, nullptr, false));
            SR_HIP(hipEventRecord(e1, p->stream));
            SR_HIP(hipEventSynchronize(e1));
            float t = 0.f;
            SR_HIP(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t);
          }
          // a stack prefers tiles that hold whole problems in the passes that
          // sum per-problem partials (power iteration and loss traces stack too)
          const bool whole = P > 1 && stack_spectral_ok(p, g) && stack_trace_ok(p, g);
          if (whole && !best_whole_found) best = 1e30f;
          if ((whole || !best_whole_found) && ms < best) {
            best = ms;
            cb = copt[i];
            rb = ropt[j];
            tb = tab;
            best_whole_found = best_whole_found || whole;
          }
        }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      tune_cache_store(cache, key, cb, rb, tb);
    }
    p->tiles[{g.M1, 1}] = cb;
    p->tiles[{g.M2, 0}] = rb;
    p->use_table = tb != 0;
    const char* verbose = std::getenv("SR_TUNE_VERBOSE");
    if (verbose != nullptr && std::atoi(verbose) != 0)
      std::fprintf(stderr, "[srpr tune] %s: column tile %d, row tile %d, phase table %d\n", key.c_str(), cb, rb, tb);
  }
  return SR_OK;
}

// ------------------------------------------------- persistent (one launch)

// Tile width of the persistent kernels (SR_PERSIST_B overrides; 0 disables).
static int persist_b() {
  const char* e = std::getenv("SR_PERSIST_B");
  if (e != nullptr) return std::atoi(e);
  return 0;  // grid barriers cost more than kernel boundaries on this path; opt-in
}

static bool use_persistent(const sr_plan_s* p, const Geo& g) {
  if (p->schedule == SR_SCHED_LOOP || p->loss != SR_LOSS_L2) return false;  // built for the l2 epilogue
  if (g.ndim != 2 || g.M1 != g.M2 || g.L > (kMaxPersistPasses - 1) / 2) return false;
  return persistent_supported(g.M1, persist_b());
}

// Record one iteration's passes (with `record`) and run `iters` iterations of
// them in one cooperative launch.
template <class F>
static sr_status run_persistent(sr_plan_s* p, const Geo& g, int op, int iters, F&& record, float* loss_trace,
                                int npart0) {
  std::vector<PassRecord> rec;
  g_recording = &rec;
  sr_status st = record();
  g_recording = nullptr;
  SR_CHECK(st);
  if ((int)rec.size() > kMaxPersistPasses) return fail(SR_E_UNSUPPORTED, "too many passes for one launch");
  const int B = persist_b();
  PersistArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  int max_tiles = 1;
  pa.loss_pass = -1;
  for (size_t i = 0; i < rec.size(); ++i) {
    pa.pass[i] = rec[i].a;
    pa.kind[i] = rec[i].kind;
    pa.col[i] = pass_col(rec[i].k);
    max_tiles = std::max(max_tiles, (rec[i].a.ntr + B - 1) / B);
    if (rec[i].kind == PK_TURN_GD) pa.loss_pass = (int)i;
    if (rec[i].kind == PK_TURN_GD) pa.loss_nparts = (rec[i].a.ntr + B - 1) / B;
    if (rec[i].kind == PK_LAST_SPEC) pa.npart_iter = (rec[i].a.ntr + B - 1) / B;
  }
  if (max_tiles > p->part_cap) return fail(SR_E_UNSUPPORTED, "partial-sum buffer too small for the persistent tile");
  pa.npass = (int)rec.size();
  pa.iters = iters;
  pa.bar = p->sync;
  pa.err = (int*)(p->sync + 1);
  pa.part_base = p->part;
  pa.part_cap = p->part_cap;
  pa.npart0 = npart0;
  pa.loss_trace = loss_trace;
  hipError_t e = launch_persistent(g.M1, B, op, pa, max_tiles, p->stream);
  if (e != hipSuccess) return hip_fail(e, "persistent launch");
  return SR_OK;
}

// ------------------------------------------------------------ 1D (fused)

static Fused1DArgs args_1d(const sr_plan_s* p, const Geo& g, Fused1DArgs a) {
  a.n = g.N1;
  a.m = g.M1;
  a.L = g.L;
  a.off = g.o1;
  a.mw = g.W1;
  a.moff = g.c1;
  a.theta = p->theta_l(g, 1);
  a.tw = p->twiddles(g.M1, 1) ? p->twiddles(g.M1, 1) : p->twiddles(g.M1, 0);  // the 1D kernels' shape
  a.loss = p->loss;
  a.loss_eps = p->loss_eps;
  a.nf = p->sync + 2;
  return a;
}

// The 1D problems of one call, launched together: one workgroup per problem,
// one launch per grid length (a single problem launches on its own).
using Batch1D = std::vector<std::pair<int, Fused1DArgs>>;

static sr_status flush_1d(sr_plan_s* p, int op, Batch1D& items) {
  if (items.empty()) return SR_OK;
  if (items.size() == 1) {
    hipError_t e = launch_fused1d(items[0].first, op, items[0].second, p->stream);
    items.clear();
    return e == hipSuccess ? SR_OK : hip_fail(e, "fused 1D launch");
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const std::pair<int, Fused1DArgs>& a, const std::pair<int, Fused1DArgs>& b) { return a.first < b.first; });
  const size_t bytes = items.size() * sizeof(Fused1DArgs);
  if (p->f1_cap < items.size()) {
    if (p->f1_args) {
      // launches already queued may still read the old arguments
      if (hipError_t w = hipStreamSynchronize(p->stream); w != hipSuccess) return hip_fail(w, "stream wait");
      (void)hipFree(p->f1_args);
    }
    p->f1_args = nullptr;
    p->f1_cap = 0;
    hipError_t e = hipMalloc(&p->f1_args, bytes);
    if (e != hipSuccess) return fail(SR_E_NOMEM, "1D argument allocation failed");
    p->f1_cap = items.size();
  }
  p->f1_host.resize(bytes);  // kept alive by the plan while the upload is in flight
  for (size_t i = 0; i < items.size(); ++i)
    std::memcpy(p->f1_host.data() + i * sizeof(Fused1DArgs), &items[i].second, sizeof(Fused1DArgs));
  SR_HIP(hipMemcpyAsync(p->f1_args, p->f1_host.data(), bytes, hipMemcpyHostToDevice, p->stream));
  const Fused1DArgs* dev = (const Fused1DArgs*)p->f1_args;
  for (size_t lo = 0; lo < items.size();) {
    size_t hi = lo;
    while (hi < items.size() && items[hi].first == items[lo].first) ++hi;
    hipError_t e = launch_fused1d_batch(items[lo].first, op, dev + lo, (int)(hi - lo), p->stream);
    if (e != hipSuccess) return hip_fail(e, "fused 1D batch launch");
    lo = hi;
  }
  items.clear();
  return SR_OK;
}

// ====================================================================== ABI

// ------------------------------------------------ no-allocation GD scratch
// sr_gd_solve_noalloc keeps its two ping-pong grids in this file-scope device
// array instead of the plan's workspace, so that the call allocates nothing.
// Each GPU the library runs on holds its own copy until the process ends; its
// address on a device comes from hipGetSymbolAddress, taken once per device
// at plan creation with that device current (in host code the array's name
// is not a device address and is never used directly).  Every call on a GPU
// shares that GPU's array: calls that overlap on one GPU (two streams, two
// threads) race.  No part of it needs clearing: every pass reads only what an
// earlier pass of the same call wrote.
namespace {
constexpr size_t kScratchBytes = size_t(16) << 20;  // two grids of up to 2^20 points
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Once per device, with that device current: the device address of `scratch`.
sr_status scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(SR_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] != nullptr) return SR_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (ptr == nullptr) return fail(SR_E_HIP, "no device address for the scratch array");
  g_scratch_ptr[device] = ptr;
  return SR_OK;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}
}  // namespace

extern "C" {

const char* sr_status_string(sr_status s) {
  switch (s) {
    case SR_OK: return "ok";
    case SR_E_ARG: return "invalid argument";
    case SR_E_SHAPE: return "inconsistent shape";
    case SR_E_UNSUPPORTED: return "unsupported configuration";
    case SR_E_HIP: return "HIP runtime error";
    case SR_E_NONFINITE: return "non-finite value";
    case SR_E_STATE: return "call not valid for this plan";
    case SR_E_NOMEM: return "out of device memory";
    default: return "unknown status";
  }
}

const char* sr_last_error(void) { return g_last_error.c_str(); }

sr_status sr_plan_create(sr_plan* out, const sr_problem* probs, int32_t nprob, const float* theta_host,
                         int64_t theta_len, const void* dense_A, void* hip_stream) {
  g_last_error.clear();
  if (out == nullptr) return fail(SR_E_ARG, "out is NULL");
  *out = nullptr;
  if (probs == nullptr || nprob <= 0) return fail(SR_E_ARG, "need at least one problem");
  const int kind = probs[0].kind;
  if (kind != SR_STRUCTURED && kind != SR_DENSE) return fail(SR_E_ARG, "unknown problem kind");
  std::vector<Geo> geo(nprob);
  for (int i = 0; i < nprob; ++i) {
    const sr_problem& q = probs[i];
    Geo& g = geo[i];
    if (q.kind != kind) return fail(SR_E_ARG, "all problems of a plan must have the same kind");
    if (q.ndim != 1 && q.ndim != 2) return fail(SR_E_ARG, "ndim must be 1 or 2");
    g.ndim = q.ndim;
    g.N1 = q.n[0];
    g.W1 = q.m[0];
    g.N2 = q.ndim == 2 ? q.n[1] : 1;
    g.W2 = q.ndim == 2 ? q.m[1] : 1;
    if (g.N1 < 1 || g.N2 < 1) return fail(SR_E_SHAPE, "signal sizes must be positive");
    if (g.W1 < 1 || g.W2 < 1) return fail(SR_E_SHAPE, "measurement sizes must be positive");
    // transform grid: zero padding for M > N (U), centred trimming for M < N (S)
    g.M1 = kind == SR_STRUCTURED ? std::max(g.N1, g.W1) : g.W1;
    g.M2 = kind == SR_STRUCTURED ? std::max(g.N2, g.W2) : g.W2;
    g.o1 = (g.M1 - g.N1) / 2;
    g.o2 = (g.M2 - g.N2) / 2;
    g.c1 = (g.M1 - g.W1) / 2;
    g.c2 = (g.M2 - g.W2) / 2;
    g.n = (int64_t)g.N1 * g.N2;
    g.m = (int64_t)g.W1 * g.W2;
    g.mg = (int64_t)g.M1 * g.M2;
    g.L = q.layers;
    g.th_off = q.theta_offset;
    if (kind == SR_STRUCTURED) {
      if (g.L < 1 || g.L > 16) return fail(SR_E_ARG, "layers must be in [1, 16]");
      if (g.th_off < 0 || g.th_off + (int64_t)g.L * g.mg > theta_len)
        return fail(SR_E_SHAPE, "problem " + std::to_string(i) + ": theta block out of range");
      if (q.ndim == 1) {
        if (!supported_len_1d(g.M1)) return fail(SR_E_UNSUPPORTED, "unsupported 1D length " + std::to_string(g.M1));
        if ((int64_t)g.L * g.M1 > kFused1DPhaseSlots) return fail(SR_E_UNSUPPORTED, "1D problems need L*m <= 4096");
      } else {
        if (!supported_len_2d(g.M1) || !supported_len_2d(g.M2))
          return fail(SR_E_UNSUPPORTED, "unsupported 2D grid " + std::to_string(g.M1) + "x" + std::to_string(g.M2));
      }
    } else {
      if (i > 0 && (g.n != geo[0].n || g.m != geo[0].m))
        return fail(SR_E_SHAPE, "dense problems of one plan share one matrix and must have one shape");
      if (g.n % 2 != 0) return fail(SR_E_UNSUPPORTED, "dense problems need an even signal length");
      if (g.m > (1 << 30) / 2 || g.n > (1 << 28)) return fail(SR_E_UNSUPPORTED, "dense problem too large");
    }
  }
  if (kind == SR_STRUCTURED) {
    if (theta_host == nullptr || theta_len <= 0) return fail(SR_E_ARG, "theta is required for structured plans");
    if (dense_A != nullptr) return fail(SR_E_ARG, "dense_A must be NULL for structured plans");
  } else {
    if (dense_A == nullptr) return fail(SR_E_ARG, "dense_A is required for dense plans");
    if (theta_host != nullptr || theta_len != 0) return fail(SR_E_ARG, "theta must be NULL for dense plans");
  }

  int device = 0;
  SR_HIP(hipGetDevice(&device));
  if (kind == SR_STRUCTURED) SR_CHECK(scratch_setup(device));
  sr_plan_s* p = new (std::nothrow) sr_plan_s();
  if (p == nullptr) return fail(SR_E_NOMEM, "host allocation failed");
  p->device = device;
  p->geo = geo;
  p->kind = kind;
  p->stream = (hipStream_t)hip_stream;
  p->theta_len = theta_len;
  p->dense_A = (const float2*)dense_A;
  sr_status st = p->init(theta_host);
  if (st == SR_OK && kind == SR_STRUCTURED) st = tune_plan(p);
  if (st == SR_OK && kind == SR_DENSE) st = dense_lib_setup(p);
  if (st != SR_OK) {
    delete p;
    return st;
  }
  *out = p;
  return SR_OK;
}

sr_status sr_plan_set_theta(sr_plan p, const float* theta_dev, int64_t theta_len) {
  if (p == nullptr || theta_dev == nullptr) return fail(SR_E_ARG, "NULL argument");
  if (p->kind != SR_STRUCTURED) return fail(SR_E_STATE, "dense plans have no phases");
  if (theta_len != p->theta_len) return fail(SR_E_SHAPE, "theta length differs from the plan's");
  SR_HIP(hipMemcpyAsync(p->theta, theta_dev, sizeof(float) * theta_len, hipMemcpyDeviceToDevice, p->stream));
  return fill_phase_table(p);
}

sr_status sr_plan_workspace_size(sr_plan p, size_t* bytes) {
  if (p == nullptr || bytes == nullptr) return fail(SR_E_ARG, "NULL argument");
  *bytes = p->ws_bytes;
  return SR_OK;
}

sr_status sr_plan_set_workspace(sr_plan p, void* dev_ptr, size_t bytes) {
  if (p == nullptr || dev_ptr == nullptr) return fail(SR_E_ARG, "NULL argument");
  if (bytes < p->ws_bytes) return fail(SR_E_ARG, "workspace smaller than sr_plan_workspace_size");
  if (((uintptr_t)dev_ptr & 255) != 0) return fail(SR_E_ARG, "workspace must be 256-byte aligned");
  if (dev_ptr == p->ws) return SR_OK;
  const uintptr_t lo = (uintptr_t)dev_ptr, hi = lo + p->ws_bytes, olo = (uintptr_t)p->ws, ohi = olo + p->ws_bytes;
  if (lo < ohi && olo < hi) return fail(SR_E_ARG, "workspace overlaps the current one");
  // queued work still uses the old workspace: finish it, move the contents
  SR_HIP(hipStreamSynchronize(p->stream));
  if (p->aux_stream) SR_HIP(hipStreamSynchronize(p->aux_stream));
  SR_HIP(hipMemcpyAsync(dev_ptr, p->ws, p->ws_bytes, hipMemcpyDeviceToDevice, p->stream));
  SR_HIP(hipStreamSynchronize(p->stream));
  const ptrdiff_t d = (char*)dev_ptr - (char*)p->ws;
  auto mv = [d](auto*& q) {
    if (q != nullptr) q = (std::remove_reference_t<decltype(q)>)((char*)q + d);
  };
  mv(p->theta);
  mv(p->eph);
  mv(p->twbuf);
  mv(p->bufA);
  mv(p->bufB);
  mv(p->bufC);
  mv(p->bufD);
  mv(p->part);
  mv(p->ysum);
  mv(p->fscratch);
  mv(p->sync);
  mv(p->red_ws);
  mv(p->dsplit);
  for (auto& t : p->tw) mv(t.second);
  // recorded schedules and captured graphs hold the old addresses
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.second);
  p->graphs.clear();
  if (p->batch) destroy_batch_state(p->batch);
  p->batch = nullptr;
  if (p->spec_batch) destroy_spec_batch_state(p->spec_batch);
  p->spec_batch = nullptr;
  if (p->op_batch) destroy_op_batch_state(p->op_batch);
  p->op_batch = nullptr;
  if (p->vjp_batch) destroy_vjp_batch_state(p->vjp_batch);
  p->vjp_batch = nullptr;
  if (p->ws_owned) SR_HIP(hipFree(p->ws));
  p->ws = dev_ptr;
  p->ws_owned = false;
  return SR_OK;
}

sr_status sr_plan_offsets(sr_plan p, int64_t* x_off, int64_t* y_off) {
  if (p == nullptr) return fail(SR_E_ARG, "NULL plan");
  const size_t np = p->geo.size();
  for (size_t i = 0; i <= np; ++i) {
    if (x_off) x_off[i] = p->xoff[i];
    if (y_off) y_off[i] = p->yoff[i];
  }
  return SR_OK;
}

sr_status sr_plan_set_schedule(sr_plan p, int32_t schedule) {
  if (p == nullptr) return fail(SR_E_ARG, "NULL plan");
  if (schedule < SR_SCHED_AUTO || schedule > SR_SCHED_BATCHED) return fail(SR_E_ARG, "unknown schedule");
  p->schedule = schedule;
  return SR_OK;
}

sr_status sr_plan_set_loss(sr_plan p, int32_t loss, float eps) {
  if (p == nullptr) return fail(SR_E_ARG, "NULL plan");
  if (loss != SR_LOSS_L2 && loss != SR_LOSS_POISSON) return fail(SR_E_ARG, "unknown loss");
  if (loss == SR_LOSS_POISSON && !(std::isfinite(eps) && eps > 0.f))
    return fail(SR_E_ARG, "the Poisson loss needs a finite eps > 0");
  p->loss = loss;
  p->loss_eps = loss == SR_LOSS_POISSON ? eps : 0.f;
  return SR_OK;
}

sr_status sr_plan_sync(sr_plan p) {
  if (p == nullptr) return fail(SR_E_ARG, "NULL plan");
  SR_HIP(hipStreamSynchronize(p->stream));
  // [1] barrier time-out, [2] non-finite result; both cleared once reported
  unsigned flags[2] = {0, 0};
  SR_HIP(hipMemcpy(flags, p->sync + 1, sizeof(flags), hipMemcpyDeviceToHost));
  if (flags[0] != 0 || flags[1] != 0) {
    const unsigned zero[2] = {0, 0};
    SR_HIP(hipMemcpy(p->sync + 1, zero, sizeof(zero), hipMemcpyHostToDevice));
  }
  if (flags[0] != 0)
    return fail(SR_E_HIP, "a grid-wide barrier wait exceeded its bound; results of that solve are invalid");
  if (flags[1] != 0)
    return fail(SR_E_NONFINITE,
                "a solve since the last sync produced a NaN or Inf (iterate, spectral estimate or loss-trace entry)");
  return SR_OK;
}

sr_status sr_plan_destroy(sr_plan p) {
  if (p == nullptr) return SR_OK;
  (void)hipStreamSynchronize(p->stream);  // the plan's work ends before its memory goes
  delete p;
  return SR_OK;
}

// A x for a stack of problems (stack_size > 1): problem 0's schedule, each
// pass launched once for all of them.
static sr_status forward_stacked(sr_plan_s* p, int P, int ths, const float2* x, float2* z, float* y) {
  const Geo& g = p->geo[0];
  SR_CHECK(ensure_stack_bufs(p, 2 * (size_t)P * g.mg));
  StackScope sc(p, P, ths);
  p->stk.add(x, g.n, sizeof(float2), (int)g.n);
  if (z) p->stk.add(z, g.m, sizeof(float2), (int)g.m);
  if (y) p->stk.add(y, g.m, sizeof(float), (int)g.m);
  return forward_2d(p, g, x, z, y);
}

static sr_status adjoint_stacked(sr_plan_s* p, int P, int ths, const float2* r, float2* x) {
  const Geo& g = p->geo[0];
  SR_CHECK(ensure_stack_bufs(p, 2 * (size_t)P * g.mg));
  StackScope sc(p, P, ths);
  p->stk.add(r, g.m, sizeof(float2), (int)g.m);
  p->stk.add(x, g.n, sizeof(float2), (int)g.n);
  return adjoint_2d(p, g, r, x);
}

// A batched plan applies A (A^H) to its 2D problems by level launches; the
// rest (1D problems, lengths the level kernel lacks) stay with the loop.
static sr_status batched_op_part(sr_plan_s* p, bool adjoint, const float2* in, float2* out, float* y,
                                 std::vector<char>& done) {
  const bool want_batched = p->schedule == SR_SCHED_BATCHED || (p->schedule == SR_SCHED_AUTO && p->geo.size() >= 8);
  if (!want_batched) return SR_OK;
  std::vector<int> lvl;
  for (size_t i = 0; i < p->geo.size(); ++i)
    if (batch_level_capable(p->geo[i])) lvl.push_back((int)i);
  if (lvl.size() < 2) return SR_OK;
  SR_CHECK(batched_operator(p, lvl, adjoint, in, out, y));
  for (int i : lvl) done[i] = 1;
  return SR_OK;
}

sr_status sr_forward(sr_plan p, const void* x, void* z, float* y) {
  if (p == nullptr || x == nullptr) return fail(SR_E_ARG, "NULL argument");
  if (z == nullptr && y == nullptr) return fail(SR_E_ARG, "need z or y");
  const float2* xs = (const float2*)x;
  float2* zs = (float2*)z;
  if (p->kind == SR_DENSE) return dense_forward(p, xs, zs, y);
  int ths = 0;
  const int P = stack_size(p, &ths);
  if (P > 1) return forward_stacked(p, P, ths, xs, zs, y);
  std::vector<char> done(p->geo.size(), 0);
  SR_CHECK(batched_op_part(p, false, xs, zs, y, done));
  Batch1D b1;
  for (size_t i = 0; i < p->geo.size(); ++i) {
    if (done[i]) continue;
    const Geo& g = p->geo[i];
    const float2* xi = xs + p->xoff[i];
    float2* zi = zs ? zs + p->yoff[i] : nullptr;
    float* yi = y ? y + p->yoff[i] : nullptr;
    if (g.ndim == 1) {
      Fused1DArgs a{};
      a.x_in = xi;
      a.z_out = zi;
      a.y_out = yi;
      b1.push_back({g.M1, args_1d(p, g, a)});
    } else {
      SR_CHECK(forward_2d(p, g, xi, zi, yi));
    }
  }
  return flush_1d(p, F1_FORWARD, b1);
}

sr_status sr_adjoint(sr_plan p, const void* r, void* x_out) {
  if (p == nullptr || r == nullptr || x_out == nullptr) return fail(SR_E_ARG, "NULL argument");
  const float2* rs = (const float2*)r;
  float2* xs = (float2*)x_out;
  if (p->kind == SR_DENSE) return dense_adjoint(p, rs, xs);
  int ths = 0;
  const int P = stack_size(p, &ths);
  if (P > 1) return adjoint_stacked(p, P, ths, rs, xs);
  std::vector<char> done(p->geo.size(), 0);
  SR_CHECK(batched_op_part(p, true, rs, xs, nullptr, done));
  Batch1D b1;
  for (size_t i = 0; i < p->geo.size(); ++i) {
    if (done[i]) continue;
    const Geo& g = p->geo[i];
    if (g.ndim == 1) {
      Fused1DArgs a{};
      a.r_in = rs + p->yoff[i];
      a.x_out = xs + p->xoff[i];
      b1.push_back({g.M1, args_1d(p, g, a)});
    } else {
      SR_CHECK(adjoint_2d(p, g, rs + p->yoff[i], xs + p->xoff[i]));
    }
  }
  return flush_1d(p, F1_ADJOINT, b1);
}

// Whether a stack's turnaround pass keeps each tile inside one problem (its
// loss partials are then each problem's own).
static bool stack_trace_ok(const sr_plan_s* p, const Geo& g) {
  const int k = g.L + 1;
  const int ntr = (k == 2) ? g.M1 : (pass_col(k) ? g.M2 : g.M1);
  const int bt = tile_other(p, pass_len(g, k), pass_col(k)) & (kSingleBuffer - 1);
  return ntr % bt == 0;
}

// GD on a stack: problem 0's schedule, each pass launched once for all
// problems, each with its own step; with a loss trace, each problem's loss
// partials (whole problems per turnaround tile) reduced in one launch.
static sr_status gd_stacked(sr_plan_s* p, int P, int ths, const float* y, float2* x, int iters,
                            const float* eta_host, float* loss_trace) {
  const Geo& g = p->geo[0];
  SR_CHECK(ensure_stack_bufs(p, 2 * (size_t)P * g.mg));
  const int nparts = turn_groups(p, g);
  if (loss_trace != nullptr) SR_CHECK(ensure_stack_parts(p, (size_t)P * nparts));
  if (p->stk_steps_cap < P) {
    if (p->stk_steps) {
      SR_HIP(hipStreamSynchronize(p->stream));  // queued work may still read the old array
      SR_HIP(hipFree(p->stk_steps));
      p->stk_steps = nullptr;
      p->stk_steps_cap = 0;
    }
    if (hipMalloc(&p->stk_steps, sizeof(float) * P) != hipSuccess) return fail(SR_E_NOMEM, "step array allocation failed");
    p->stk_steps_cap = P;
  }
  std::vector<float> steps(P);
  for (int i = 0; i < P; ++i) steps[i] = eta_host[i] / (float)p->geo[i].m;
  SR_CHECK(put_floats(p, p->stk_steps, steps.data(), P));
  StackScope sc(p, P, ths);
  p->stk.steps = p->stk_steps;
  p->stk.add(x, g.n, sizeof(float2), (int)g.n);
  p->stk.add(y, g.m, sizeof(float), (int)g.m);
  const float step = steps[0];  // (unused by the stacked update, which reads the array)
  SR_CHECK(first_pass(p, g, x, 1.f, nullptr, 0));
  int it = 0;
  if (loss_trace != nullptr) {
    for (; it < iters; ++it) {
      SR_CHECK(gd_steady(p, g, y, x, step, p->stk_part, it == iters - 1));
      SR_CHECK(reduce_partials(p, p->stk_part, nparts, loss_trace + it, P, iters));
    }
    return SR_OK;
  }
  if (graphs_enabled(p) && iters - 1 >= kGraphChunk) {
    const std::string key = "gdstack:" + std::to_string(P) + ":" + ptr_key(y) + ":" + ptr_key(x) + ":" +
                            ptr_key(p->stk_buf) + ":" + ptr_key(p->stk_steps);
    for (; it + kGraphChunk <= iters - 1; it += kGraphChunk)
      SR_CHECK(launch_captured(p, key, [&]() -> sr_status {
        for (int c = 0; c < kGraphChunk; ++c) SR_CHECK(gd_steady(p, g, y, x, step, nullptr, false));
        return SR_OK;
      }));
    const int rest = iters - 1 - it;  // the steady iterations short of a chunk, as one graph of their own
    if (rest >= kGraphTail) {
      SR_CHECK(launch_captured(p, key + ":" + std::to_string(rest), [&]() -> sr_status {
        for (int c = 0; c < rest; ++c) SR_CHECK(gd_steady(p, g, y, x, step, nullptr, false));
        return SR_OK;
      }));
      it += rest;
    }
  }
  for (; it < iters; ++it) SR_CHECK(gd_steady(p, g, y, x, step, nullptr, it == iters - 1));
  return SR_OK;
}

sr_status sr_gd_solve(sr_plan p, const float* y, void* x_inout, int32_t iters, const float* eta_host,
                      float* loss_trace) {
  if (p == nullptr || y == nullptr || x_inout == nullptr || eta_host == nullptr)
    return fail(SR_E_ARG, "NULL argument");
  if (iters < 0) return fail(SR_E_ARG, "iters must be >= 0");
  for (size_t i = 0; i < p->geo.size(); ++i)
    if (!std::isfinite(eta_host[i])) return fail(SR_E_NONFINITE, "step size is not finite");
  if (iters == 0) return SR_OK;
  float2* xs = (float2*)x_inout;
  if (p->kind == SR_DENSE) return dense_gd(p, y, xs, iters, eta_host, loss_trace);
  // a uniform plan runs as one stack (unless the level launches or the
  // LDS-resident solver are asked for)
  if (p->schedule == SR_SCHED_AUTO && !fused2d_enabled(false)) {
    int ths = 0;
    const int P = stack_size(p, &ths);
    if (P > 1 && (loss_trace == nullptr || stack_trace_ok(p, p->geo[0])))
      return gd_stacked(p, P, ths, y, xs, iters, eta_host, loss_trace);
  }
  const bool want_batched = p->schedule == SR_SCHED_BATCHED || (p->schedule == SR_SCHED_AUTO && p->geo.size() >= 8);
  if (want_batched && batched_supported(p) && (loss_trace == nullptr || !batched_any_resident(p)))
    return batched_gd(p, y, xs, iters, eta_host, loss_trace);
  Batch1D b1;
  for (size_t i = 0; i < p->geo.size(); ++i) {
    const Geo& g = p->geo[i];
    const float* yi = y + p->yoff[i];
    float2* xi = xs + p->xoff[i];
    const float step = eta_host[i] / (float)g.m;
    float* lt = loss_trace ? loss_trace + (int64_t)i * iters : nullptr;
    if (g.ndim == 1) {
      Fused1DArgs a{};
      a.x_out = xi;
      a.y = yi;
      a.iters = iters;
      a.step = step;
      a.loss_trace = lt;
      b1.push_back({g.M1, args_1d(p, g, a)});
      continue;
    }
    if (use_persistent(p, g)) {
      SR_CHECK(run_persistent(
          p, g, PO_GD, iters, [&]() { return gd_iter_2d(p, g, yi, xi, step, lt ? p->part : nullptr); }, lt, 0));
      continue;
    }
    const int nparts = turn_groups(p, g);
    SR_CHECK(first_pass(p, g, xi, 1.f, nullptr, 0));
    int it = 0;
    if (lt == nullptr && graphs_enabled(p) && iters - 1 >= kGraphChunk) {
      const std::string key = "gd:" + std::to_string(i) + ":" + ptr_key(yi) + ":" + ptr_key(xi) + ":" + float_key(step);
      for (; it + kGraphChunk <= iters - 1; it += kGraphChunk)
        SR_CHECK(launch_captured(p, key, [&]() -> sr_status {
          for (int c = 0; c < kGraphChunk; ++c) SR_CHECK(gd_steady(p, g, yi, xi, step, nullptr, false));
          return SR_OK;
        }));
      // the steady iterations short of a chunk, as one graph of their own
      // (direct launches cost about 1.4 us more per iteration here)
      const int rest = iters - 1 - it;
      if (rest >= kGraphTail) {
        SR_CHECK(launch_captured(p, key + ":" + std::to_string(rest), [&]() -> sr_status {
          for (int c = 0; c < rest; ++c) SR_CHECK(gd_steady(p, g, yi, xi, step, nullptr, false));
          return SR_OK;
        }));
        it += rest;
      }
    }
    for (; it < iters; ++it) {
      SR_CHECK(gd_steady(p, g, yi, xi, step, lt ? p->part : nullptr, it == iters - 1));
      if (lt) SR_CHECK(reduce_partials(p, p->part, nparts, lt + it));
    }
  }
  return flush_1d(p, F1_GD, b1);
}

// GD with the ping-pong grids in the device's scratch array: the passes of
// sr_gd_solve's per-problem schedule (first pass, then steady iterations with
// the update fused into the next first pass), launched directly (no graphs,
// whose instantiation allocates), problem after problem on the plan's stream.
sr_status sr_gd_solve_noalloc(sr_plan p, const float* y, void* x_inout, int32_t iters, const float* eta_host) {
  if (p == nullptr || y == nullptr || x_inout == nullptr || eta_host == nullptr)
    return fail(SR_E_ARG, "NULL argument");
  if (iters < 0) return fail(SR_E_ARG, "iters must be >= 0");
  if (p->kind != SR_STRUCTURED) return fail(SR_E_STATE, "the no-allocation GD takes structured plans only");
  for (size_t i = 0; i < p->geo.size(); ++i) {
    const Geo& g = p->geo[i];
    if (!std::isfinite(eta_host[i])) return fail(SR_E_NONFINITE, "step size is not finite");
    if (g.ndim != 2)
      return fail(SR_E_UNSUPPORTED, "the no-allocation GD takes 2D problems only (1D solves need no scratch: "
                                    "sr_gd_solve runs them in LDS)");
    const size_t need = 2 * (size_t)g.mg * sizeof(float2);
    if (need > kScratchBytes)
      return fail(SR_E_ARG, "problem " + std::to_string(i) + ": a " + std::to_string(g.M1) + "x" +
                                std::to_string(g.M2) + " grid needs " + std::to_string(need) +
                                " bytes of scratch; the no-allocation GD holds " + std::to_string(kScratchBytes) +
                                " (grids up to 2^20 points)");
  }
  float2* const ptr = (float2*)scratch_ptr(p->device);
  if (ptr == nullptr) return fail(SR_E_STATE, "no scratch address for the plan's device");
  if (iters == 0) return SR_OK;
  float2* xs = (float2*)x_inout;
  float2* const a0 = p->bufA;
  float2* const b0 = p->bufB;
  sr_status st = SR_OK;
  for (size_t i = 0; i < p->geo.size() && st == SR_OK; ++i) {
    const Geo& g = p->geo[i];
    const float* yi = y + p->yoff[i];
    float2* xi = xs + p->xoff[i];
    const float step = eta_host[i] / (float)g.m;
    p->bufA = ptr;
    p->bufB = ptr + g.mg;
    st = first_pass(p, g, xi, 1.f, nullptr, 0);
    for (int it = 0; it < iters && st == SR_OK; ++it) st = gd_steady(p, g, yi, xi, step, nullptr, it == iters - 1);
  }
  p->bufA = a0;
  p->bufB = b0;
  return st;
}

// Whether a stack's spectral passes keep each tile inside one problem (the
// passes that read and write per-problem norm partials need it).
static bool stack_spectral_ok(const sr_plan_s* p, const Geo& g) {
  const int bt = tile_other(p, g.M1, true) & (kSingleBuffer - 1);
  return g.N2 % bt == 0;
}

// Power iteration on a stack: problem 0's schedule, each pass launched once
// for all problems; each problem keeps its own sum(y) and norm partials.
static sr_status spectral_stacked(sr_plan_s* p, int P, int ths, const float* y, const float2* v0, int iters,
                                  float lambda, float2* x) {
  const Geo& g = p->geo[0];
  const float inv_mc = (float)((double)g.mg / (double)g.m);
  const int nq = last_pass_groups(p, g);
  const size_t pstride = (size_t)P * (size_t)std::max(nq, 1);
  SR_CHECK(ensure_stack_bufs(p, 2 * (size_t)P * g.mg));
  SR_CHECK(ensure_stack_parts(p, 2 * pstride));
  float* parts[2] = {p->stk_part, p->stk_part + pstride};
  // sum(y) and the start vector's squared norm, per problem (one partial each)
  SR_HIP(hipMemcpyAsync(x, v0, sizeof(float2) * g.n * P, hipMemcpyDeviceToDevice, p->stream));
  SR_CHECK(sum_floats(p, y, g.m, p->ysum, P));
  SR_CHECK(norm2_partial(p, x, g.n, parts[0], P));
  int npart = 1;
  {
    StackScope sc(p, P, ths);
    p->stk.add(x, g.n, sizeof(float2), (int)g.n);
    p->stk.add(y, g.m, sizeof(float), (int)g.m);
    int it = 0;
    if (iters > 0) SR_CHECK(first_pass(p, g, x, 1.f, nullptr, 0));
    if (iters > 1) {
      SR_CHECK(spec_steady(p, g, y, x, lambda, inv_mc, p->ysum, parts[0], npart, parts[1], false));
      npart = nq;
      it = 1;
    }
    if (graphs_enabled(p) && iters - 1 - it >= kGraphChunk) {
      const std::string key = "specstack:" + std::to_string(P) + ":" + ptr_key(y) + ":" + ptr_key(x) + ":" +
                              ptr_key(p->stk_buf) + ":" + ptr_key(p->stk_part) + ":" + float_key(lambda);
      for (; it + kGraphChunk <= iters - 1; it += kGraphChunk)
        SR_CHECK(launch_captured(p, key, [&]() -> sr_status {
          for (int c = 0; c < kGraphChunk; ++c) {
            const int q = it + c;
            SR_CHECK(spec_steady(p, g, y, x, lambda, inv_mc, p->ysum, parts[q & 1], nq, parts[(q + 1) & 1], false));
          }
          return SR_OK;
        }));
    }
    for (; it < iters; ++it) {
      SR_CHECK(spec_steady(p, g, y, x, lambda, inv_mc, p->ysum, parts[it & 1], npart, parts[(it + 1) & 1],
                           it == iters - 1));
      npart = nq;
    }
  }
  // x0 = sqrt(sum(y)/(m c)) u / ||u||, per problem
  return final_scale(p, x, g.n, parts[iters & 1], npart, p->ysum, inv_mc, P);
}

sr_status sr_spectral_init(sr_plan p, const float* y, const void* v0, int32_t iters, float lambda, void* x0_out) {
  if (p == nullptr || y == nullptr || v0 == nullptr || x0_out == nullptr) return fail(SR_E_ARG, "NULL argument");
  if (iters < 0) return fail(SR_E_ARG, "iters must be >= 0");
  if (!(lambda < 0.f) || !std::isfinite(lambda)) return fail(SR_E_ARG, "lambda must be finite and negative");
  if (v0 == x0_out) return fail(SR_E_ARG, "x0_out must not alias v0");
  const float2* vs = (const float2*)v0;
  float2* xs = (float2*)x0_out;
  if (p->kind == SR_DENSE) return dense_spectral(p, y, vs, iters, lambda, xs);
  // a uniform plan runs as one stack (unless the LDS-resident solver is
  // asked for by name, or the level launches are)
  if (p->schedule == SR_SCHED_AUTO && !fused2d_enabled(false)) {
    int ths = 0;
    const int P = stack_size(p, &ths);
    if (P > 1 && stack_spectral_ok(p, p->geo[0])) return spectral_stacked(p, P, ths, y, vs, iters, lambda, xs);
  }
  // batched plans: with SR_LDS_RESIDENT=1, problems whose grid fits one
  // workgroup's LDS run their whole solve in the LDS-resident solver, beside
  // the level launches of the others
  const bool want_batched = p->schedule == SR_SCHED_BATCHED || (p->schedule == SR_SCHED_AUTO && p->geo.size() >= 8);
  std::vector<char> resident(p->geo.size(), 0);
  std::vector<int> small;
  if (want_batched && p->geo.size() >= 2)
    for (size_t i = 0; i < p->geo.size(); ++i)
      if (fused2d_enabled(false) && fused2d_supported(p->geo[i])) {
        resident[i] = 1;
        small.push_back((int)i);
      }
  const bool forked = !small.empty() && small.size() < p->geo.size();
  if (!small.empty()) {
    hipStream_t s2 = p->stream;
    if (forked) {
      SR_CHECK(aux_fork(p));
      s2 = p->aux_stream;
    }
    SR_CHECK(fused2d_spectral(p, small, y, vs, iters, lambda, xs, s2));
  }
  // the other 2D problems of a batched plan: one launch per pass level
  if (want_batched) {
    std::vector<int> lvl;
    for (size_t i = 0; i < p->geo.size(); ++i)
      if (!resident[i] && batch_level_capable(p->geo[i])) lvl.push_back((int)i);
    if (lvl.size() >= 2) {
      SR_CHECK(batched_spectral(p, lvl, y, vs, iters, lambda, xs));
      for (int i : lvl) resident[i] = 1;  // done
    }
  }
  Batch1D b1;
  for (size_t i = 0; i < p->geo.size(); ++i) {
    if (resident[i]) continue;
    const Geo& g = p->geo[i];
    const float* yi = y + p->yoff[i];
    const float2* vi = vs + p->xoff[i];
    float2* xi = xs + p->xoff[i];
    const float inv_mc = (float)((double)g.mg / (double)g.m);  // structured: c = 1/(grid size)
    if (g.ndim == 1) {
      Fused1DArgs a{};
      a.x_in = vi;
      a.x_out = xi;
      a.y = yi;
      a.iters = iters;
      a.step = inv_mc;
      a.lam = lambda;
      b1.push_back({g.M1, args_1d(p, g, a)});
      continue;
    }
    // sum(y), then u_0 = v0 with its squared-norm partial
    SR_CHECK(sum_floats(p, yi, g.m, p->ysum));
    SR_HIP(hipMemcpyAsync(xi, vi, sizeof(float2) * g.n, hipMemcpyDeviceToDevice, p->stream));
    float* parts[2] = {p->part, p->part + p->part_cap};
    SR_CHECK(norm2_partial(p, xi, g.n, parts[0]));
    int npart = 1;
    if (use_persistent(p, g) && iters > 0) {
      SR_CHECK(run_persistent(
          p, g, PO_SPEC, iters,
          [&]() { return spec_iter_2d(p, g, yi, xi, lambda, inv_mc, p->ysum, parts[0], 1, parts[1]); }, nullptr, 1));
      const int B = persist_b();
      npart = (g.N2 + B - 1) / B;
    } else {
      const int nq = last_pass_groups(p, g);
      int it = 0;
      if (iters > 0) SR_CHECK(first_pass(p, g, xi, 1.f, nullptr, 0));
      if (iters > 1) {  // the first iteration reads the start vector's single partial
        SR_CHECK(spec_steady(p, g, yi, xi, lambda, inv_mc, p->ysum, parts[0], npart, parts[1], false));
        npart = nq;
        it = 1;
      }
      if (graphs_enabled(p) && iters - 1 - it >= kGraphChunk) {
        // chunks start at odd iterations, so every chunk has the same partial-buffer parity
        const std::string key = "spec:" + std::to_string(i) + ":" + ptr_key(yi) + ":" + ptr_key(xi) + ":" +
                                float_key(lambda);
        for (; it + kGraphChunk <= iters - 1; it += kGraphChunk)
          SR_CHECK(launch_captured(p, key, [&]() -> sr_status {
            for (int c = 0; c < kGraphChunk; ++c) {
              const int q = it + c;
              SR_CHECK(spec_steady(p, g, yi, xi, lambda, inv_mc, p->ysum, parts[q & 1], nq, parts[(q + 1) & 1],
                                   false));
            }
            return SR_OK;
          }));
        // the remainder short of a chunk (it starts on an odd iteration too)
        const int rest = iters - 1 - it;
        if (rest >= kGraphTail) {
          SR_CHECK(launch_captured(p, key + ":" + std::to_string(rest), [&]() -> sr_status {
            for (int c = 0; c < rest; ++c) {
              const int q = it + c;
              SR_CHECK(spec_steady(p, g, yi, xi, lambda, inv_mc, p->ysum, parts[q & 1], nq, parts[(q + 1) & 1],
                                   false));
            }
            return SR_OK;
          }));
          it += rest;
        }
      }
      for (; it < iters; ++it) {
        SR_CHECK(spec_steady(p, g, yi, xi, lambda, inv_mc, p->ysum, parts[it & 1], npart, parts[(it + 1) & 1],
                             it == iters - 1));
        npart = nq;
      }
    }
    // x0 = sqrt(sum(y)/(m c)) u / ||u||
    SR_CHECK(final_scale(p, xi, g.n, parts[iters & 1], npart, p->ysum, inv_mc));
  }
  SR_CHECK(flush_1d(p, F1_SPECTRAL, b1));
  if (forked) SR_CHECK(aux_join(p));
  return SR_OK;
}

sr_status sr_forward_vjp(sr_plan p, const void* x, const void* gz, void* gx_out, float* gtheta_accum) {
  if (p == nullptr || x == nullptr || gz == nullptr || gtheta_accum == nullptr) return fail(SR_E_ARG, "NULL argument");
  if (p->kind != SR_STRUCTURED) return fail(SR_E_STATE, "VJPs need a structured plan");
  return vjp_forward(p, (const float2*)x, (const float2*)gz, (float2*)gx_out, gtheta_accum);
}

sr_status sr_adjoint_vjp(sr_plan p, const void* r, const void* gv, void* gr_out, float* gtheta_accum) {
  if (p == nullptr || r == nullptr || gv == nullptr || gtheta_accum == nullptr) return fail(SR_E_ARG, "NULL argument");
  if (p->kind != SR_STRUCTURED) return fail(SR_E_STATE, "VJPs need a structured plan");
  return vjp_adjoint(p, (const float2*)r, (const float2*)gv, (float2*)gr_out, gtheta_accum);
}

sr_status sr_gd_step_vjp(sr_plan p, const float* y, const void* x, const float* eta_host, const void* gx_next,
                         void* gx_out, float* gy_accum, float* gtheta_accum) {
  if (p == nullptr || y == nullptr || x == nullptr || eta_host == nullptr || gx_next == nullptr || gx_out == nullptr ||
      gtheta_accum == nullptr)
    return fail(SR_E_ARG, "NULL argument");
  if (p->kind != SR_STRUCTURED) return fail(SR_E_STATE, "VJPs need a structured plan");
  if (p->loss != SR_LOSS_L2) return fail(SR_E_UNSUPPORTED, "the GD-step derivative covers the l2 intensity loss");
  for (size_t i = 0; i < p->geo.size(); ++i)
    if (!std::isfinite(eta_host[i])) return fail(SR_E_NONFINITE, "step size is not finite");
  if (gx_out == gx_next) return fail(SR_E_ARG, "gx_out must not alias gx_next");
  return gd_step_vjp(p, y, (const float2*)x, eta_host, (const float2*)gx_next, (float2*)gx_out, gy_accum,
                     gtheta_accum);
}

sr_status sr_intensity_vjp(sr_plan p, const void* x, const float* gy, void* gx_out, float* gtheta_accum) {
  if (p == nullptr || x == nullptr || gy == nullptr || gtheta_accum == nullptr) return fail(SR_E_ARG, "NULL argument");
  if (p->kind != SR_STRUCTURED) return fail(SR_E_STATE, "VJPs need a structured plan");
  return intensity_vjp(p, (const float2*)x, gy, (float2*)gx_out, gtheta_accum);
}

}  // extern "C"
