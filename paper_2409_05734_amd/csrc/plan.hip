// Plan construction: geometry offsets, FFT twiddle tables, workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <set>
#include <vector>

#include "launch.hpp"
#include "plan.hpp"

using sr::Geo;

namespace {
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Thread-order twiddle table of one tile shape (see Tile::load_twiddles):
// slot i of thread t at i * TPT + t, exp(-2 pi i e/N) evaluated in float64
// and rounded once.
template <int N, int EV>
void fill_twiddles(std::vector<float2>& out) {
  using T = sr::TileV<N, 1, false, true, EV>;
  out.assign((size_t)T::NTW * T::TPT, make_float2(1.f, 0.f));
  T::for_each_twiddle([&](int slot, int t, int e) {
    const double ang = -2.0 * M_PI * (double)e / (double)N;
    out[(size_t)slot * T::TPT + t] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  });
}

template <int N>
bool twiddles_for(int shape, std::vector<float2>& out) {
  if (shape == 0) {
    fill_twiddles<N, 0>(out);
    return true;
  }
  if constexpr (sr::HasNarrow<N>::value) {
    if (shape == 1) {
      fill_twiddles<N, 1>(out);
      return true;
    }
  }
  if constexpr (sr::HasWide<N>::value) {
    if (shape == 2) {
      fill_twiddles<N, 2>(out);
      return true;
    }
  }
  return false;
}

// false if the length has no such shape
bool thread_twiddles(int N, int shape, std::vector<float2>& out) {
  switch (N) {
#define SR_TW(n) \
  case n:        \
    return twiddles_for<n>(shape, out);
    SR_TW(16) SR_TW(32) SR_TW(64) SR_TW(96) SR_TW(128) SR_TW(192) SR_TW(256) SR_TW(384) SR_TW(512) SR_TW(768)
    SR_TW(1024) SR_TW(2048) SR_TW(4096)
#undef SR_TW
    default:
      return false;
  }
}
}  // namespace

sr_status sr_plan_s::init(const float* theta_host) {
  const size_t np = geo.size();
  xoff.assign(np + 1, 0);
  yoff.assign(np + 1, 0);
  for (size_t i = 0; i < np; ++i) {
    xoff[i + 1] = xoff[i] + geo[i].n;
    yoff[i + 1] = yoff[i] + geo[i].m;
  }

  // twiddle tables of every FFT length (and thread shape) the plan uses
  std::set<int> lens;
  int64_t max_m = 0;
  int cap = 1;
  int64_t max_grid = 0;
  for (const Geo& g : geo) {
    max_m = std::max(max_m, g.m);
    max_grid = std::max(max_grid, g.mg);
    if (kind != SR_STRUCTURED) continue;
    lens.insert(g.M1);
    if (g.ndim == 2) lens.insert(g.M2);
  }
  std::vector<float2> host_tw;
  std::vector<std::pair<std::pair<int, int>, size_t>> tw_at;  // ((length, shape), offset)
  for (int N : lens)
    for (int shape = 0; shape < 3; ++shape) {
      std::vector<float2> t;
      if (!thread_twiddles(N, shape, t)) continue;
      tw_at.push_back({{N, shape}, host_tw.size()});
      host_tw.insert(host_tw.end(), t.begin(), t.end());
      host_tw.resize((host_tw.size() + 31) / 32 * 32, make_float2(0.f, 0.f));  // 256-byte aligned tables
    }
  const size_t tw_elems = host_tw.size();

  // partial sums: one per workgroup of any pass (at most one per transform)
  for (const Geo& g : geo) cap = std::max<int>(cap, (int)std::max(g.M1, g.M2) + 1);
  part_cap = std::max(cap, 64);
  int64_t grid_elems = (kind == SR_DENSE) ? (int64_t)max_m * (int64_t)np : max_grid;
  size_t b_theta = align256(sizeof(float) * (size_t)std::max<int64_t>(theta_len, 0));
  size_t b_eph = align256(sizeof(float2) * (size_t)std::max<int64_t>(theta_len, 0));
  size_t b_tw = align256(sizeof(float2) * tw_elems);
  size_t b_grid = align256(sizeof(float2) * (size_t)grid_elems);
  size_t b_part = align256(sizeof(float) * 2 * (size_t)part_cap);
  size_t b_ysum = align256(sizeof(double) * (np + 8));
  size_t b_fs = align256(sizeof(float) * (8 * np + 64));
  size_t b_sync = 256;
  size_t b_red = align256(sizeof(double) * 1024);
  int ngrid = (kind == SR_DENSE) ? 2 : 4;
  size_t b_dsplit = 0;
  if (kind == SR_DENSE)
    b_dsplit = align256(sizeof(float) * sr::dense_split_floats((int)geo[0].m, (int)geo[0].n, (int)np));
  ws_bytes = b_theta + b_eph + b_tw + ngrid * b_grid + b_part + b_ysum + b_fs + b_sync + b_red + b_dsplit;
  hipError_t e = hipMalloc(&ws, ws_bytes);
  if (e != hipSuccess) {
    ws = nullptr;
    return sr::fail(SR_E_NOMEM, std::string("workspace allocation failed: ") + hipGetErrorString(e));
  }
  char* c = (char*)ws;
  theta = theta_len > 0 ? (float*)c : nullptr;
  c += b_theta;
  eph = theta_len > 0 ? (float2*)c : nullptr;
  c += b_eph;
  twbuf = (float2*)c;
  c += b_tw;
  bufA = (float2*)c;
  c += b_grid;
  bufB = (float2*)c;
  c += b_grid;
  if (ngrid == 4) {
    bufC = (float2*)c;
    c += b_grid;
    bufD = (float2*)c;
    c += b_grid;
  }
  part = (float*)c;
  c += b_part;
  ysum = (double*)c;
  c += b_ysum;
  fscratch = (float*)c;
  c += b_fs;
  sync = (unsigned*)c;
  c += b_sync;
  red_ws = (double*)c;
  c += b_red;
  if (b_dsplit) dsplit = (float*)c;

  for (const auto& ta : tw_at) tw[ta.first] = twbuf + ta.second;
  if (tw_elems) {
    e = hipMemcpy(twbuf, host_tw.data(), sizeof(float2) * tw_elems, hipMemcpyHostToDevice);
    if (e != hipSuccess) return sr::hip_fail(e, "twiddle upload");
  }
  if (theta_len > 0) {
    e = hipMemcpy(theta, theta_host, sizeof(float) * theta_len, hipMemcpyHostToDevice);
    if (e != hipSuccess) return sr::hip_fail(e, "theta upload");
  }
  // the tuner runs iterations on zeroed stand-in data in bufC / bufD
  if (bufC != nullptr) {
    e = hipMemset(bufC, 0, 2 * b_grid);
    if (e != hipSuccess) return sr::hip_fail(e, "workspace clear");
  }
  e = hipMemset(sync, 0, b_sync);
  if (e != hipSuccess) return sr::hip_fail(e, "workspace clear");
  e = hipMemset(part, 0, b_part);
  if (e != hipSuccess) return sr::hip_fail(e, "workspace clear");
  e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return sr::hip_fail(e, "capture stream");
  sr_status st = sr::fill_phase_table(this);
  if (st != SR_OK) return st;
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return sr::hip_fail(e, "plan setup");
  return SR_OK;
}

const float2* sr_plan_s::twiddles(int N, int shape) const {
  auto it = tw.find({N, shape});
  return it == tw.end() ? nullptr : it->second;
}

sr_status sr::aux_fork(sr_plan_s* p) {
  hipError_t e = hipSuccess;
  if (p->aux_stream == nullptr) {
    e = hipStreamCreateWithFlags(&p->aux_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
    if (e != hipSuccess) return sr::hip_fail(e, "auxiliary stream");
  }
  e = hipEventRecord(p->ev_fork, p->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->aux_stream, p->ev_fork, 0);
  if (e != hipSuccess) return sr::hip_fail(e, "stream fork");
  return SR_OK;
}

sr_status sr::aux_join(sr_plan_s* p) {
  hipError_t e = hipEventRecord(p->ev_join, p->aux_stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->ev_join, 0);
  if (e != hipSuccess) return sr::hip_fail(e, "stream join");
  return SR_OK;
}

sr_plan_s::~sr_plan_s() {
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
  if (aux_stream) {
    (void)hipStreamSynchronize(aux_stream);
    (void)hipStreamDestroy(aux_stream);
  }
  if (ev_fork) (void)hipEventDestroy(ev_fork);
  if (ev_join) (void)hipEventDestroy(ev_join);
  if (f2_descs) (void)hipFree(f2_descs);
  if (f1_args) (void)hipFree(f1_args);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
  if (vjp_buf) (void)hipFree(vjp_buf);
  if (gstep_buf) (void)hipFree(gstep_buf);
  if (d_off) (void)hipFree(d_off);
  if (d_scale) (void)hipFree(d_scale);
  if (stk_buf) (void)hipFree(stk_buf);
  if (stk_gth) (void)hipFree(stk_gth);
  if (stk_steps) (void)hipFree(stk_steps);
  if (stk_part) (void)hipFree(stk_part);
  if (batch) sr::destroy_batch_state(batch);
  if (spec_batch) sr::destroy_spec_batch_state(spec_batch);
  if (op_batch) sr::destroy_op_batch_state(op_batch);
  if (vjp_batch) sr::destroy_vjp_batch_state(vjp_batch);
  if (dense_lib) sr::destroy_dense_lib(dense_lib);
  if (lvl_bufs) (void)hipFree(lvl_bufs);
  if (ws && ws_owned) (void)hipFree(ws);
}
