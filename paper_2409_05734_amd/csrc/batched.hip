// Batched gradient descent over many independent problems of uneven shape:
// one launch per pass level advances every problem by one fused pass, instead
// of one launch per (problem, pass).
//
// Every problem's GD iteration is its own list of 2L+1 fused passes (its
// lengths, layers and step size); level q of a batched iteration runs pass q
// of every problem that has one.  A launch is a flat list of work items
// (descriptor, tile); all tiles are 256-thread workgroups, the tile width of
// each length chosen so that (N / E) * B = 256.  Each problem owns private
// ping-pong buffers, so problems never share scratch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "passes.hpp"
#include "schedule.hpp"

namespace sr {

namespace {

constexpr int kBatchThreads = 256;

struct BatchDesc {
  PassArgs a;
  int N;
  int col;
  int kind;
  int pad;
};

struct BatchItem {
  int desc;
  int tile;
};

template <int N>
constexpr int batch_b() {
  return kBatchThreads * FftShape<N>::E / N;
}

template <int N, bool COL>
__device__ __forceinline__ void run_kind(const PassArgs& a, int kind, int tile, float2* lds, float* red) {
  constexpr int B = batch_b<N>();
  if constexpr (COL) {
    switch (kind) {
      case PK_FIRST_FWD:
        pass_tile<N, B, COL, PRE_PHASE, MID_NONE, false, false, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                   nullptr);
        return;
      case PK_LAST_GD:
        pass_tile<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_GD>(a, tile, lds, red, nullptr, 0, nullptr);
        return;
      default:
        break;
    }
  }
  switch (kind) {
    case PK_MID_FWD:
      pass_tile<N, B, COL, PRE_NONE, MID_PHASE, true, false, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                nullptr);
      return;
    case PK_TURN_GD:
      pass_tile<N, B, COL, PRE_NONE, MID_GD, true, false, true, POST_STORE>(a, tile, lds, red, nullptr, 0, nullptr);
      return;
    case PK_MID_ADJ:
      pass_tile<N, B, COL, PRE_NONE, MID_PHASE_CONJ, true, true, true, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                   nullptr);
      return;
    default:
      return;
  }
}

template <int N>
__device__ __forceinline__ void run_len(const BatchDesc& d, int tile, float2* lds, float* red) {
  static_assert(Tile<N, batch_b<N>(), true>::THREADS == kBatchThreads, "batched tiles are 256 threads");
  if (d.col) run_kind<N, true>(d.a, d.kind, tile, lds, red);
  else run_kind<N, false>(d.a, d.kind, tile, lds, red);
}

__global__ void __launch_bounds__(kBatchThreads) batched_level_kernel(const BatchItem* __restrict__ items,
                                                                      const BatchDesc* __restrict__ descs) {
  extern __shared__ float2 lds[];
  __shared__ float red[kBatchThreads];
  const BatchItem it = items[blockIdx.x];
  const BatchDesc& d = descs[it.desc];
  switch (d.N) {
    case 16: run_len<16>(d, it.tile, lds, red); break;
    case 32: run_len<32>(d, it.tile, lds, red); break;
    case 64: run_len<64>(d, it.tile, lds, red); break;
    case 96: run_len<96>(d, it.tile, lds, red); break;
    case 128: run_len<128>(d, it.tile, lds, red); break;
    case 192: run_len<192>(d, it.tile, lds, red); break;
    case 256: run_len<256>(d, it.tile, lds, red); break;
    case 384: run_len<384>(d, it.tile, lds, red); break;
    case 512: run_len<512>(d, it.tile, lds, red); break;
    default: break;
  }
}

constexpr size_t kBatchLds = 2 * sizeof(float2) * kBatchThreads * 12;  // 2 * B * N elements, E <= 12

int batch_tile_width(int N) {
  switch (N) {
    case 16: return batch_b<16>();
    case 32: return batch_b<32>();
    case 64: return batch_b<64>();
    case 96: return batch_b<96>();
    case 128: return batch_b<128>();
    case 192: return batch_b<192>();
    case 256: return batch_b<256>();
    case 384: return batch_b<384>();
    case 512: return batch_b<512>();
    default: return 0;
  }
}

}  // namespace

// Per-plan state of the batched schedule (device descriptors + item lists of
// each level, private pass buffers), rebuilt when the call's pointers change.
struct BatchState {
  std::string key;
  float2* bufs = nullptr;  // per problem: two full grids
  BatchDesc* d_descs = nullptr;
  BatchItem* d_items = nullptr;
  std::vector<int> level_off, level_cnt;  // item ranges per level
  ~BatchState() {
    if (bufs) hipFree(bufs);
    if (d_descs) hipFree(d_descs);
    if (d_items) hipFree(d_items);
  }
};

void destroy_batch_state(BatchState* s) { delete s; }

bool batched_supported(const sr_plan_s* p) {
  if (p->kind != SR_STRUCTURED || p->geo.size() < 2) return false;
  for (const Geo& g : p->geo)
    if (g.ndim != 2 || batch_tile_width(g.M1) == 0 || batch_tile_width(g.M2) == 0) return false;
  return true;
}

sr_status gd_iter_2d_public(sr_plan_s* p, const Geo& g, const float* y, float2* x, float step, float* loss_part);

// Build (or reuse) the level lists for GD on (y, x, eta).
static sr_status batch_prepare(sr_plan_s* p, const float* y, float2* x, const float* eta, BatchState** out) {
  std::string key = std::to_string((uintptr_t)y) + ":" + std::to_string((uintptr_t)x);
  for (size_t i = 0; i < p->geo.size(); ++i) {
    uint32_t u;
    std::memcpy(&u, &eta[i], 4);
    key += ":" + std::to_string(u);
  }
  BatchState* st = p->batch;
  if (st != nullptr && st->key == key) {
    *out = st;
    return SR_OK;
  }
  if (st == nullptr) {
    st = new BatchState();
    p->batch = st;
    size_t elems = 0;
    for (const Geo& g : p->geo) elems += 2 * (size_t)g.m;
    hipError_t e = hipMalloc(&st->bufs, elems * sizeof(float2));
    if (e != hipSuccess) {
      st->bufs = nullptr;
      return fail(SR_E_NOMEM, "batched workspace allocation failed");
    }
  }
  st->key = key;
  // record every problem's iteration with its private buffers
  std::vector<std::vector<PassRecord>> recs(p->geo.size());
  float2* saveA = p->bufA;
  float2* saveB = p->bufB;
  size_t off = 0;
  size_t max_levels = 0;
  sr_status status = SR_OK;
  for (size_t i = 0; i < p->geo.size() && status == SR_OK; ++i) {
    const Geo& g = p->geo[i];
    p->bufA = st->bufs + off;
    p->bufB = st->bufs + off + g.m;
    off += 2 * (size_t)g.m;
    g_recording = &recs[i];
    status = gd_iter_2d_public(p, g, y + p->yoff[i], x + p->xoff[i], eta[i] / (float)g.m, nullptr);
    g_recording = nullptr;
    max_levels = std::max(max_levels, recs[i].size());
  }
  p->bufA = saveA;
  p->bufB = saveB;
  if (status != SR_OK) return status;
  std::vector<BatchDesc> descs;
  std::vector<BatchItem> items;
  st->level_off.assign(max_levels, 0);
  st->level_cnt.assign(max_levels, 0);
  for (size_t q = 0; q < max_levels; ++q) {
    st->level_off[q] = (int)items.size();
    for (size_t i = 0; i < recs.size(); ++i) {
      if (q >= recs[i].size()) continue;
      const PassRecord& r = recs[i][q];
      const Geo& g = p->geo[i];
      BatchDesc d;
      std::memset(&d, 0, sizeof(d));
      d.a = r.a;
      d.N = pass_len(g, r.k);
      d.col = pass_col(r.k);
      d.kind = r.kind;
      const int B = batch_tile_width(d.N);
      const int di = (int)descs.size();
      descs.push_back(d);
      for (int t = 0; t * B < r.a.ntr; ++t) items.push_back({di, t});
    }
    st->level_cnt[q] = (int)items.size() - st->level_off[q];
  }
  if (st->d_descs) hipFree(st->d_descs);
  if (st->d_items) hipFree(st->d_items);
  st->d_descs = nullptr;
  st->d_items = nullptr;
  hipError_t e = hipMalloc(&st->d_descs, descs.size() * sizeof(BatchDesc));
  if (e == hipSuccess) e = hipMalloc(&st->d_items, items.size() * sizeof(BatchItem));
  if (e != hipSuccess) return fail(SR_E_NOMEM, "batched descriptor allocation failed");
  e = hipMemcpyAsync(st->d_descs, descs.data(), descs.size() * sizeof(BatchDesc), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(st->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);  // host vectors go out of scope
  if (e != hipSuccess) return hip_fail(e, "batched descriptor upload");
  *out = st;
  return SR_OK;
}

static sr_status batch_iteration(sr_plan_s* p, BatchState* st) {
  for (size_t q = 0; q < st->level_cnt.size(); ++q) {
    if (st->level_cnt[q] == 0) continue;
    hipLaunchKernelGGL(batched_level_kernel, dim3(st->level_cnt[q]), dim3(kBatchThreads), kBatchLds, p->stream,
                       st->d_items + st->level_off[q], st->d_descs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batched level launch");
  }
  return SR_OK;
}

sr_status batched_gd(sr_plan_s* p, const float* y, float2* x, int iters, const float* eta) {
  BatchState* st = nullptr;
  sr_status s = batch_prepare(p, y, x, eta, &st);
  if (s != SR_OK) return s;
  constexpr int kChunk = 50;
  int it = 0;
  if (iters >= kChunk && graphs_enabled(p)) {
    const std::string gkey = "batch:" + st->key;
    for (; it + kChunk <= iters; it += kChunk) {
      s = launch_captured(p, gkey, [&]() -> sr_status {
        for (int c = 0; c < kChunk; ++c) {
          sr_status q = batch_iteration(p, st);
          if (q != SR_OK) return q;
        }
        return SR_OK;
      });
      if (s != SR_OK) return s;
    }
  }
  for (; it < iters; ++it) {
    s = batch_iteration(p, st);
    if (s != SR_OK) return s;
  }
  return SR_OK;
}

}  // namespace sr
