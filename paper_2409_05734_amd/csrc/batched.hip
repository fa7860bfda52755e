// Batched gradient descent over many independent problems of uneven shape:
// one launch per pass level advances every problem by one fused pass, instead
// of one launch per (problem, pass).
//
// Every problem's GD iteration is its own list of 2L+1 fused passes (its
// lengths, layers and step size); level q of a batched iteration runs pass q
// of every problem that has one.  A launch is a flat list of work items
// (descriptor, tile); all tiles are 256-thread workgroups, the tile width of
// each length chosen so that (N / E) * B = 256.  For the GD and power-
// iteration passes, each (length, axis) runs the default thread shape (E = 8
// or 12, radix-8 stages) or, where the length has one, the narrow shape (E =
// 4, radix-4 stages, twice the threads per transform), as the level tuner
// picks per plan.  Each problem owns private ping-pong buffers, so problems
// never share scratch.
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
  int ev;  // thread shape: 0 default, 1 narrow (GD and power-iteration sets)
};

struct BatchItem {
  int desc;
  int tile;
};

template <int N, int EV = 0>
constexpr int batch_b() {
  return kBatchThreads * (EV ? 4 : FftShape<N>::E) / N;
}

template <int N, bool COL, int EV = 0>
__device__ __forceinline__ void run_kind_gd(const PassArgs& a, int kind, int tile, float2* lds, float* red) {
  constexpr int B = batch_b<N, EV>();
  if constexpr (COL) {
    switch (kind) {
      case PK_FIRST_FWD:
        pass_tile_rt<N, B, COL, PRE_PHASE, MID_NONE, false, false, false, POST_STORE, EV>(a, tile, lds, red, nullptr, 0,
                                                                                   nullptr);
        return;
      case PK_LAST_GD:
        pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_GD, EV>(a, tile, lds, red, nullptr, 0, nullptr);
        return;
      case PK_LAST_GD_FWD:
        pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_GD_FWD, EV>(a, tile, lds, red, nullptr, 0,
                                                                                  nullptr);
        return;
      default:
        break;
    }
  }
  switch (kind) {
    case PK_MID_FWD:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE, true, false, false, POST_STORE, EV>(a, tile, lds, red, nullptr, 0,
                                                                                nullptr);
      return;
    case PK_TURN_GD:  // (loss partials where the descriptor asks for a trace)
      pass_tile_rt<N, B, COL, PRE_NONE, MID_GD, true, false, true, POST_STORE, EV>(a, tile, lds, red, nullptr, 0,
                                                                            a.part_out);
      return;
    case PK_TURN_GD_POIS:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_GD_POIS, true, false, true, POST_STORE, EV>(a, tile, lds, red, nullptr, 0,
                                                                                 a.part_out);
      return;
    case PK_MID_ADJ:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE_CONJ, true, true, true, POST_STORE, EV>(a, tile, lds, red, nullptr, 0,
                                                                                   nullptr);
      return;
    default:
      return;
  }
}


// The passes of a power iteration (deferred normalisation: the last pass
// reads the previous iterate's squared-norm partials and writes the new
// ones, each problem's own, through its descriptor).
template <int N, bool COL, int EV = 0>
__device__ __forceinline__ void run_kind_spec(const PassArgs& a, int kind, int tile, float2* lds, float* red) {
  constexpr int B = batch_b<N, EV>();
  if constexpr (COL) {
    switch (kind) {
      case PK_FIRST_FWD:
        pass_tile_rt<N, B, COL, PRE_PHASE, MID_NONE, false, false, false, POST_STORE, EV>(a, tile, lds, red, nullptr, 0,
                                                                                   nullptr);
        return;
      case PK_LAST_SPEC:
        pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_SPEC, EV>(a, tile, lds, red, a.part_in, a.npart,
                                                                                a.part_out);
        return;
      case PK_LAST_SPEC_FWD:
        pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_SPEC_FWD, EV>(a, tile, lds, red, a.part_in,
                                                                                    a.npart, a.part_out);
        return;
      default:
        break;
    }
  }
  switch (kind) {
    case PK_MID_FWD:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE, true, false, false, POST_STORE, EV>(a, tile, lds, red, nullptr, 0,
                                                                                nullptr);
      return;
    case PK_TURN_SPEC:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_SPEC, true, false, true, POST_STORE, EV>(a, tile, lds, red, nullptr, 0, nullptr);
      return;
    case PK_MID_ADJ:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE_CONJ, true, true, true, POST_STORE, EV>(a, tile, lds, red, nullptr, 0,
                                                                                   nullptr);
      return;
    default:
      return;
  }
}

// The passes of A and A^H alone.
template <int N, bool COL>
__device__ __forceinline__ void run_kind_op(const PassArgs& a, int kind, int tile, float2* lds, float* red) {
  constexpr int B = batch_b<N>();
  if constexpr (COL) {
    switch (kind) {
      case PK_FIRST_FWD:
        pass_tile_rt<N, B, COL, PRE_PHASE, MID_NONE, false, false, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                   nullptr);
        return;
      case PK_LAST_ADJ:
        pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_PHASE_CONJ_STORE>(a, tile, lds, red,
                                                                                            nullptr, 0, nullptr);
        return;
      default:
        break;
    }
  }
  switch (kind) {
    case PK_MID_FWD:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE, true, false, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                nullptr);
      return;
    case PK_LAST_STORE:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_STORE, false, false, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                 nullptr);
      return;
    case PK_FIRST_ADJ:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                               nullptr);
      return;
    case PK_MID_ADJ:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE_CONJ, true, true, true, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                   nullptr);
      return;
    default:
      return;
  }
}

// The passes of both reverse-mode products (recomputation with saved
// intermediates, phase cotangents accumulated at each diagonal).
template <int N, bool COL>
__device__ __forceinline__ void run_kind_vjp(const PassArgs& a, int kind, int tile, float2* lds, float* red) {
  constexpr int B = batch_b<N>();
  if constexpr (COL) {
    switch (kind) {
      case PK_FIRST_FWD:
        pass_tile_rt<N, B, COL, PRE_PHASE, MID_NONE, false, false, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                   nullptr);
        return;
      case PK_LAST_ADJ:
        pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_PHASE_CONJ_STORE>(a, tile, lds, red,
                                                                                            nullptr, 0, nullptr);
        return;
      case PK_LAST_ADJ_GT:
        pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_PHASE_CONJ_GT>(a, tile, lds, red,
                                                                                         nullptr, 0, nullptr);
        return;
      default:
        break;
    }
  }
  switch (kind) {
    case PK_MID_FWD_SAVE:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE_SAVE, true, false, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                     nullptr);
      return;
    case PK_MID_FWD_GT:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE_GT, true, false, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                   nullptr);
      return;
    case PK_MID_ADJ_GT:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE_CONJ_GT, true, true, true, POST_STORE>(a, tile, lds, red, nullptr,
                                                                                      0, nullptr);
      return;
    case PK_MID_ADJ_SAVE:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE_CONJ_SAVE, true, true, true, POST_STORE>(a, tile, lds, red, nullptr,
                                                                                        0, nullptr);
      return;
    case PK_FIRST_ADJ:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                               nullptr);
      return;
    case PK_LAST_STORE:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_STORE, false, false, false, POST_STORE>(a, tile, lds, red, nullptr, 0,
                                                                                 nullptr);
      return;
    default:
      return;
  }
}

constexpr size_t kBatchLds = 2 * sizeof(float2) * kBatchThreads * 12;  // covers 2 * B * NP elements for E <= 12

// Length classes of the GD level kernel.  The twelve-element lengths (96,
// 192, 384) hold the kernel's register count up (about 200 VGPRs, with 27
// twiddles per thread); without them it needs 124 and no spill, and its
// tiles fit a 36 KB LDS budget, so four workgroups share a CU.  A GD solve
// runs the problems with no twelve-element axis on that instantiation and
// the others on one with every length, on two streams.
enum LevelCls : int { LEN_ALL = 0, LEN_POW2 = 1, LEN_TWELVE = 2 };
constexpr int level_groups(int cls) { return cls == LEN_POW2 ? 4 : cls == LEN_TWELVE ? 2 : 3; }
constexpr size_t level_lds(int cls) {
  return cls == LEN_POW2 ? 2 * sizeof(float2) * kBatchThreads * 9 : kBatchLds;  // E = 8 tiles pad 1 in 8
}
constexpr bool twelve_len(int N) { return N == 96 || N == 192 || N == 384; }

// Pass sets of the level kernel, one instantiation each (so that no set
// carries the registers of the others).
enum LevelSetKind : int { LS_GD = 0, LS_SPEC = 1, LS_OP = 2, LS_VJP = 3 };

template <int N, int SET, int CLS>
__device__ __forceinline__ void run_len(const BatchDesc& d, int tile, float2* lds, float* red) {
  static_assert(Tile<N, batch_b<N>(), true>::THREADS == kBatchThreads, "batched tiles are 256 threads");
  static_assert(2 * sizeof(float2) * Tile<N, batch_b<N>(), true>::BUF <= level_lds(CLS), "batched LDS budget");
  if constexpr (HasNarrow<N>::value && (SET == LS_GD || SET == LS_SPEC)) {
    using TN = TileV<N, batch_b<N, 1>(), true, true, 1>;
    static_assert(TN::THREADS == kBatchThreads, "batched narrow tiles are 256 threads");
    static_assert(2 * sizeof(float2) * TN::BUF <= level_lds(CLS), "batched LDS budget");
    if (d.ev) {
      if constexpr (SET == LS_SPEC) {
        if (d.col) run_kind_spec<N, true, 1>(d.a, d.kind, tile, lds, red);
        else run_kind_spec<N, false, 1>(d.a, d.kind, tile, lds, red);
      } else {
        if (d.col) run_kind_gd<N, true, 1>(d.a, d.kind, tile, lds, red);
        else run_kind_gd<N, false, 1>(d.a, d.kind, tile, lds, red);
      }
      return;
    }
  }
  if constexpr (SET == LS_SPEC) {
    if (d.col) run_kind_spec<N, true>(d.a, d.kind, tile, lds, red);
    else run_kind_spec<N, false>(d.a, d.kind, tile, lds, red);
  } else if constexpr (SET == LS_OP) {
    if (d.col) run_kind_op<N, true>(d.a, d.kind, tile, lds, red);
    else run_kind_op<N, false>(d.a, d.kind, tile, lds, red);
  } else if constexpr (SET == LS_VJP) {
    if (d.col) run_kind_vjp<N, true>(d.a, d.kind, tile, lds, red);
    else run_kind_vjp<N, false>(d.a, d.kind, tile, lds, red);
  } else {
    if (d.col) run_kind_gd<N, true>(d.a, d.kind, tile, lds, red);
    else run_kind_gd<N, false>(d.a, d.kind, tile, lds, red);
  }
}

// The power-of-two class compiles only those lengths; the twelve-element
// class compiles every length, since its problems may have a power-of-two
// length on their other axis.
template <int N, int SET, int CLS>
__device__ __forceinline__ void run_len_if(const BatchDesc& d, int tile, float2* lds, float* red) {
  if constexpr (CLS != LEN_POW2 || !twelve_len(N)) run_len<N, SET, CLS>(d, tile, lds, red);
}

// All lengths: three workgroups per CU (the LDS budget's limit); the compiler
// fits the kernel in 168 VGPRs (a small spill on the twelve-element lengths)
// instead of 197, which held it to two (71 -> 62.5 ms on 256 uneven
// problems).  The power-of-two class: four workgroups per CU, 124 VGPRs, no
// spill; the twelve-element class: two, no spill.
template <int SET, int CLS>
__global__ void __launch_bounds__(kBatchThreads, level_groups(CLS))
    batched_level_kernel(const BatchItem* __restrict__ items, const BatchDesc* __restrict__ descs) {
  extern __shared__ float2 lds[];
  __shared__ float red[kBatchThreads];
  const BatchItem it = items[xcd_tile(blockIdx.x, gridDim.x)];
  const BatchDesc& d = descs[it.desc];
  switch (d.N) {
    case 16: run_len_if<16, SET, CLS>(d, it.tile, lds, red); break;
    case 32: run_len_if<32, SET, CLS>(d, it.tile, lds, red); break;
    case 64: run_len_if<64, SET, CLS>(d, it.tile, lds, red); break;
    case 96: run_len_if<96, SET, CLS>(d, it.tile, lds, red); break;
    case 128: run_len_if<128, SET, CLS>(d, it.tile, lds, red); break;
    case 192: run_len_if<192, SET, CLS>(d, it.tile, lds, red); break;
    case 256: run_len_if<256, SET, CLS>(d, it.tile, lds, red); break;
    case 384: run_len_if<384, SET, CLS>(d, it.tile, lds, red); break;
    case 512: run_len_if<512, SET, CLS>(d, it.tile, lds, red); break;
    default: break;
  }
}

// Transforms per 256-thread tile: default shape, or the narrow one (ev = 1)
// where the length has it (0: length not taken by the level kernel).
int batch_tile_width(int N, int ev = 0) {
  if (ev) {
    switch (N) {
      case 64: return batch_b<64, 1>();
      case 128: return batch_b<128, 1>();
      case 256: return batch_b<256, 1>();
      case 512: return batch_b<512, 1>();
      default: break;
    }
  }
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

// Each pass set's kernel is compiled in a translation unit of its own (this
// file built with SR_LEVEL_SET = 0..3; they compile in parallel), behind a
// plain host launcher (untyped pointers: the descriptor types are local to
// each translation unit); the build without it holds the host side.
hipError_t launch_level_set0(dim3 grid, hipStream_t s, const void* items, const void* descs);
hipError_t launch_level_set1(dim3 grid, hipStream_t s, const void* items, const void* descs);
hipError_t launch_level_set2(dim3 grid, hipStream_t s, const void* items, const void* descs);
hipError_t launch_level_set3(dim3 grid, hipStream_t s, const void* items, const void* descs);
// the GD and spectral sets by length class (SR_LEVEL_SET = 0 / 1 built with
// SR_LEVEL_CLS = 1 / 2): launch_level_s<set>_c<class>
hipError_t launch_level_s0_c1(dim3 grid, hipStream_t s, const void* items, const void* descs);
hipError_t launch_level_s0_c2(dim3 grid, hipStream_t s, const void* items, const void* descs);
hipError_t launch_level_s1_c1(dim3 grid, hipStream_t s, const void* items, const void* descs);
hipError_t launch_level_s1_c2(dim3 grid, hipStream_t s, const void* items, const void* descs);

#if defined(SR_LEVEL_SET)
#if !defined(SR_LEVEL_CLS) || SR_LEVEL_CLS == 0
#define SR_LAUNCHER_NAME(k) launch_level_set##k
#define SR_LAUNCHER(k) SR_LAUNCHER_NAME(k)
hipError_t SR_LAUNCHER(SR_LEVEL_SET)(dim3 grid, hipStream_t s, const void* items, const void* descs) {
  hipLaunchKernelGGL((batched_level_kernel<SR_LEVEL_SET, LEN_ALL>), grid, dim3(kBatchThreads), level_lds(LEN_ALL), s,
                     (const BatchItem*)items, (const BatchDesc*)descs);
  return hipGetLastError();
}
#else
#define SR_CLS_LAUNCHER_NAME(k, c) launch_level_s##k##_c##c
#define SR_CLS_LAUNCHER(k, c) SR_CLS_LAUNCHER_NAME(k, c)
hipError_t SR_CLS_LAUNCHER(SR_LEVEL_SET, SR_LEVEL_CLS)(dim3 grid, hipStream_t s, const void* items, const void* descs) {
  hipLaunchKernelGGL((batched_level_kernel<SR_LEVEL_SET, SR_LEVEL_CLS>), grid, dim3(kBatchThreads),
                     level_lds(SR_LEVEL_CLS), s, (const BatchItem*)items, (const BatchDesc*)descs);
  return hipGetLastError();
}
#endif
}  // namespace sr
#else

// Level lists of one recorded pass sequence (device descriptors and items).
struct LevelSet {
  int set = LS_GD;  // pass set (which instantiation of the level kernel)
  int cls = LEN_ALL;  // length class (GD set only)
  BatchDesc* d_descs = nullptr;
  BatchItem* d_items = nullptr;
  std::vector<int> level_off, level_cnt;  // item ranges per level
  ~LevelSet() {
    if (d_descs) (void)hipFree(d_descs);
    if (d_items) (void)hipFree(d_items);
  }
};

// Per-plan state of the batched schedule, rebuilt when the call's pointers
// change: private pass buffers and three level sets -- the first pass of
// every problem, the steady iteration (ending with the update fused with the
// next first pass), and the final iteration (plain update).
struct BatchState {
  std::string key;
  LevelSet first, steady, last;  // every problem (loss traces)
  // without a trace: the same per length class of the problem (0: both
  // axes a power of two, 1: an axis of twelve-element length), each on its
  // own instantiation and stream
  LevelSet cfirst[2], csteady[2], clast[2];
  bool has[2] = {false, false};
  bool split = false;
  // with a loss trace: the turnaround of each problem writes its loss
  // partials (nparts of them, at its own offset), summed per problem
  bool trace = false;
  float* parts = nullptr;
  int2* d_pdesc = nullptr;  // per problem: (offset, count) of its partials
  ~BatchState() {
    if (parts) (void)hipFree(parts);
    if (d_pdesc) (void)hipFree(d_pdesc);
  }
};

void destroy_batch_state(BatchState* s) { delete s; }

bool batch_level_capable(const Geo& g) {
  return g.ndim == 2 && batch_tile_width(g.M1) != 0 && batch_tile_width(g.M2) != 0;
}

// The private ping-pong buffers (two grids) of every problem the level
// kernel can take, shared by the GD, power-iteration and operator levels,
// which all run in order on the plan's stream.
static sr_status level_bufs(sr_plan_s* p) {
  if (p->lvl_bufs != nullptr) return SR_OK;
  size_t elems = 0;
  p->lvl_off.assign(p->geo.size(), 0);
  for (size_t i = 0; i < p->geo.size(); ++i) {
    p->lvl_off[i] = elems;
    if (batch_level_capable(p->geo[i])) elems += 2 * (size_t)p->geo[i].mg;
  }
  if (hipMalloc(&p->lvl_bufs, std::max<size_t>(elems, 1) * sizeof(float2)) != hipSuccess) {
    p->lvl_bufs = nullptr;
    return fail(SR_E_NOMEM, "batched workspace allocation failed");
  }
  return SR_OK;
}

// Problems whose whole grid fits one workgroup's LDS run in the LDS-resident
// solver (one launch for the whole solve); the others run as level launches.
static bool lds_resident(const Geo& g) { return fused2d_enabled(false) && fused2d_supported(g); }

bool batched_any_resident(const sr_plan_s* p) {
  for (const Geo& g : p->geo)
    if (lds_resident(g)) return true;
  return false;
}

bool batched_supported(const sr_plan_s* p) {
  if (p->kind != SR_STRUCTURED || p->geo.size() < 2) return false;
  for (const Geo& g : p->geo)
    if (g.ndim != 2 || (!lds_resident(g) && (batch_tile_width(g.M1) == 0 || batch_tile_width(g.M2) == 0)))
      return false;
  return true;
}

sr_status gd_first_pass_public(sr_plan_s* p, const Geo& g, const float2* x);
sr_status gd_steady_public(sr_plan_s* p, const Geo& g, const float* y, float2* x, float step, bool last,
                           float* loss_part = nullptr);

// Loss trace: out[i * ostride] = sum of problem i's partials, in index order
// (one thread per problem, the order of the single-problem reduction).
__global__ void batch_loss_reduce(const float* __restrict__ parts, const int2* __restrict__ desc, int count,
                                  float* out, int ostride) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    double acc = 0.0;
    const int2 d = desc[i];
    for (int k = 0; k < d.y; ++k) acc += (double)parts[d.x + k];
    out[(long long)i * ostride] = (float)acc;
  }
}

// Turn per-problem pass recordings into levels (level q = pass q of every
// problem that has one) and upload them.
static sr_status build_levels(sr_plan_s* p, const std::vector<std::vector<PassRecord>>& recs, LevelSet& ls) {
  size_t max_levels = 0;
  for (const auto& r : recs) max_levels = std::max(max_levels, r.size());
  std::vector<BatchDesc> descs;
  std::vector<BatchItem> items;
  ls.level_off.assign(max_levels, 0);
  ls.level_cnt.assign(max_levels, 0);
  for (size_t q = 0; q < max_levels; ++q) {
    ls.level_off[q] = (int)items.size();
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
      d.ev = (ls.set == LS_GD || ls.set == LS_SPEC) ? p->bev(d.N, d.col != 0) : 0;
      const int B = batch_tile_width(d.N, d.ev);
      const int di = (int)descs.size();
      descs.push_back(d);
      for (int t = 0; t * B < r.a.ntr; ++t) items.push_back({di, t});
    }
    ls.level_cnt[q] = (int)items.size() - ls.level_off[q];
  }
  if (ls.d_descs != nullptr || ls.d_items != nullptr) {
    // launches already queued may still read the old lists
    if (hipError_t w = hipStreamSynchronize(p->stream); w != hipSuccess) return hip_fail(w, "stream wait");
    if (ls.d_descs) (void)hipFree(ls.d_descs);
    if (ls.d_items) (void)hipFree(ls.d_items);
  }
  ls.d_descs = nullptr;
  ls.d_items = nullptr;
  hipError_t e = hipMalloc(&ls.d_descs, std::max<size_t>(descs.size(), 1) * sizeof(BatchDesc));
  if (e == hipSuccess) e = hipMalloc(&ls.d_items, std::max<size_t>(items.size(), 1) * sizeof(BatchItem));
  if (e != hipSuccess) return fail(SR_E_NOMEM, "batched descriptor allocation failed");
  e = hipMemcpyAsync(ls.d_descs, descs.data(), descs.size() * sizeof(BatchDesc), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ls.d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);  // the host vectors go out of scope
  if (e != hipSuccess) return hip_fail(e, "batched descriptor upload");
  return SR_OK;
}

// Build (or reuse) the level sets for GD on (y, x, eta), with or without the
// loss partials of a trace.
static sr_status batch_prepare(sr_plan_s* p, const float* y, float2* x, const float* eta, bool trace,
                               BatchState** out) {
  std::string key = std::to_string((uintptr_t)y) + ":" + std::to_string((uintptr_t)x) + (trace ? ":tr" : "") +
                    (fused2d_enabled(false) ? ":r" : "");
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
  // graphs captured over the old lists (keys "batch:...", "batch0:...", "batch1:...")
  if (sr_status dg = drop_graphs(p, "batch"); dg != SR_OK) return dg;
  if (sr_status lb = level_bufs(p); lb != SR_OK) return lb;
  if (st == nullptr) {
    st = new BatchState();
    p->batch = st;
  }
  st->key.clear();
  const size_t np = p->geo.size();
  std::vector<int> poff(np, 0);
  if (trace && st->parts == nullptr) {
    // the turnaround's tiles under the level kernel's widths
    std::vector<int2> pd(np);
    int tot = 0;
    for (size_t i = 0; i < np; ++i) {
      const Geo& g = p->geo[i];
      const int k = g.L + 1;
      const int ntr = (k == 2) ? g.M1 : (pass_col(k) ? g.M2 : g.M1);
      const int bt = batch_tile_width(pass_len(g, k), p->bev(pass_len(g, k), pass_col(k)));
      pd[i] = make_int2(tot, bt > 0 ? (ntr + bt - 1) / bt : 0);
      tot += pd[i].y;
    }
    hipError_t e = hipMalloc(&st->parts, sizeof(float) * std::max(tot, 1));
    if (e == hipSuccess) e = hipMalloc(&st->d_pdesc, sizeof(int2) * np);
    if (e == hipSuccess)
      e = hipMemcpyAsync(st->d_pdesc, pd.data(), sizeof(int2) * np, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);  // pd goes out of scope
    if (e != hipSuccess) return fail(SR_E_NOMEM, "loss-trace workspace allocation failed");
  }
  if (trace) {
    int tot = 0;
    for (size_t i = 0; i < np; ++i) {
      const Geo& g = p->geo[i];
      const int k = g.L + 1;
      const int ntr = (k == 2) ? g.M1 : (pass_col(k) ? g.M2 : g.M1);
      const int bt = batch_tile_width(pass_len(g, k), p->bev(pass_len(g, k), pass_col(k)));
      poff[i] = tot;
      tot += bt > 0 ? (ntr + bt - 1) / bt : 0;
    }
  }
  st->trace = trace;
  std::vector<std::vector<PassRecord>> rec_first(np), rec_steady(np), rec_last(np);
  float2* saveA = p->bufA;
  float2* saveB = p->bufB;
  sr_status status = SR_OK;
  for (size_t i = 0; i < np && status == SR_OK; ++i) {
    const Geo& g = p->geo[i];
    // solved by the LDS-resident kernel, or not by the level kernel at all
    // (the level tuner comes here for any plan with level problems; only
    // those have private buffers)
    if (lds_resident(g) || !batch_level_capable(g)) continue;
    p->bufA = p->lvl_bufs + p->lvl_off[i];  // each problem's private ping-pong buffers
    p->bufB = p->lvl_bufs + p->lvl_off[i] + g.mg;
    const float* yi = y + p->yoff[i];
    float2* xi = x + p->xoff[i];
    const float step = eta[i] / (float)g.m;
    g_recording = &rec_first[i];
    status = gd_first_pass_public(p, g, xi);
    g_recording = &rec_steady[i];
    float* lp = trace ? st->parts + poff[i] : nullptr;
    if (status == SR_OK) status = gd_steady_public(p, g, yi, xi, step, false, lp);
    g_recording = &rec_last[i];
    if (status == SR_OK) status = gd_steady_public(p, g, yi, xi, step, true, lp);
    g_recording = nullptr;
  }
  p->bufA = saveA;
  p->bufB = saveB;
  if (status != SR_OK) return status;
  st->split = !trace && !batched_any_resident(p);  // (the aux stream serves the LDS-resident solver otherwise)
  if (st->split) {
    std::vector<std::vector<PassRecord>> cf[2], cs[2], cl[2];
    for (int c = 0; c < 2; ++c) {
      cf[c].assign(np, {});
      cs[c].assign(np, {});
      cl[c].assign(np, {});
      st->has[c] = false;
    }
    for (size_t i = 0; i < np; ++i) {
      if (rec_first[i].empty()) continue;
      const Geo& g = p->geo[i];
      const int c = (twelve_len(g.M1) || twelve_len(g.M2)) ? 1 : 0;
      cf[c][i] = std::move(rec_first[i]);
      cs[c][i] = std::move(rec_steady[i]);
      cl[c][i] = std::move(rec_last[i]);
      st->has[c] = true;
    }
    for (int c = 0; c < 2; ++c) {
      if (!st->has[c]) continue;
      const int cls = c == 0 ? LEN_POW2 : LEN_TWELVE;
      st->cfirst[c].cls = st->csteady[c].cls = st->clast[c].cls = cls;
      if ((status = build_levels(p, cf[c], st->cfirst[c])) != SR_OK) return status;
      if ((status = build_levels(p, cs[c], st->csteady[c])) != SR_OK) return status;
      if ((status = build_levels(p, cl[c], st->clast[c])) != SR_OK) return status;
    }
  } else {
    if ((status = build_levels(p, rec_first, st->first)) != SR_OK) return status;
    if ((status = build_levels(p, rec_steady, st->steady)) != SR_OK) return status;
    if ((status = build_levels(p, rec_last, st->last)) != SR_OK) return status;
  }
  st->key = key;
  *out = st;
  return SR_OK;
}

static sr_status run_levels(sr_plan_s* p, const LevelSet& ls) {
  for (size_t q = 0; q < ls.level_cnt.size(); ++q) {
    if (ls.level_cnt[q] == 0) continue;
    const dim3 grid(ls.level_cnt[q]);
    const BatchItem* items = ls.d_items + ls.level_off[q];
    hipError_t e;
    if (ls.set == LS_GD && ls.cls == LEN_POW2) e = launch_level_s0_c1(grid, p->stream, items, ls.d_descs);
    else if (ls.set == LS_GD && ls.cls == LEN_TWELVE) e = launch_level_s0_c2(grid, p->stream, items, ls.d_descs);
    else if (ls.set == LS_SPEC && ls.cls == LEN_POW2) e = launch_level_s1_c1(grid, p->stream, items, ls.d_descs);
    else if (ls.set == LS_SPEC && ls.cls == LEN_TWELVE) e = launch_level_s1_c2(grid, p->stream, items, ls.d_descs);
    else if (ls.set == LS_SPEC) e = launch_level_set1(grid, p->stream, items, ls.d_descs);
    else if (ls.set == LS_OP) e = launch_level_set2(grid, p->stream, items, ls.d_descs);
    else if (ls.set == LS_VJP) e = launch_level_set3(grid, p->stream, items, ls.d_descs);
    else e = launch_level_set0(grid, p->stream, items, ls.d_descs);
    if (e != hipSuccess) return hip_fail(e, "batched level launch");
  }
  return SR_OK;
}

static sr_status batched_levels_gd(sr_plan_s* p, const float* y, float2* x, int iters, const float* eta);

static sr_status batched_levels_gd_trace(sr_plan_s* p, const float* y, float2* x, int iters, const float* eta,
                                        float* loss_trace);

// Level tuner: for each (length, axis) of the plan's level passes that has a
// narrow thread shape, in decreasing order of the grid points it transforms,
// try the narrow shape against the current choice by timing batched GD
// iterations on zeroed stand-ins (best of three runs of six iterations after
// a warm-up), and keep the faster.  Runs once per plan, on its first batched
// solve.  SR_BATCH_EV=0 / 1 pins every length to the default / narrow shape;
// SR_TUNE=0 keeps the defaults.
#define SR_CHECK_B(x)          \
  do {                         \
    sr_status s_ = (x);        \
    if (s_ != SR_OK) return s_; \
  } while (0)

static sr_status batch_tune(sr_plan_s* p) {
  if (p->batch_tuned) return SR_OK;
  p->batch_tuned = true;
  std::map<std::pair<int, int>, double> weight;
  bool any = false;
  for (const Geo& g : p->geo) {
    if (!batch_level_capable(g) || lds_resident(g)) continue;
    any = true;
    if (batch_tile_width(g.M1, 1) != 0) weight[{g.M1, 1}] += (double)g.mg * (g.L + 1);
    if (batch_tile_width(g.M2, 1) != 0) weight[{g.M2, 0}] += (double)g.mg * g.L;
  }
  if (!any || weight.empty()) return SR_OK;
  if (const char* force = std::getenv("SR_BATCH_EV"); force != nullptr) {
    const int v = std::atoi(force) != 0 ? 1 : 0;
    for (const auto& w : weight) p->batch_ev[w.first] = v;
    return SR_OK;
  }
  if (const char* env = std::getenv("SR_TUNE"); env != nullptr && std::atoi(env) == 0) return SR_OK;
  const size_t n_tot = (size_t)p->xoff.back(), m_tot = (size_t)p->yoff.back();
  float2* sx = nullptr;
  float* sy = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    (void)hipStreamSynchronize(p->stream);  // nothing queued may still read the stand-ins
    if (sx) (void)hipFree(sx);
    if (sy) (void)hipFree(sy);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (p->batch) p->batch->key.clear();  // the caller's solve rebuilds its lists
  };
  if (hipMalloc(&sx, std::max<size_t>(n_tot, 1) * sizeof(float2)) != hipSuccess ||
      hipMalloc(&sy, std::max<size_t>(m_tot, 1) * sizeof(float)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    release();
    return SR_OK;  // no room to tune: keep the defaults
  }
  (void)hipMemsetAsync(sx, 0, n_tot * sizeof(float2), p->stream);
  (void)hipMemsetAsync(sy, 0, m_tot * sizeof(float), p->stream);
  const std::vector<float> eta(p->geo.size(), 0.f);
  sr_status st = SR_OK;
  auto time_levels = [&](float* ms) -> sr_status {
    if (p->batch) p->batch->key.clear();  // rebuild the lists under the current shapes
    SR_CHECK_B(batched_levels_gd(p, sy, sx, 2, eta.data()));
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      if (hipEventRecord(e0, p->stream) != hipSuccess) return fail(SR_E_HIP, "tuner event");
      SR_CHECK_B(batched_levels_gd(p, sy, sx, 6, eta.data()));
      if (hipEventRecord(e1, p->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return fail(SR_E_HIP, "tuner event");
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      best = std::min(best, t);
    }
    *ms = best;
    return SR_OK;
  };
  std::vector<std::pair<double, std::pair<int, int>>> order;
  for (const auto& w : weight) order.push_back({-w.second, w.first});
  std::sort(order.begin(), order.end());
  float base = 0.f;
  st = time_levels(&base);
  for (size_t c = 0; c < order.size() && st == SR_OK; ++c) {
    const auto key = order[c].second;
    p->batch_ev[key] = 1;
    float t = 0.f;
    st = time_levels(&t);
    if (st == SR_OK && t < base) base = t;
    else p->batch_ev[key] = 0;
  }
  release();
  return st;
}

sr_status batched_gd(sr_plan_s* p, const float* y, float2* x, int iters, const float* eta, float* loss_trace) {
  if (iters <= 0) return SR_OK;
  if (sr_status t = batch_tune(p); t != SR_OK) return t;
  if (loss_trace != nullptr) return batched_levels_gd_trace(p, y, x, iters, eta, loss_trace);
  std::vector<int> small, rest;
  for (size_t i = 0; i < p->geo.size(); ++i) (lds_resident(p->geo[i]) ? small : rest).push_back((int)i);
  if (rest.empty()) return fused2d_gd(p, small, y, x, iters, eta, p->stream);
  sr_status s = SR_OK;
  if (!small.empty()) {
    // the LDS-resident solves run on the auxiliary stream beside the levels
    if ((s = aux_fork(p)) != SR_OK) return s;
    if ((s = fused2d_gd(p, small, y, x, iters, eta, p->aux_stream)) != SR_OK) return s;
  }
  s = batched_levels_gd(p, y, x, iters, eta);
  if (!small.empty()) {
    sr_status j = aux_join(p);
    if (s == SR_OK) s = j;
  }
  return s;
}

// GD of the problems that are not LDS-resident, one launch per pass level.
// One solve on one group of level sets, on the plan's current stream.
static sr_status levels_gd_run(sr_plan_s* p, const LevelSet& first, const LevelSet& steady, const LevelSet& last,
                               int iters, const std::string& gkey) {
  constexpr int kChunk = 50;
  sr_status s = run_levels(p, first);
  if (s != SR_OK) return s;
  int it = 0;
  if (iters - 1 >= kChunk && graphs_enabled(p)) {
    for (; it + kChunk <= iters - 1; it += kChunk) {
      s = launch_captured(p, gkey, [&]() -> sr_status {
        for (int c = 0; c < kChunk; ++c) {
          sr_status q = run_levels(p, steady);
          if (q != SR_OK) return q;
        }
        return SR_OK;
      });
      if (s != SR_OK) return s;
    }
  }
  for (; it < iters - 1; ++it) {
    s = run_levels(p, steady);
    if (s != SR_OK) return s;
  }
  return run_levels(p, last);
}

static sr_status batched_levels_gd(sr_plan_s* p, const float* y, float2* x, int iters, const float* eta) {
  BatchState* st = nullptr;
  sr_status s = batch_prepare(p, y, x, eta, false, &st);
  if (s != SR_OK) return s;
  if (!st->split) return levels_gd_run(p, st->first, st->steady, st->last, iters, "batch:" + st->key);
  // the two length classes are independent problems: the twelve-element one
  // on the auxiliary stream beside the other (SR_BATCH_STREAMS=1: both on
  // the plan's stream, one after the other)
  const char* ns = std::getenv("SR_BATCH_STREAMS");
  const bool two = st->has[0] && st->has[1] && (ns == nullptr || std::atoi(ns) != 1);
  if (two && (s = aux_fork(p)) != SR_OK) return s;
  for (int c = 0; c < 2 && s == SR_OK; ++c) {
    if (!st->has[c]) continue;
    hipStream_t own = p->stream;
    if (two && c == 1) p->stream = p->aux_stream;
    s = levels_gd_run(p, st->cfirst[c], st->csteady[c], st->clast[c], iters,
                      "batch" + std::to_string(c) + ":" + st->key);
    p->stream = own;
  }
  if (two) {
    const sr_status j = aux_join(p);
    if (s == SR_OK) s = j;
  }
  return s;
}

// GD with a loss trace (no LDS-resident problems: the caller checks): the
// steady iteration's turnaround writes each problem's loss partials, summed
// per problem into the trace after every iteration (no graph: each
// iteration writes another trace entry).
static sr_status batched_levels_gd_trace(sr_plan_s* p, const float* y, float2* x, int iters, const float* eta,
                                        float* loss_trace) {
  BatchState* st = nullptr;
  sr_status s = batch_prepare(p, y, x, eta, true, &st);
  if (s != SR_OK) return s;
  if ((s = run_levels(p, st->first)) != SR_OK) return s;
  const int np = (int)p->geo.size();
  for (int it = 0; it < iters; ++it) {
    if ((s = run_levels(p, it == iters - 1 ? st->last : st->steady)) != SR_OK) return s;
    hipLaunchKernelGGL(batch_loss_reduce, dim3((np + 63) / 64), dim3(64), 0, p->stream, st->parts, st->d_pdesc, np,
                       loss_trace + it, iters);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "loss-trace reduction");
  }
  return SR_OK;
}

// ------------------------------------------------------- derivative levels
// Level lists of recorded derivative passes, for the reverse-mode driver.

struct LevelLists {
  LevelSet ls;
};
LevelLists* level_lists_new() { return new LevelLists(); }
void level_lists_delete(LevelLists* l) { delete l; }
sr_status level_lists_build(sr_plan_s* p, const std::vector<std::vector<PassRecord>>& recs, LevelLists* l) {
  l->ls.set = LS_VJP;
  return build_levels(p, recs, l->ls);
}
sr_status level_lists_run(sr_plan_s* p, const LevelLists* l) { return run_levels(p, l->ls); }
sr_status level_bufs_alloc(sr_plan_s* p) { return level_bufs(p); }

// ------------------------------------------------------------ A and A^H
// One application of A (or A^H) to every listed problem, one launch per pass
// level.  The recorded levels are kept per direction for the last pointers
// they were built for.

sr_status forward_2d_public(sr_plan_s* p, const Geo& g, const float2* x, float2* z, float* y);
sr_status adjoint_2d_public(sr_plan_s* p, const Geo& g, const float2* r, float2* x);

struct OpBatchState {
  std::string key[2];
  LevelSet ls[2];  // [0] A, [1] A^H
};

void destroy_op_batch_state(OpBatchState* s) { delete s; }

sr_status batched_operator(sr_plan_s* p, const std::vector<int>& which, bool adjoint, const float2* in, float2* out,
                           float* y_out) {
  if (sr_status lb = level_bufs(p); lb != SR_OK) return lb;
  OpBatchState* st = p->op_batch;
  if (st == nullptr) {
    st = new OpBatchState();
    p->op_batch = st;
  }
  const int d = adjoint ? 1 : 0;
  std::string key = std::to_string((uintptr_t)in) + ":" + std::to_string((uintptr_t)out) + ":" +
                    std::to_string((uintptr_t)y_out);
  for (int i : which) key += "," + std::to_string(i);
  if (st->key[d] != key) {
    st->key[d].clear();
    const size_t np = p->geo.size();
    std::vector<std::vector<PassRecord>> rec(np);
    float2* saveA = p->bufA;
    float2* saveB = p->bufB;
    sr_status status = SR_OK;
    for (int i : which) {
      if (status != SR_OK) break;
      const Geo& g = p->geo[i];
      p->bufA = p->lvl_bufs + p->lvl_off[i];  // each problem's private ping-pong buffers
      p->bufB = p->lvl_bufs + p->lvl_off[i] + g.mg;
      g_recording = &rec[i];
      if (adjoint)
        status = adjoint_2d_public(p, g, in + p->yoff[i], out + p->xoff[i]);
      else
        status = forward_2d_public(p, g, in + p->xoff[i], out ? out + p->yoff[i] : nullptr,
                                   y_out ? y_out + p->yoff[i] : nullptr);
      g_recording = nullptr;
    }
    p->bufA = saveA;
    p->bufB = saveB;
    if (status != SR_OK) return status;
    st->ls[d].set = LS_OP;
    if ((status = build_levels(p, rec, st->ls[d])) != SR_OK) return status;
    st->key[d] = key;
  }
  return run_levels(p, st->ls[d]);
}

// ------------------------------------------------------------ power iteration
// The same level launches for the power iteration of the problems that are
// not LDS-resident: each problem's recorded passes carry its own sum(y) and
// its own two sets of squared-norm partials (the last pass of iteration it
// reads set it & 1 and writes the other), so one launch per level serves
// every problem.  Seven recordings: the first pass, iteration 0 (reading the
// start vector's single partial), odd and even iterations, each also as the
// final iteration (plain update).

sr_status spec_steady_public(sr_plan_s* p, const Geo& g, const float* y, float2* u, float lam, float inv_mc,
                             const double* ysum, const float* part_in, int npart_in, float* part_out, bool last);

// Set-up and finish of a batched power iteration, one launch each for all
// problems (instead of a few small launches per problem).  Stage 1 reduces
// sum(y_i) and ||v0_i||^2 in the chunks, order and tree of the
// single-problem reductions (so the sums come out the same), copying v0_i to
// x_i on the way; stage 2 sums each problem's stage-1 partials in index
// order.  The finish scales each x_i to sqrt(sum(y_i) / (m c)) u / ||u||
// (Eq. (4)).
struct SpecProb {
  long long yoff, xoff, m, n;  // element offsets and lengths of y_i and x_i
  long long cy, cx;            // stage-1 chunk lengths
  int gy, gx;                  // stage-1 workgroups
  int wy, wx;                  // offsets of the stage-1 partials in the workspace
  int part_off, nq;            // the problem's two partial sets: offset, partials per set
  int idx;                     // problem index in the plan
  float inv_mc;
};

namespace {
constexpr int kSpecRed = 256;

__device__ double spec_block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = kSpecRed / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// grid (max workgroups, problems, 2): z = 0 reduces y_i, z = 1 copies v0_i
// to x_i and reduces its squared magnitudes
__global__ void __launch_bounds__(kSpecRed) spec_setup_stage1(const SpecProb* __restrict__ d, const float* __restrict__ y,
                                                              const float2* __restrict__ v0, float2* __restrict__ x,
                                                              double* __restrict__ ws) {
  __shared__ double red[kSpecRed];
  const SpecProb q = d[blockIdx.y];
  const bool isx = blockIdx.z == 1;
  if ((int)blockIdx.x >= (isx ? q.gx : q.gy)) return;  // (the whole workgroup)
  double acc = 0.0;
  if (!isx) {
    const long long lo = blockIdx.x * q.cy, hi = min(q.m, lo + q.cy);
    for (long long i = lo + threadIdx.x; i < hi; i += kSpecRed) acc += (double)y[q.yoff + i];
  } else {
    const long long lo = blockIdx.x * q.cx, hi = min(q.n, lo + q.cx);
    for (long long i = lo + threadIdx.x; i < hi; i += kSpecRed) {
      const float2 v = v0[q.xoff + i];
      x[q.xoff + i] = v;
      acc += (double)v.x * v.x + (double)v.y * v.y;
    }
  }
  const double s = spec_block_sum(acc, red);
  if (threadIdx.x == 0) ws[(isx ? q.wx : q.wy) + blockIdx.x] = s;
}

// one thread per problem: sum(y_i) into ysum, ||u_0||^2 as the first
// partial set's single partial
__global__ void spec_setup_stage2(const SpecProb* __restrict__ d, int count, const double* __restrict__ ws,
                                  double* ysum, float* parts) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  const SpecProb q = d[j];
  double a = 0.0, b = 0.0;
  for (int k = 0; k < q.gy; ++k) a += ws[q.wy + k];
  for (int k = 0; k < q.gx; ++k) b += ws[q.wx + k];
  ysum[q.idx] = a;
  parts[q.part_off] = (float)b;
}

// grid (workgroups, problems): after `iters` iterations the estimate's
// squared norm is in partial set iters & 1 (a single partial after none)
__global__ void spec_finish(const SpecProb* __restrict__ d, float2* x, const float* __restrict__ parts,
                            const double* __restrict__ ysum, int iters, unsigned* nf) {
  const SpecProb q = d[blockIdx.y];
  const float* P = parts + q.part_off + ((iters & 1) ? max(q.nq, 1) : 0);
  const int np = iters == 0 ? 1 : q.nq;
  double acc = 0.0;
  for (int i = 0; i < np; ++i) acc += (double)P[i];
  const float sc = (float)(sqrt(ysum[q.idx] * (double)q.inv_mc) / sqrt(acc));
  bool bad = false;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < q.n; i += (long long)gridDim.x * blockDim.x) {
    const float2 v = cscale(x[q.xoff + i], sc);
    x[q.xoff + i] = v;
    bad |= !finite2(v);
  }
  flag_nonfinite(nf, bad);
}
}  // namespace

struct SpecSets {
  LevelSet first, it0, it0_last, odd, odd_last, even, even_last;
};

struct SpecBatchState {
  std::string key;
  float* parts = nullptr;              // per problem of the plan: two partial sets
  std::vector<size_t> part_off;
  std::vector<int> nq;                 // partials per set (tiles of the last pass)
  // the level sets: of every problem in cls[0] (split == false), or per
  // length class of the problem (0: both axes a power of two, 1: an axis
  // of twelve-element length), each on its own instantiation and stream
  SpecSets cls[2];
  bool has[2] = {false, false};
  bool split = false;
  SpecProb* d_prob = nullptr;          // the call's problems (set-up and finish)
  double* ws = nullptr;                // their stage-1 partials
  int nprob = 0, gmax = 1, fgroups = 1;
  ~SpecBatchState() {
    if (parts) (void)hipFree(parts);
    if (d_prob) (void)hipFree(d_prob);
    if (ws) (void)hipFree(ws);
  }
};

void destroy_spec_batch_state(SpecBatchState* s) { delete s; }

static float spec_inv_mc(const Geo& g) { return (float)((double)g.mg / (double)g.m); }  // c = 1/(grid size)

static sr_status spec_prepare(sr_plan_s* p, const std::vector<int>& which, const float* y, float2* x, float lam,
                              SpecBatchState** out) {
  std::string key = std::to_string((uintptr_t)y) + ":" + std::to_string((uintptr_t)x);
  {
    uint32_t u;
    std::memcpy(&u, &lam, 4);
    key += ":" + std::to_string(u);
  }
  for (int i : which) key += "," + std::to_string(i);
  if (fused2d_enabled(false)) key += ":r";
  SpecBatchState* st = p->spec_batch;
  if (st != nullptr && st->key == key) {
    *out = st;
    return SR_OK;
  }
  if (sr_status dg = drop_graphs(p, "bspec"); dg != SR_OK) return dg;  // captured over the old lists
  const size_t np = p->geo.size();
  if (sr_status lb = level_bufs(p); lb != SR_OK) return lb;
  if (st == nullptr) {
    st = new SpecBatchState();
    p->spec_batch = st;
    size_t pelems = 0;
    st->part_off.assign(np, 0);
    st->nq.assign(np, 0);
    for (size_t i = 0; i < np; ++i) {
      const Geo& g = p->geo[i];
      st->part_off[i] = pelems;
      if (!batch_level_capable(g)) continue;
      const int bq = batch_tile_width(g.M1, p->bev(g.M1, true));  // the last (column) pass's tiles
      st->nq[i] = (g.N2 + bq - 1) / bq;
      pelems += 2 * (size_t)std::max(st->nq[i], 1);
    }
    if (hipMalloc(&st->parts, std::max<size_t>(pelems, 1) * sizeof(float)) != hipSuccess) {
      st->parts = nullptr;
      return fail(SR_E_NOMEM, "batched power-iteration workspace allocation failed");
    }
  }
  st->key.clear();
  std::vector<std::vector<PassRecord>> r_first(np), r_it0(np), r_it0l(np), r_odd(np), r_oddl(np), r_even(np),
      r_evenl(np);
  float2* saveA = p->bufA;
  float2* saveB = p->bufB;
  sr_status status = SR_OK;
  for (int i : which) {
    if (status != SR_OK) break;
    const Geo& g = p->geo[i];
    p->bufA = p->lvl_bufs + p->lvl_off[i];  // each problem's private ping-pong buffers
    p->bufB = p->lvl_bufs + p->lvl_off[i] + g.mg;
    const float* yi = y + p->yoff[i];
    float2* xi = x + p->xoff[i];
    const double* ys = p->ysum + i;
    float* P0 = st->parts + st->part_off[i];
    float* P1 = P0 + std::max(st->nq[i], 1);
    const float imc = spec_inv_mc(g);
    const int nq = st->nq[i];
    struct Rec {
      std::vector<PassRecord>* r;
      const float* in;
      int npart;
      float* out;
      bool last;
    } recs[6] = {{&r_it0[i], P0, 1, P1, false}, {&r_it0l[i], P0, 1, P1, true}, {&r_odd[i], P1, nq, P0, false},
                 {&r_oddl[i], P1, nq, P0, true}, {&r_even[i], P0, nq, P1, false}, {&r_evenl[i], P0, nq, P1, true}};
    g_recording = &r_first[i];
    status = gd_first_pass_public(p, g, xi);
    for (const Rec& r : recs) {
      if (status != SR_OK) break;
      g_recording = r.r;
      status = spec_steady_public(p, g, yi, xi, lam, imc, ys, r.in, r.npart, r.out, r.last);
    }
    g_recording = nullptr;
  }
  p->bufA = saveA;
  p->bufB = saveB;
  if (status != SR_OK) return status;
  // the call's problems for the set-up and finish launches
  {
    std::vector<SpecProb> dp;
    int woff = 0;
    st->gmax = 1;
    st->fgroups = 1;
    for (int i : which) {
      const Geo& g = p->geo[i];
      SpecProb q{};
      q.yoff = p->yoff[i];
      q.xoff = p->xoff[i];
      q.m = g.m;
      q.n = g.n;
      red_shape(g.m, &q.gy, &q.cy);
      red_shape(g.n, &q.gx, &q.cx);
      q.wy = woff;
      woff += q.gy;
      q.wx = woff;
      woff += q.gx;
      q.part_off = (int)st->part_off[i];
      q.nq = st->nq[i];
      q.idx = i;
      q.inv_mc = spec_inv_mc(g);
      st->gmax = std::max({st->gmax, q.gy, q.gx});
      st->fgroups = std::max(st->fgroups, (int)std::min<int64_t>((g.n + 255) / 256, 1024));
      dp.push_back(q);
    }
    if (st->d_prob != nullptr || st->ws != nullptr) {
      // set-up and finish launches already queued may still read the old ones
      if (hipError_t w = hipStreamSynchronize(p->stream); w != hipSuccess) return hip_fail(w, "stream wait");
    }
    if (st->d_prob) (void)hipFree(st->d_prob);
    if (st->ws) (void)hipFree(st->ws);
    st->d_prob = nullptr;
    st->ws = nullptr;
    st->nprob = (int)dp.size();
    hipError_t e = hipMalloc(&st->d_prob, sizeof(SpecProb) * std::max<size_t>(dp.size(), 1));
    if (e == hipSuccess) e = hipMalloc(&st->ws, sizeof(double) * std::max(woff, 1));
    if (e != hipSuccess) return fail(SR_E_NOMEM, "batched power-iteration workspace allocation failed");
    e = hipMemcpyAsync(st->d_prob, dp.data(), sizeof(SpecProb) * dp.size(), hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);  // dp goes out of scope
    if (e != hipSuccess) return hip_fail(e, "batched power-iteration descriptors");
  }
  // level sets, per length class where the auxiliary stream is free (the
  // LDS-resident problems' solves use it otherwise)
  std::vector<std::vector<PassRecord>>* recsets[7] = {&r_first, &r_it0, &r_it0l, &r_odd, &r_oddl, &r_even, &r_evenl};
  st->split = !batched_any_resident(p);
  st->has[0] = st->has[1] = false;
  for (int c = 0; c < 2; ++c) {
    std::vector<std::vector<PassRecord>> part[7];
    for (int k = 0; k < 7; ++k) part[k].assign(np, {});
    for (int i : which) {
      const Geo& g = p->geo[i];
      const int ci = st->split && (twelve_len(g.M1) || twelve_len(g.M2)) ? 1 : 0;
      if (ci != c) continue;
      for (int k = 0; k < 7; ++k) part[k][i] = (*recsets[k])[i];
      st->has[c] = true;
    }
    if (!st->has[c]) continue;
    SpecSets& S = st->cls[c];
    LevelSet* sets[7] = {&S.first, &S.it0, &S.it0_last, &S.odd, &S.odd_last, &S.even, &S.even_last};
    const int cls = !st->split ? LEN_ALL : c == 0 ? LEN_POW2 : LEN_TWELVE;
    for (int k = 0; k < 7; ++k) {
      sets[k]->set = LS_SPEC;
      sets[k]->cls = cls;
      if ((status = build_levels(p, part[k], *sets[k])) != SR_OK) return status;
    }
  }
  st->key = key;
  *out = st;
  return SR_OK;
}

// The iterations of one group of level sets, on the plan's current stream.
static sr_status spec_run_sets(sr_plan_s* p, const SpecSets& S, int iters, const std::string& gkey) {
  sr_status s = SR_OK;
  if (iters > 0) {
    if ((s = run_levels(p, S.first)) != SR_OK) return s;
    if ((s = run_levels(p, iters == 1 ? S.it0_last : S.it0)) != SR_OK) return s;
  }
  int it = 1;
  constexpr int kChunk = 50;  // even: every chunk starts on an odd iteration
  if (iters - 1 - it >= kChunk && graphs_enabled(p)) {
    for (; it + kChunk <= iters - 1; it += kChunk) {
      s = launch_captured(p, gkey, [&]() -> sr_status {
        for (int c = 0; c < kChunk; ++c) {
          sr_status q = run_levels(p, ((it + c) & 1) ? S.odd : S.even);
          if (q != SR_OK) return q;
        }
        return SR_OK;
      });
      if (s != SR_OK) return s;
    }
  }
  for (; it < iters; ++it) {
    const bool last = it == iters - 1;
    const LevelSet& ls = (it & 1) ? (last ? S.odd_last : S.odd) : (last ? S.even_last : S.even);
    if ((s = run_levels(p, ls)) != SR_OK) return s;
  }
  return SR_OK;
}

sr_status batched_spectral(sr_plan_s* p, const std::vector<int>& which, const float* y, const float2* v0, int iters,
                           float lam, float2* x) {
  if (sr_status t = batch_tune(p); t != SR_OK) return t;  // shapes fixed before any list is built
  SpecBatchState* st = nullptr;
  sr_status s = spec_prepare(p, which, y, x, lam, &st);
  if (s != SR_OK) return s;
  // sum(y), u_0 = v0 and its squared norm (one partial), every problem
  hipLaunchKernelGGL(spec_setup_stage1, dim3(st->gmax, st->nprob, 2), dim3(kSpecRed), 0, p->stream, st->d_prob, y, v0,
                     x, st->ws);
  hipLaunchKernelGGL(spec_setup_stage2, dim3((st->nprob + 63) / 64), dim3(64), 0, p->stream, st->d_prob, st->nprob,
                     st->ws, p->ysum, st->parts);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return hip_fail(e, "power-iteration set-up");
  const bool two = st->split && st->has[0] && st->has[1];
  if (two && (s = aux_fork(p)) != SR_OK) return s;
  for (int c = 0; c < 2 && s == SR_OK; ++c) {
    if (!st->has[c]) continue;
    hipStream_t own = p->stream;
    if (two && c == 1) p->stream = p->aux_stream;
    s = spec_run_sets(p, st->cls[c], iters, "bspec" + std::to_string(c) + ":" + st->key);
    p->stream = own;
  }
  if (two) {
    const sr_status j = aux_join(p);
    if (s == SR_OK) s = j;
  }
  if (s != SR_OK) return s;
  // x0 = sqrt(sum(y)/(m c)) u / ||u||
  hipLaunchKernelGGL(spec_finish, dim3(st->fgroups, st->nprob), dim3(256), 0, p->stream, st->d_prob, x, st->parts,
                     p->ysum, iters, p->sync + 2);
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return hip_fail(e, "power-iteration finish");
  return SR_OK;
}

}  // namespace sr
#endif  // SR_LEVEL_SET
