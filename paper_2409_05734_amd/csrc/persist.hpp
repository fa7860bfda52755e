// Persistent single-launch solver for 2D problems on square grids: every
// iteration of a GD or spectral solve runs inside one cooperative launch, the
// fused passes separated by grid-wide barriers instead of kernel boundaries.
#pragma once
#include "passes.hpp"

namespace sr {

constexpr int kMaxPersistPasses = 9;  // 2L+1 passes, L <= 4

enum PersistOp : int { PO_GD = 0, PO_SPEC = 1 };

struct PersistArgs {
  PassArgs pass[kMaxPersistPasses];
  int kind[kMaxPersistPasses];
  int col[kMaxPersistPasses];
  int npass;
  int iters;
  unsigned* bar;      // monotonic arrival counter, zero at launch
  int* err;           // set to 1 if a barrier wait exceeded its bound
  // spectral: partial sums alternate between part_base and part_base + part_cap
  float* part_base;
  int part_cap;
  int npart0;         // partial count of the start vector's norm
  int npart_iter;     // partial count written by the last pass
  // GD loss trace: partials of pass `loss_pass` (loss_nparts of them)
  float* loss_trace;
  int loss_pass;
  int loss_nparts;
};

// Grid-wide barrier on a monotonic counter: block arrives, then waits until
// the counter reaches `target` (= number of barriers so far x grid size).
// The wait is bounded; on timeout (or if another block timed out) the error
// flag is set and every thread of the block gets `false`, so all waves exit.
constexpr unsigned kSpinLimit = 1u << 22;  // s_sleep(2) polls: well over a second

__device__ __forceinline__ bool grid_sync(unsigned* bar, unsigned target, int* err) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = 1;
    __threadfence();  // release this block's global writes
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kSpinLimit || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
    }
    __threadfence();  // acquire the other blocks' writes
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

template <int N, int B, bool COL, int OP>
__device__ __forceinline__ void persist_tile(const PassArgs& a, int kind, int tile, float2* lds, float* red,
                                             const float* part_in, int npart, float* part_out) {
  if constexpr (COL) {
    switch (kind) {
      case PK_FIRST_FWD:
        pass_tile_rt<N, B, COL, PRE_PHASE, MID_NONE, false, false, false, POST_STORE>(a, tile, lds, red, part_in, npart,
                                                                                   part_out);
        return;
      case PK_LAST_GD:
        if constexpr (OP == PO_GD)
          pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_GD>(a, tile, lds, red, part_in, npart,
                                                                                part_out);
        return;
      case PK_LAST_SPEC:
        if constexpr (OP == PO_SPEC)
          pass_tile_rt<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_SPEC>(a, tile, lds, red, part_in, npart,
                                                                                  part_out);
        return;
      default:
        break;
    }
  }
  switch (kind) {
    case PK_MID_FWD:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE, true, false, false, POST_STORE>(a, tile, lds, red, part_in, npart,
                                                                                part_out);
      return;
    case PK_TURN_GD:
      if constexpr (OP == PO_GD)
        pass_tile_rt<N, B, COL, PRE_NONE, MID_GD, true, false, true, POST_STORE>(a, tile, lds, red, part_in, npart,
                                                                              part_out);
      return;
    case PK_TURN_SPEC:
      if constexpr (OP == PO_SPEC)
        pass_tile_rt<N, B, COL, PRE_NONE, MID_SPEC, true, false, true, POST_STORE>(a, tile, lds, red, part_in, npart,
                                                                                part_out);
      return;
    case PK_MID_ADJ:
      pass_tile_rt<N, B, COL, PRE_NONE, MID_PHASE_CONJ, true, true, true, POST_STORE>(a, tile, lds, red, part_in, npart,
                                                                                   part_out);
      return;
    default:
      return;
  }
}

template <int N, int B, int OP>
__global__ void __launch_bounds__((Tile<N, B, true>::THREADS)) persistent_kernel(const PersistArgs pa) {
  static_assert(Tile<N, B, true>::THREADS == Tile<N, B, false>::THREADS, "row and column tiles must match");
  extern __shared__ float2 lds[];
  __shared__ float red[Tile<N, B, true>::THREADS];
  unsigned target = 0;
  for (int it = 0; it < pa.iters; ++it) {
    float* pin = nullptr;
    float* pout = nullptr;
    int npin = 0;
    if constexpr (OP == PO_SPEC) {
      pin = pa.part_base + (it & 1) * pa.part_cap;
      pout = pa.part_base + ((it + 1) & 1) * pa.part_cap;
      npin = it == 0 ? pa.npart0 : pa.npart_iter;
    }
    for (int p = 0; p < pa.npass; ++p) {
      const PassArgs& a = pa.pass[p];
      const int kind = pa.kind[p];
      const int ntiles = (a.ntr + B - 1) / B;
      const float* part_in = nullptr;
      float* part_out = nullptr;
      if constexpr (OP == PO_SPEC) {
        if (kind == PK_LAST_SPEC) part_in = pin;  // normalisation is applied in the last pass
        if (kind == PK_LAST_SPEC) part_out = pout;
      } else {
        if (p == pa.loss_pass && pa.loss_trace != nullptr) part_out = pa.part_base;
      }
      for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        __syncthreads();  // LDS reuse between consecutive tiles
        if (pa.col[p]) persist_tile<N, B, true, OP>(a, kind, tile, lds, red, part_in, npin, part_out);
        else persist_tile<N, B, false, OP>(a, kind, tile, lds, red, part_in, npin, part_out);
      }
      target += gridDim.x;
      if (!grid_sync(pa.bar, target, pa.err)) return;
      if constexpr (OP == PO_GD) {
        if (p == pa.loss_pass && pa.loss_trace != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
          double acc = 0.0;
          for (int i = 0; i < pa.loss_nparts; ++i) acc += (double)pa.part_base[i];
          pa.loss_trace[it] = (float)acc;
        }
      }
    }
  }
}

}  // namespace sr
