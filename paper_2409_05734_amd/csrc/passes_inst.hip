// Kernel instantiations for one FFT length, selected by -DSR_FFT_N=<length>.
// SR_PASS_SET=0 builds the operator/solver passes, SR_PASS_SET=1 the
// reverse-mode passes; the build compiles every (length, set) pair as its own
// translation unit so they compile in parallel.
#include "launch.hpp"

#ifndef SR_FFT_N
#error "compile with -DSR_FFT_N=<length>"
#endif
#ifndef SR_PASS_SET
#define SR_PASS_SET 0
#endif

namespace sr {

namespace {

// Tile widths are encoded as B | kSingleBuffer for single-buffered tiles,
// B | kNarrow for the narrow thread shape and B | kWide | kSingleBuffer for
// the wide one.
template <int N, int BE, bool COL, int PRE, int MID, bool FFT2, bool INV1, bool INV2, int POST, bool TAB, bool WIN>
hipError_t go_src(const PassArgs& a, hipStream_t s) {
  constexpr int B = BE & (kSingleBuffer - 1);
  constexpr bool DB = (BE & kSingleBuffer) == 0;
  constexpr int EV = (BE & kNarrow) ? 1 : (BE & kWide) ? 2 : 0;
  using T = TileV<N, B, COL, DB, EV>;
  auto kern = pass_kernel<N, B, COL, PRE, MID, FFT2, INV1, INV2, POST, DB, EV, TAB, WIN>;
  const size_t lds = T::NBUF * sizeof(float2) * (size_t)T::BUF;
  if (lds > 65536) {
    static bool raised = false;  // once per instantiation
    if (!raised) {
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      raised = true;
    }
  }
  const int groups = (a.ntr + B - 1) / B;
  if (groups <= 0) return hipSuccess;
  hipLaunchKernelGGL(kern, dim3(groups), dim3(T::THREADS), lds, s, a);
  return hipGetLastError();
}

// Phase source: the exp(i theta) tables when the pass carries them (they are
// set for every diagonal of a pass or for none), else the phases.
template <int N, int BE, bool COL, int PRE, int MID, bool FFT2, bool INV1, bool INV2, int POST, bool WIN = false>
hipError_t go(const PassArgs& a, hipStream_t s) {
  if constexpr (pass_has_phase<PRE, MID, POST>()) {
    if (a.ep_pre != nullptr || a.ep_mid != nullptr || a.ep_post != nullptr)
      return go_src<N, BE, COL, PRE, MID, FFT2, INV1, INV2, POST, true, WIN>(a, s);
  }
  return go_src<N, BE, COL, PRE, MID, FFT2, INV1, INV2, POST, false, WIN>(a, s);
}

// Shapes that touch the measurement window (the epilogue, the stores of z
// and |z|^2, the adjoint's input): the window-aware build when the window is
// smaller than the grid, else the build that takes the whole grid.
template <int N, int BE, bool COL, int PRE, int MID, bool FFT2, bool INV1, bool INV2, int POST>
hipError_t go_w(const PassArgs& a, hipStream_t s) {
  if (a.crop) return go<N, BE, COL, PRE, MID, FFT2, INV1, INV2, POST, true>(a, s);
  return go<N, BE, COL, PRE, MID, FFT2, INV1, INV2, POST, false>(a, s);
}

template <int N, bool COL, int B>  // B: encoded tile width
hipError_t dispatch(int kind, const PassArgs& a, hipStream_t s) {
#if SR_PASS_SET == 0
  if constexpr (COL) {
    switch (kind) {
      case PK_FIRST_FWD:
        return go<N, B, COL, PRE_PHASE, MID_NONE, false, false, false, POST_STORE>(a, s);
      case PK_LAST_ADJ:
        return go<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_PHASE_CONJ_STORE>(a, s);
      case PK_LAST_GD:
        return go<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_GD>(a, s);
      case PK_LAST_SPEC:
        return go<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_SPEC>(a, s);
      case PK_LAST_GD_FWD:
        return go<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_GD_FWD>(a, s);
      case PK_LAST_SPEC_FWD:
        return go<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_SPEC_FWD>(a, s);
      default:
        break;
    }
  }
  switch (kind) {
    case PK_MID_FWD:
      return go<N, B, COL, PRE_NONE, MID_PHASE, true, false, false, POST_STORE>(a, s);
    case PK_LAST_STORE:
      return go_w<N, B, COL, PRE_NONE, MID_STORE, false, false, false, POST_STORE>(a, s);
    case PK_TURN_GD:
      return go_w<N, B, COL, PRE_NONE, MID_GD, true, false, true, POST_STORE>(a, s);
    case PK_TURN_GD_POIS:
      return go_w<N, B, COL, PRE_NONE, MID_GD_POIS, true, false, true, POST_STORE>(a, s);
    case PK_TURN_SPEC:
      return go_w<N, B, COL, PRE_NONE, MID_SPEC, true, false, true, POST_STORE>(a, s);
    case PK_FIRST_ADJ:
      return go_w<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_STORE>(a, s);
    case PK_MID_ADJ:
      return go<N, B, COL, PRE_NONE, MID_PHASE_CONJ, true, true, true, POST_STORE>(a, s);
    default:
      return hipErrorInvalidValue;
  }
#else
  if constexpr (COL) {
    if (kind == PK_LAST_ADJ_GT)
      return go<N, B, COL, PRE_NONE, MID_NONE, false, true, false, POST_PHASE_CONJ_GT>(a, s);
  }
  switch (kind) {
    case PK_MID_FWD_SAVE:
      return go<N, B, COL, PRE_NONE, MID_PHASE_SAVE, true, false, false, POST_STORE>(a, s);
    case PK_MID_ADJ_GT:
      return go<N, B, COL, PRE_NONE, MID_PHASE_CONJ_GT, true, true, true, POST_STORE>(a, s);
    case PK_MID_ADJ_SAVE:
      return go<N, B, COL, PRE_NONE, MID_PHASE_CONJ_SAVE, true, true, true, POST_STORE>(a, s);
    case PK_MID_FWD_GT:
      return go<N, B, COL, PRE_NONE, MID_PHASE_GT, true, false, false, POST_STORE>(a, s);
    default:
      return hipErrorInvalidValue;
  }
#endif
}

using Cfg = TileCfg<SR_FFT_N>;
// narrow shapes are built for the operator/solver passes only (the reverse-
// mode passes run on the default shape of the same tile width)
constexpr bool kHasNarrow = HasNarrow<SR_FFT_N>::value && SR_PASS_SET == 0;
using CfgN = TileCfg<SR_FFT_N, kHasNarrow ? 1 : 0>;
constexpr int kColOpts[4] = {2, 4, 8, 16};
// the wide shape: the column passes with two transforms and a phase between
// them ([F D F] and [F^H D^* F^H]), eight-column single-buffered tiles
constexpr bool kHasWide = HasWide<SR_FFT_N>::value && SR_PASS_SET == 0;
constexpr int kWideCols = 8;
template <int N, int EV>
constexpr bool wide_fits() {
  if constexpr (EV == 2 && HasWide<N>::value) {
    using T = TileV<N, kWideCols, true, false, 2>;
    return T::THREADS <= 1024 && sizeof(float2) * T::BUF <= (size_t)TileCfg<N>::kMaxLds;
  } else {
    return false;
  }
}

template <int N, int B>
hipError_t col_tile(int kind, bool single, bool narrow, const PassArgs& a, hipStream_t s) {
  if (narrow) {
    if constexpr (kHasNarrow && CfgN::col_ok(B)) return dispatch<N, true, B | kNarrow>(kind, a, s);
  } else if (single) {
    if constexpr (Cfg::col_sb_ok(B)) return dispatch<N, true, B | kSingleBuffer>(kind, a, s);
  } else {
    if constexpr (Cfg::col_ok(B)) return dispatch<N, true, B>(kind, a, s);
  }
  return hipErrorInvalidValue;
}

template <int N>
hipError_t by_tile(int kind, bool col, int Benc, const PassArgs& a, hipStream_t s) {
  if (Benc & kWide) {
    // (only the two shapes below are built wide; the same template arguments
    // as dispatch() gives these kinds)
    if constexpr (kHasWide && wide_fits<N, 2>()) {
      constexpr int W = kWideCols | kWide | kSingleBuffer;
      if (col && Benc == W && kind == PK_MID_FWD)
        return go<N, W, true, PRE_NONE, MID_PHASE, true, false, false, POST_STORE>(a, s);
      if (col && Benc == W && kind == PK_MID_ADJ)
        return go<N, W, true, PRE_NONE, MID_PHASE_CONJ, true, true, true, POST_STORE>(a, s);
    }
    return hipErrorInvalidValue;
  }
  const bool narrow = (Benc & kNarrow) != 0;
  if (col) {
    const bool single = (Benc & kSingleBuffer) != 0;
    if (single && narrow) return hipErrorInvalidValue;
    switch (Benc & (kSingleBuffer - 1)) {
      case 2: return col_tile<N, 2>(kind, single, narrow, a, s);
      case 4: return col_tile<N, 4>(kind, single, narrow, a, s);
      case 8: return col_tile<N, 8>(kind, single, narrow, a, s);
      case 16: return col_tile<N, 16>(kind, single, narrow, a, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (narrow) {
    if constexpr (kHasNarrow) {
      const int B = Benc & ~kNarrow;
      if (B == CfgN::ROW_SMALL) return dispatch<N, false, CfgN::ROW_SMALL | kNarrow>(kind, a, s);
      if constexpr (CfgN::ROW_BIG != CfgN::ROW_SMALL) {
        if (B == CfgN::ROW_BIG) return dispatch<N, false, CfgN::ROW_BIG | kNarrow>(kind, a, s);
      }
    }
    return hipErrorInvalidValue;
  }
  if (Benc & kSingleBuffer) {
    const int B = Benc & ~kSingleBuffer;
    if constexpr (Cfg::row_sb_ok(Cfg::ROW_SMALL)) {
      if (B == Cfg::ROW_SMALL) return dispatch<N, false, Cfg::ROW_SMALL | kSingleBuffer>(kind, a, s);
    }
    if constexpr (Cfg::ROW_BIG != Cfg::ROW_SMALL && Cfg::row_sb_ok(Cfg::ROW_BIG)) {
      if (B == Cfg::ROW_BIG) return dispatch<N, false, Cfg::ROW_BIG | kSingleBuffer>(kind, a, s);
    }
    return hipErrorInvalidValue;
  }
  const int B = Benc;
  if (B == Cfg::ROW_SMALL) return dispatch<N, false, Cfg::ROW_SMALL>(kind, a, s);
  if constexpr (Cfg::ROW_BIG != Cfg::ROW_SMALL) {
    if (B == Cfg::ROW_BIG) return dispatch<N, false, Cfg::ROW_BIG>(kind, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

#if SR_PASS_SET == 0
template <>
int tile_options_n<SR_FFT_N>(bool col, int* out, int max_out) {
  int n = 0;
  if (col) {
    for (int b : kColOpts)
      if (Cfg::col_ok(b) && n < max_out) out[n++] = b;
    for (int b : kColOpts)
      if (Cfg::col_sb_ok(b) && n < max_out) out[n++] = b | kSingleBuffer;
    if (kHasNarrow)
      for (int b : kColOpts)
        if (CfgN::col_ok(b) && n < max_out) out[n++] = b | kNarrow;
    if constexpr (kHasWide && wide_fits<SR_FFT_N, 2>())
      if (n < max_out) out[n++] = kWideCols | kWide | kSingleBuffer;
  } else {
    if (n < max_out) out[n++] = Cfg::ROW_SMALL;
    if (Cfg::ROW_BIG != Cfg::ROW_SMALL && n < max_out) out[n++] = Cfg::ROW_BIG;
    if (Cfg::row_sb_ok(Cfg::ROW_SMALL) && n < max_out) out[n++] = Cfg::ROW_SMALL | kSingleBuffer;
    if (Cfg::ROW_BIG != Cfg::ROW_SMALL && Cfg::row_sb_ok(Cfg::ROW_BIG) && n < max_out)
      out[n++] = Cfg::ROW_BIG | kSingleBuffer;
    if (kHasNarrow) {
      if (n < max_out) out[n++] = CfgN::ROW_SMALL | kNarrow;
      if (CfgN::ROW_BIG != CfgN::ROW_SMALL && n < max_out) out[n++] = CfgN::ROW_BIG | kNarrow;
    }
  }
  return n;
}

template <>
hipError_t launch_pass_n<SR_FFT_N>(int kind, bool col, int B, const PassArgs& a, hipStream_t s) {
  return by_tile<SR_FFT_N>(kind, col, B, a, s);
}
#else
template <>
hipError_t launch_pass_rev_n<SR_FFT_N>(int kind, bool col, int B, const PassArgs& a, hipStream_t s) {
  return by_tile<SR_FFT_N>(kind, col, B, a, s);
}
#endif

}  // namespace sr
