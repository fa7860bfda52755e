// Runtime dispatch from FFT length to the per-length kernel instantiations.
#include "fused1d.hpp"
#include "launch.hpp"

namespace sr {

#define SR_FOR_EACH_2D_LEN(X) X(16) X(32) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024) X(2048)

hipError_t launch_pass(int N, int kind, bool col, int B, const PassArgs& a, hipStream_t s) {
  const bool rev = kind >= PK_MID_FWD_SAVE && kind <= PK_LAST_ADJ_GT;
  // the reverse-mode passes are built for the default thread shape only, and
  // the wide shape for the column passes [F D F] and [F^H D^* F^H] only: the
  // others run the length's default tile
  if (B <= 0 || (rev && (B & kNarrow))) B = default_tile(N, col);
  if ((B & kWide) && (rev || !col || (kind != PK_MID_FWD && kind != PK_MID_ADJ))) B = default_tile(N, col);
  switch (N) {
#define SR_CASE(n) \
  case n:          \
    return rev ? launch_pass_rev_n<n>(kind, col, B, a, s) : launch_pass_n<n>(kind, col, B, a, s);
    SR_FOR_EACH_2D_LEN(SR_CASE)
#undef SR_CASE
    default:
      return hipErrorInvalidValue;
  }
}

int tile_options(int N, bool col, int* out, int max_out) {
  switch (N) {
#define SR_CASE(n) \
  case n:          \
    return tile_options_n<n>(col, out, max_out);
    SR_FOR_EACH_2D_LEN(SR_CASE)
#undef SR_CASE
    default:
      return 0;
  }
}

// Default tile: the widest column tile (longest contiguous segments) and the
// four-wave row tile.
int default_tile(int N, bool col) {
  int opts[16];
  const int n = tile_options(N, col, opts, 16);
  int best = 1;
  for (int i = 0; i < n; ++i)
    if (opts[i] < kSingleBuffer && opts[i] > best) best = opts[i];  // widest double-buffered tile
  return n > 0 ? best : 1;
}

int pass_groups(int N, bool col, int B, int ntr) {
  if (B <= 0) B = default_tile(N, col);
  B &= kSingleBuffer - 1;
  return (ntr + B - 1) / B;
}

namespace {
template <int N, int OP>
void go1d_batch_op(const Fused1DArgs* as, int count, hipStream_t s) {
  hipLaunchKernelGGL((fused1d_batch_kernel<N, OP>), dim3(count), dim3(F1Tile<N>::THREADS), 0, s, as);
}

template <int N>
hipError_t go1d_batch(int op, const Fused1DArgs* as, int count, hipStream_t s) {
  switch (op) {
    case F1_FORWARD: go1d_batch_op<N, F1_FORWARD>(as, count, s); break;
    case F1_ADJOINT: go1d_batch_op<N, F1_ADJOINT>(as, count, s); break;
    case F1_GD: go1d_batch_op<N, F1_GD>(as, count, s); break;
    case F1_SPECTRAL: go1d_batch_op<N, F1_SPECTRAL>(as, count, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N>
hipError_t go1d(int op, const Fused1DArgs& a, hipStream_t s) {
  constexpr int NT = F1Tile<N>::THREADS;
  switch (op) {
    case F1_FORWARD:
      hipLaunchKernelGGL((fused1d_kernel<N, F1_FORWARD>), dim3(1), dim3(NT), 0, s, a);
      break;
    case F1_ADJOINT:
      hipLaunchKernelGGL((fused1d_kernel<N, F1_ADJOINT>), dim3(1), dim3(NT), 0, s, a);
      break;
    case F1_GD:
      hipLaunchKernelGGL((fused1d_kernel<N, F1_GD>), dim3(1), dim3(NT), 0, s, a);
      break;
    case F1_SPECTRAL:
      hipLaunchKernelGGL((fused1d_kernel<N, F1_SPECTRAL>), dim3(1), dim3(NT), 0, s, a);
      break;
    case F1_FWD_VJP:
      hipLaunchKernelGGL((fused1d_kernel<N, F1_FWD_VJP>), dim3(1), dim3(NT), 0, s, a);
      break;
    case F1_ADJ_VJP:
      hipLaunchKernelGGL((fused1d_kernel<N, F1_ADJ_VJP>), dim3(1), dim3(NT), 0, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

hipError_t launch_fused1d_batch(int m, int op, const Fused1DArgs* dev_args, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  switch (m) {
#define SR_CASE(n) \
  case n:          \
    return go1d_batch<n>(op, dev_args, count, s);
    SR_FOR_EACH_2D_LEN(SR_CASE)
    SR_CASE(4096)
#undef SR_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_fused1d(int m, int op, const Fused1DArgs& a, hipStream_t s) {
  switch (m) {
#define SR_CASE(n) \
  case n:          \
    return go1d<n>(op, a, s);
    SR_FOR_EACH_2D_LEN(SR_CASE)
    SR_CASE(4096)
#undef SR_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace sr
