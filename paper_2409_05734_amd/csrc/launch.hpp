// Host-side launch interface between the plan logic and the per-length
// kernel translation units (one object file per FFT length).
#pragma once
#include <hip/hip_runtime.h>

#include "passes.hpp"

namespace sr {

// The fused pass shapes used by the operator and the solvers.
enum PassKind : int {
  PK_FIRST_FWD = 0,   // [U, D_1, F_0]           column mode over the support columns
  PK_MID_FWD = 1,     // [F_a, D_k, F_a]
  PK_LAST_STORE = 2,  // [F_a -> z, |z|^2]
  PK_TURN_GD = 3,     // [F_a -> (|z|^2 - y) z -> F_a^H]
  PK_TURN_SPEC = 4,   // [F_a -> T(y) z -> F_a^H]
  PK_FIRST_ADJ = 5,   // [F_a^H]
  PK_MID_ADJ = 6,     // [F_a^H, D_k^*, F_a^H]
  PK_LAST_ADJ = 7,    // [F_0^H, D_1^*, U^H]      column mode over the support columns
  PK_LAST_GD = 8,     // ... then x <- x - step * g
  PK_LAST_SPEC = 9,   // ... then u <- step * g - 2 lambda u/||u|| (+ norm partials)
  // reverse mode (derivatives with respect to the phases)
  PK_MID_FWD_SAVE = 10,  // (kinds 10..14 live in the reverse-mode kernel set)  // [F_a, D_k (save u_k), F_a]
  PK_MID_ADJ_GT = 11,    // [F_a^H, gth_k += Im(u conj(u_k)), D_k^*, F_a^H]
  PK_MID_ADJ_SAVE = 12,  // [F_a^H, D_k^* (save q_k), F_a^H]
  PK_MID_FWD_GT = 13,    // [F_a, gth_k += Im(conj(q) q_k), D_k, F_a]
  PK_LAST_ADJ_GT = 14,   // [F_0^H, gth_1 += Im(u conj(D_1 U x)), D_1^*, U^H]
  // GD / spectral update fused with the next iteration's [U, D_1, F_0]
  PK_LAST_GD_FWD = 15,
  PK_LAST_SPEC_FWD = 16,
  PK_TURN_GD_POIS = 17,  // [F_a -> (1 - y/(|z|^2 + eps)) z -> F_a^H]  (Poisson loss)
  PK_COUNT = 18
};

// Tile widths: each length is compiled for a few tile widths (transforms per
// workgroup) and, for power-of-two lengths 64..1024, two thread shapes in
// each mode; the plan's tuner picks one per (length, mode).
// Row mode: 1 wave or 4 waves per workgroup.  Column mode: 2, 4, 8 or 16
// adjacent columns (16- to 128-byte row segments), within 1024 threads and
// the LDS budget (double-buffered tiles, and single-buffered ones where they
// raise occupancy).
template <int N, int EV = 0>
struct TileCfg {
  static constexpr int TPT = TileV<N, 1, true, true, EV>::TPT;
  static constexpr int NP = TileV<N, 1, true, true, EV>::NP;  // padded length in LDS
  static constexpr int lds_bytes(int b) { return 2 * b * NP * 8; }  // double-buffered tile
  static constexpr int kMaxLds = 152 * 1024;  // dynamic LDS per workgroup (160 KB minus static)
  static constexpr bool col_ok(int b) { return b * TPT <= 1024 && lds_bytes(b) <= kMaxLds; }
  static constexpr bool row_ok(int b) { return b >= 1 && b * TPT <= 1024 && lds_bytes(b) <= 65536; }
  // single-buffered tiles (half the LDS, two barriers per stage): offered
  // where the double-buffered tile of the same width needs 32 KB or more, so
  // that halving it raises the number of workgroups a CU holds
  static constexpr bool sb_ok(int b) { return b * TPT <= 1024 && lds_bytes(b) >= 32768 && lds_bytes(b) / 2 <= kMaxLds; }
  static constexpr bool col_sb_ok(int b) { return sb_ok(b); }
  static constexpr bool row_sb_ok(int b) { return sb_ok(b); }
  static constexpr int ROW_SMALL = TPT >= 64 ? 1 : 64 / TPT;   // one wave
  static constexpr int ROW_BIG = TPT >= 256 ? 1 : 256 / TPT;   // four waves
};

// Tile widths available for a length and mode, and the default.  Column
// widths with bit 256 set are single-buffered variants; widths with bit 512
// set use the narrow shape (four elements per thread), bit 1024 the wide
// one (sixteen).
int tile_options(int N, bool col, int* out, int max_out);
int default_tile(int N, bool col);

constexpr int kSingleBuffer = 256;
constexpr int kNarrow = 512;
constexpr int kWide = 1024;  // sixteen elements per thread, radix-16 stages (single-buffered columns)

// Number of workgroups a pass of this length/mode/tile launches.
int pass_groups(int N, bool col, int B, int ntr);

// Launch one fused pass with tile width B (0 = default).  Returns the launch
// error, or hipErrorInvalidValue for an unsupported length or tile width.
hipError_t launch_pass(int N, int kind, bool col, int B, const PassArgs& a, hipStream_t s);

// Per-length entry points, each defined in its own translation unit.
template <int N>
hipError_t launch_pass_n(int kind, bool col, int B, const PassArgs& a, hipStream_t s);
template <int N>
hipError_t launch_pass_rev_n(int kind, bool col, int B, const PassArgs& a, hipStream_t s);
template <int N>
int tile_options_n(bool col, int* out, int max_out);

// 1D LDS-resident kernels (fused1d.hpp)
struct Fused1DArgs;
hipError_t launch_fused1d(int m, int op, const Fused1DArgs& a, hipStream_t s);
// many problems of grid length m, one workgroup each (device argument array)
hipError_t launch_fused1d_batch(int m, int op, const Fused1DArgs* dev_args, int count, hipStream_t s);

}  // namespace sr

namespace sr {
struct PersistArgs;
bool persistent_supported(int N, int B);
// Cooperative launch of a whole GD (op 0) or spectral (op 1) solve; `grid`
// is clamped to the number of co-resident workgroups.
hipError_t launch_persistent(int N, int B, int op, const PersistArgs& pa, int grid, hipStream_t s);
}  // namespace sr
