// Plan object shared by the host-side translation units of libsrpr.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/sr.h"

namespace sr {

// Geometry of one problem.  The transforms run on an M1 x M2 grid with
// M_k = max(N_k, W_k) per axis: the N1 x N2 signal is zero-padded into the
// centred window at (o1, o2) (oversampling, U) and the W1 x W2 measurements
// are the centred window at (c1, c2) (undersampling, S; the whole grid when
// W = M).  1D problems use the first axis only (N2 = M2 = W2 = 1).
struct Geo {
  int ndim = 0;
  int N1 = 1, N2 = 1, M1 = 1, M2 = 1;
  int o1 = 0, o2 = 0;
  int W1 = 1, W2 = 1;
  int c1 = 0, c2 = 0;
  int L = 0;
  int64_t n = 0;   // signal entries
  int64_t m = 0;   // measurements (W1 W2)
  int64_t mg = 0;  // grid entries (M1 M2); the phases of one layer
  int64_t th_off = 0;
  bool cropped() const { return W1 != M1 || W2 != M2; }
};

sr_status fail(sr_status s, const std::string& msg);
sr_status hip_fail(hipError_t e, const char* what);

}  // namespace sr

namespace sr {
struct BatchState;
void destroy_batch_state(BatchState* s);
struct SpecBatchState;
void destroy_spec_batch_state(SpecBatchState* s);
struct OpBatchState;
void destroy_op_batch_state(OpBatchState* s);
struct VjpBatchState;
void destroy_vjp_batch_state(VjpBatchState* s);
struct DenseLib;
void destroy_dense_lib(DenseLib* d);

// A stack of problems of one geometry run as one: every fused pass of the
// first problem's schedule is launched once for all P problems, each buffer
// the pass touches registered with its per-problem stride (problem s's data
// sits s * stride elements after problem 0's).
struct StackRegion {
  uintptr_t lo, hi;  // problem 0's bytes
  int stride;        // elements between consecutive problems
};
struct StackState {
  int P = 1;          // problems in the stack (1: no stack)
  int th_stride = 0;  // elements between the problems' phase blocks (0: shared)
  const float* steps = nullptr;  // device: each problem's GD step (GD on a stack)
  std::vector<StackRegion> regions;
  void add(const void* base, size_t elems, size_t elem_bytes, int stride) {
    const uintptr_t lo = (uintptr_t)base;
    regions.push_back({lo, lo + elems * elem_bytes, stride});
  }
  // stride of the buffer `ptr` points into; false if no region holds it
  bool stride_of(const void* ptr, int* stride) const {
    if (ptr == nullptr) {
      *stride = 0;
      return true;
    }
    const uintptr_t q = (uintptr_t)ptr;
    for (const StackRegion& r : regions)
      if (q >= r.lo && q < r.hi) {
        *stride = r.stride;
        return true;
      }
    return false;
  }
};
}  // namespace sr

struct sr_plan_s {
  std::vector<sr::Geo> geo;
  int kind = SR_STRUCTURED;
  hipStream_t stream = nullptr;
  std::vector<int64_t> xoff, yoff;  // concatenation offsets (complex elements)

  float* theta = nullptr;  // device copy of the phases
  float2* eph = nullptr;   // exp(i theta), same layout (filled on device)
  bool use_table = false;  // passes read eph instead of evaluating sincos(theta)
  int64_t theta_len = 0;
  const float2* dense_A = nullptr;  // caller-owned dense matrix (SR_DENSE)
  sr::DenseLib* dense_lib = nullptr;  // library GEMM state of a dense plan (null: hand-written products only)

  std::map<std::pair<int, int>, float2*> tw;  // (FFT length, thread shape) -> device twiddle table
  float2* twbuf = nullptr;

  // workspace carved out of one allocation
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool ws_owned = true;  // false once the caller's memory holds the workspace
  float2* bufA = nullptr;  // ping-pong pass buffers (max m complex each)
  float2* bufB = nullptr;
  float2* bufC = nullptr;  // extra grid buffers for derivatives
  float2* bufD = nullptr;
  float* part = nullptr;   // 2 x part_cap partial sums
  int part_cap = 0;
  double* ysum = nullptr;  // sum(y) scratch (per problem)
  float* fscratch = nullptr;  // float scratch (dense solver scalars)
  float* dsplit = nullptr;    // dense plans: split-reduction partial products
  unsigned* sync = nullptr;   // [0] grid-barrier counter, [1] barrier error flag, [2] non-finite flag
  double* red_ws = nullptr;   // per-workgroup partials of the two-stage reductions (kRedGroups)
  float2* vjp_buf = nullptr;  // per-layer intermediates for derivatives (allocated on first use)
  sr::StackState stk;         // the stack being run (P = 1 outside stacked calls)
  float2* stk_buf = nullptr;  // stacked ping-pong buffers (allocated on first stacked call)
  size_t stk_elems = 0;
  float* stk_gth = nullptr;   // per-problem phase cotangents of a stack sharing its phases
  size_t stk_gth_elems = 0;
  float* stk_part = nullptr;           // squared-norm partials of a stacked spectral solve (2 sets)
  size_t stk_part_elems = 0;
  float* stk_steps = nullptr;          // device: per-problem GD steps of a stack
  int stk_steps_cap = 0;
  sr::BatchState* batch = nullptr;  // batched-schedule state (built on first batched solve)
  sr::SpecBatchState* spec_batch = nullptr;  // the same for batched power iteration
  sr::OpBatchState* op_batch = nullptr;      // and for batched A / A^H
  sr::VjpBatchState* vjp_batch = nullptr;    // and for the batched derivatives
  float2* lvl_bufs = nullptr;                // their shared per-problem ping-pong buffers
  // GD-step and intensity derivatives (vjp.hip): z, r, rbar (measurement
  // layout) and two signal-layout temporaries, allocated on first use; a
  // device copy of the concatenation offsets and the per-problem step scales
  float2* gstep_buf = nullptr;
  int64_t* d_off = nullptr;  // x offsets (nprob + 1), then y offsets (nprob + 1)
  float* d_scale = nullptr;  // nprob per-problem factors
  std::vector<size_t> lvl_off;
  size_t vjp_elems = 0;

  // LDS-resident small-problem solver (fused2d.hip): device descriptors, their
  // host staging copy, and a second stream (with fork/join events) so that it
  // runs beside the batched level launches of the larger problems
  void* f1_args = nullptr;  // batched 1D launches: device argument array and its host staging copy
  size_t f1_cap = 0;
  std::vector<unsigned char> f1_host;
  void* f2_descs = nullptr;
  size_t f2_desc_cap = 0;
  std::vector<unsigned char> f2_host;
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  int device = 0;  // the GPU the plan was created on (current device at sr_plan_create)
  int schedule = SR_SCHED_AUTO;
  int loss = SR_LOSS_L2;  // GD loss (sr_plan_set_loss) and its Poisson guard
  float loss_eps = 0.f;
  hipStream_t cap_stream = nullptr;  // private stream used only to capture graphs
  std::vector<std::pair<std::string, hipGraphExec_t>> graphs;  // captured solver chunks (most recent last)
  std::map<std::pair<int, int>, int> tiles;  // (FFT length, column mode) -> tuned tile width
  // level kernel (batched schedule): (FFT length, column mode) -> thread shape
  // of the GD and power-iteration passes (0 default, 1 narrow), tuned on the
  // first batched solve
  std::map<std::pair<int, int>, int> batch_ev;
  bool batch_tuned = false;
  int bev(int N, bool col) const {
    auto it = batch_ev.find({N, col ? 1 : 0});
    return it == batch_ev.end() ? 0 : it->second;
  }

  int tile(int N, bool col) const {
    auto it = tiles.find({N, col ? 1 : 0});
    return it == tiles.end() ? 0 : it->second;
  }

  sr_status init(const float* theta_host);
  const float2* twiddles(int N, int shape = 0) const;
  const float* theta_l(const sr::Geo& g, int l) const;
  ~sr_plan_s();
};

namespace sr {

// util_kernels.hip
// sum of n partials into *out (count > 1: that many sets of n end to end,
// set t into out[t * ostride])
sr_status reduce_partials(sr_plan_s* p, const float* part, int n, float* out, int count = 1, int ostride = 0);
// (count > 1: that many arrays of n elements end to end, each on its own)
// stage-1 shape of the deterministic reductions of n elements: workgroups
// and the contiguous chunk each one sums
void red_shape(long long n, int* groups, long long* chunk);
sr_status sum_floats(sr_plan_s* p, const float* y, int64_t n, double* out, int count = 1);
sr_status norm2_partial(sr_plan_s* p, const float2* x, int64_t n, float* out, int count = 1);
sr_status final_scale(sr_plan_s* p, float2* x, int64_t n, const float* part, int npart, const double* ysum,
                      float inv_mc, int count = 1);
sr_status fill_phase_table(sr_plan_s* p);
// count host floats into device memory, stream-ordered, through kernel
// arguments (the host array is free on return; no wait on the stream)
sr_status put_floats(sr_plan_s* p, float* dst, const float* host, int count);

// dense.hip (i.i.d. complex Gaussian baseline)
size_t dense_split_floats(int m, int n, int nb);
sr_status dense_forward(sr_plan_s* p, const float2* x, float2* z, float* y);
sr_status dense_adjoint(sr_plan_s* p, const float2* r, float2* x);
sr_status dense_gd(sr_plan_s* p, const float* y, float2* x, int iters, const float* eta, float* loss_trace);
sr_status dense_spectral(sr_plan_s* p, const float* y, const float2* v0, int iters, float lam, float2* x0);
// hipBLASLt for the dense products where it is faster (timed per product at
// plan creation; SR_DENSE_GEMM=own / lib pins the choice)
sr_status dense_lib_setup(sr_plan_s* p);

// fused2d.hip (LDS-resident solves of small 2D problems, one workgroup each)
// SR_LDS_RESIDENT=1 / 0 turns the LDS-resident solver on / off for batched
// plans; unset, the caller's default applies (off for GD, where the level
// launches are as fast; on for the power iteration, where it is slightly
// faster beside the level launches of the larger problems).
bool fused2d_enabled(bool by_default);
bool fused2d_supported(const Geo& g);
sr_status fused2d_gd(sr_plan_s* p, const std::vector<int>& which, const float* y, float2* x, int iters,
                     const float* eta, hipStream_t s);
sr_status fused2d_spectral(sr_plan_s* p, const std::vector<int>& which, const float* y, const float2* v0, int iters,
                           float lam, float2* x0, hipStream_t s);
// fork the aux stream off the plan stream / join it back
sr_status aux_fork(sr_plan_s* p);
sr_status aux_join(sr_plan_s* p);

// batched.hip (many problems advanced one pass level per launch)
bool batched_supported(const sr_plan_s* p);
// (loss_trace: nullable; with it, no problem may be LDS-resident)
sr_status batched_gd(sr_plan_s* p, const float* y, float2* x, int iters, const float* eta,
                     float* loss_trace = nullptr);
bool batched_any_resident(const sr_plan_s* p);
// power iteration of the listed problems by level launches (2D problems
// whose lengths the level kernel covers)
bool batch_level_capable(const Geo& g);
// one application of A (adjoint: A^H) to the listed problems by level launches
sr_status batched_operator(sr_plan_s* p, const std::vector<int>& which, bool adjoint, const float2* in, float2* out,
                           float* y_out);
sr_status batched_spectral(sr_plan_s* p, const std::vector<int>& which, const float* y, const float2* v0, int iters,
                           float lam, float2* x);

// vjp.hip (reverse-mode derivatives of A and A^H)
sr_status vjp_forward(sr_plan_s* p, const float2* x, const float2* gz, float2* gx, float* gtheta);
sr_status vjp_adjoint(sr_plan_s* p, const float2* r, const float2* gv, float2* gr, float* gtheta);
// one GD step's reverse (l2 loss) and the reverse of y = |A x|^2
sr_status gd_step_vjp(sr_plan_s* p, const float* y, const float2* x, const float* eta_host, const float2* gxn,
                      float2* gx, float* gy, float* gtheta);
sr_status intensity_vjp(sr_plan_s* p, const float2* x, const float* gy, float2* gx, float* gtheta);

}  // namespace sr
