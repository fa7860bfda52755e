// Device-side FFT core for gfx950: complex helpers, radix butterflies and a
// register/LDS Stockham transform over a tile of B independent length-N
// transforms.
//
// Layout contract ("canonical" register layout): the TPT = N/E threads of one
// transform each hold E elements; thread t holds elements k = t + j*TPT,
// j = 0..E-1.  Both the input and the output of `Tile::fft` use this layout,
// so that pointwise work between two transforms (phase diagonals, epilogues)
// happens in registers, and global loads/stores along a contiguous axis are
// coalesced.
//
// Each radix-R Stockham stage (span p = product of the previous radices)
// takes inputs at i + r*N/R, i = t + q*TPT, multiplies by the twiddles
// w^(r*k) with k = i mod p and w = exp(-+2 pi i/(p R)), applies the R-point
// DFT and writes output r to (i div p)*p*R + k + r*p.  Intermediate stages
// exchange through LDS (ping-pong buffers, one barrier per stage); the last
// stage's outputs land back in canonical order.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace sr {

// ----------------------------------------------------------- complex helpers
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (forward quarter turn) or +i (inverse quarter turn)
template <bool INV>
__device__ __forceinline__ float2 quarter(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// e^{i theta} scaled by s, with an optional conjugate
template <bool CONJ>
__device__ __forceinline__ float2 phase(float theta, float s) {
  float sn, cs;
  sincosf(theta, &sn, &cs);
  return make_float2(cs * s, CONJ ? -sn * s : sn * s);
}

// e^{i theta} from the hardware sine and cosine, which take their argument in
// turns: theta / (2 pi) reduced to [0, 1) first.  Absolute error about 5e-7
// (against 7e-8 for sincosf) for a few instructions instead of a full range
// reduction; used where the pass kernels evaluate the phase diagonals on the
// fly (the exp(i theta) tables are filled with sincosf).
__device__ __forceinline__ float2 phase_turns(float theta) {
  const float r = __builtin_amdgcn_fractf(theta * 0.159154943091895335768883763372514362f);
  return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
}

// Deterministic workgroup sum: a fixed shuffle tree inside each wave, lane
// 0's total broadcast to the wave, then the wave totals added in wave order.
// Every thread gets the same value.  NTHREADS must be a power of two and
// equal blockDim.x; `red` holds at least NTHREADS / 64 values.
template <int NTHREADS, class V>
__device__ __forceinline__ V block_sum_t(V v, V* red) {
  constexpr int W = NTHREADS < 64 ? NTHREADS : 64;
  constexpr int NW = NTHREADS / W;
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_down(v, o, W);
  v = __shfl(v, 0, W);
  if constexpr (NW == 1) {
    return v;
  } else {
    __syncthreads();  // `red` may still be read by an earlier call
    if ((threadIdx.x & (W - 1)) == 0) red[threadIdx.x / W] = v;
    __syncthreads();
    V s = red[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) s += red[i];
    return s;
  }
}

template <int NTHREADS>
__device__ __forceinline__ float block_sum(float v, float* red) {
  return block_sum_t<NTHREADS, float>(v, red);
}

// Workgroup index -> tile index such that consecutive tiles run on the same
// XCD.  Workgroups are dispatched to the 8 XCDs round-robin (bid mod 8), each
// with its own L2; tiles that share cache lines (adjacent column tiles) then
// hit the same L2 instead of each XCD fetching the full line.  Bijective on
// [0, G) for any G.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_tile(int bid, int G) {
  const int q = G / kNumXcd, r = G % kNumXcd, x = bid % kNumXcd, l = bid / kNumXcd;
  return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// ------------------------------------------------------- buffer memory ops
// Global loads and stores through buffer resources.  A lane whose element
// lies outside its window passes an offset past the resource's range, so the
// hardware returns zero (loads) or drops the write (stores) without a branch;
// offsets are 32-bit byte offsets from a wave-uniform base (every buffer a
// pass touches spans well under 2 GiB).
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr unsigned kOob = 0x80000000u;  // byte offset past every resource
__device__ __forceinline__ Rsrc rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ unsigned off8(bool ok, int e) { return ok ? (unsigned)e * 8u : kOob; }
__device__ __forceinline__ unsigned off4(bool ok, int e) { return ok ? (unsigned)e * 4u : kOob; }
__device__ __forceinline__ float2 ld2(Rsrc r, unsigned off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return make_float2(__builtin_bit_cast(float, (unsigned)v[0]), __builtin_bit_cast(float, (unsigned)v[1]));
}
__device__ __forceinline__ float ld1(Rsrc r, unsigned off) {
  return __builtin_bit_cast(float, (unsigned)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ void st2(Rsrc r, unsigned off, float2 x) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  u32x2 v;
  v[0] = __builtin_bit_cast(unsigned, x.x);
  v[1] = __builtin_bit_cast(unsigned, x.y);
  __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
}
__device__ __forceinline__ void st1(Rsrc r, unsigned off, float x) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, off, 0, 0);
}

// ------------------------------------------------------- non-finite values
// True unless v is NaN or +-Inf (the comparison fails for NaN).
__device__ __forceinline__ bool finite2(float2 v) {
  return fabsf(v.x) <= 3.402823466e38f && fabsf(v.y) <= 3.402823466e38f;
}

// Raise the non-finite flag from the lanes that met one: a vector store of
// the same value from every such lane (no read-modify-write needed).
__device__ __forceinline__ void flag_nonfinite(unsigned* nf, bool bad) {
  if (nf != nullptr && bad)
    __builtin_amdgcn_raw_buffer_store_b32(1u, __builtin_amdgcn_make_buffer_rsrc(nf, (short)0, 4, 0x00020000), 0u, 0, 0);
}

// --------------------------------------------------------------- butterflies
// In-place R-point DFT, y_k = sum_j u_j w^(jk), w = exp(-2 pi i/R) (forward)
// or exp(+2 pi i/R) (INV).  No scaling.
template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* u) {
    float2 a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __device__ __forceinline__ static void run(float2* u) {
    const float h = 0.866025403784438646763723170752936183f;  // sqrt(3)/2
    float2 s = cadd(u[1], u[2]);
    float2 d = csub(u[1], u[2]);
    float2 m = make_float2(u[0].x - 0.5f * s.x, u[0].y - 0.5f * s.y);
    float2 q = cscale(quarter<INV>(d), h);  // -+ i sqrt(3)/2 (u1 - u2)
    u[0] = cadd(u[0], s);
    u[1] = cadd(m, q);
    u[2] = csub(m, q);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* u) {
    float2 t0 = cadd(u[0], u[2]);
    float2 t1 = csub(u[0], u[2]);
    float2 t2 = cadd(u[1], u[3]);
    float2 t3 = quarter<INV>(csub(u[1], u[3]));
    u[0] = cadd(t0, t2);
    u[2] = csub(t0, t2);
    u[1] = cadd(t1, t3);
    u[3] = csub(t1, t3);
  }
};

template <bool INV>
struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* u) {
    const float c = 0.707106781186547524400844362104849039f;  // sqrt(2)/2
    float2 e[4] = {u[0], u[2], u[4], u[6]};
    float2 o[4] = {u[1], u[3], u[5], u[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    // w8^1 = (c, -+c), w8^2 = -+i, w8^3 = (-c, -+c)
    float2 o1 = INV ? make_float2(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y))
                    : make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
    float2 o2 = quarter<INV>(o[2]);
    float2 o3 = INV ? make_float2(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y))
                    : make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
    u[0] = cadd(e[0], o[0]);
    u[4] = csub(e[0], o[0]);
    u[1] = cadd(e[1], o1);
    u[5] = csub(e[1], o1);
    u[2] = cadd(e[2], o2);
    u[6] = csub(e[2], o2);
    u[3] = cadd(e[3], o3);
    u[7] = csub(e[3], o3);
  }
};

// 16 = 4 x 4: index n = 4 n1 + n2 in, k = k1 + 4 k2 out; four 4-point DFTs
// over n1, the twiddles w16^(n2 k1), four 4-point DFTs over n2.
template <bool INV>
struct Dft<16, INV> {
  __device__ __forceinline__ static void run(float2* u) {
    const float c1 = 0.923879532511286756128183189396788933f;  // cos(pi/8)
    const float s1 = 0.382683432365089771728459984030398866f;  // sin(pi/8)
    const float h = 0.707106781186547524400844362104849039f;   // cos(pi/4)
    float2 a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      float2 t[4] = {u[n2], u[4 + n2], u[8 + n2], u[12 + n2]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = t[k1];
    }
    // forward w16^j = (cos(2 pi j/16), -sin(2 pi j/16)); the inverse conjugates
    auto tw = [](float2 v, float re, float im) { return INV ? cmulc(v, make_float2(re, im)) : cmul(v, make_float2(re, im)); };
    a[1][1] = tw(a[1][1], c1, -s1);  // j = 1
    a[1][2] = tw(a[1][2], h, -h);    // j = 2
    a[1][3] = tw(a[1][3], s1, -c1);  // j = 3
    a[2][1] = tw(a[2][1], h, -h);    // j = 2
    a[2][2] = quarter<INV>(a[2][2]); // j = 4
    a[2][3] = tw(a[2][3], -h, -h);   // j = 6
    a[3][1] = tw(a[3][1], s1, -c1);  // j = 3
    a[3][2] = tw(a[3][2], -h, -h);   // j = 6
    a[3][3] = tw(a[3][3], -c1, s1);  // j = 9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) u[k1 + 4 * k2] = t[k2];
    }
  }
};

// ------------------------------------------------------------- radix lists
template <int... Rs>
struct RadixList {
  static constexpr int count = sizeof...(Rs);
  static constexpr int values[count] = {Rs...};
  static constexpr int product() {
    int p = 1;
    for (int i = 0; i < count; ++i) p *= values[i];
    return p;
  }
  static constexpr int span(int s) {  // product of the first s radices
    int p = 1;
    for (int i = 0; i < s; ++i) p *= values[i];
    return p;
  }
};

// Factorisation and elements-per-thread for each supported length.
template <int N>
struct FftShape;
template <> struct FftShape<16>   { static constexpr int E = 4;  using R = RadixList<4, 4>; };
template <> struct FftShape<32>   { static constexpr int E = 8;  using R = RadixList<8, 4>; };
template <> struct FftShape<64>   { static constexpr int E = 8;  using R = RadixList<8, 8>; };
template <> struct FftShape<128>  { static constexpr int E = 8;  using R = RadixList<8, 4, 4>; };
template <> struct FftShape<256>  { static constexpr int E = 8;  using R = RadixList<8, 8, 4>; };
template <> struct FftShape<512>  { static constexpr int E = 8;  using R = RadixList<8, 8, 8>; };
template <> struct FftShape<1024> { static constexpr int E = 8;  using R = RadixList<8, 8, 4, 4>; };
template <> struct FftShape<2048> { static constexpr int E = 8;  using R = RadixList<8, 8, 8, 4>; };
template <> struct FftShape<4096> { static constexpr int E = 8;  using R = RadixList<8, 8, 8, 8>; };
template <> struct FftShape<24>   { static constexpr int E = 12; using R = RadixList<3, 4, 2>; };
template <> struct FftShape<48>   { static constexpr int E = 12; using R = RadixList<3, 4, 4>; };
template <> struct FftShape<96>   { static constexpr int E = 12; using R = RadixList<3, 4, 4, 2>; };
template <> struct FftShape<192>  { static constexpr int E = 12; using R = RadixList<3, 4, 4, 4>; };
template <> struct FftShape<384>  { static constexpr int E = 12; using R = RadixList<3, 4, 4, 4, 2>; };
template <> struct FftShape<768>  { static constexpr int E = 12; using R = RadixList<3, 4, 4, 4, 4>; };

// Narrow variant of the power-of-two lengths: four elements per thread
// (radix-4 stages, one radix-2 stage for odd powers), i.e. twice the threads
// per transform.  It costs more LDS exchanges but halves each wave's serial
// arithmetic, which pays when a pass has too few transforms to give every
// SIMD of the chip a wave of the default shape.
template <int N>
struct FftNarrow;
template <> struct FftNarrow<64>   { using R = RadixList<4, 4, 4>; };
template <> struct FftNarrow<128>  { using R = RadixList<4, 4, 4, 2>; };
template <> struct FftNarrow<256>  { using R = RadixList<4, 4, 4, 4>; };
template <> struct FftNarrow<512>  { using R = RadixList<4, 4, 4, 4, 2>; };
template <> struct FftNarrow<1024> { using R = RadixList<4, 4, 4, 4, 4>; };
// Wide thread shape: sixteen elements per thread with radix-16 stages, for
// column tiles of eight 2048-point transforms in 1024 threads.
template <int N> struct FftWide;
template <> struct FftWide<2048> { using R = RadixList<16, 16, 8>; };
template <int N> struct HasWide { static constexpr bool value = false; };
template <> struct HasWide<2048> { static constexpr bool value = true; };
template <int N> struct HasNarrow { static constexpr bool value = false; };
template <> struct HasNarrow<64> { static constexpr bool value = true; };
template <> struct HasNarrow<128> { static constexpr bool value = true; };
template <> struct HasNarrow<256> { static constexpr bool value = true; };
template <> struct HasNarrow<512> { static constexpr bool value = true; };
template <> struct HasNarrow<1024> { static constexpr bool value = true; };

// ------------------------------------------------------------------- tile
// A tile of B transforms of length N.  COL selects the thread mapping used for
// column-mode tiles: lane = t*B + b (consecutive lanes walk the batch, which is
// the contiguous direction in memory) with LDS layout [k][b]; otherwise
// lane = b*TPT + t with LDS layout [b][k + pad].  DB: ping-pong LDS buffers
// (one barrier per stage) or a single buffer (half the LDS, two barriers per
// stage) -- the single buffer lets two large column tiles share a CU.
template <int N, int B, bool COL, bool DB = true, int E_ = FftShape<N>::E, class RL = typename FftShape<N>::R>
struct Tile {
  static constexpr int E = E_;
  static constexpr int TPT = N / E;
  static constexpr int THREADS = TPT * B;
  // One pad slot every R0 elements for radix-8- or radix-4-first lengths:
  // the stage-0 scatter (stride R0) would otherwise put lanes on one LDS
  // bank pair.
  static constexpr int PADSHIFT =
      RL::values[0] == 16 ? 4 : RL::values[0] == 8 ? 3 : (RL::values[0] == 4 && E_ == 4) ? 2 : 0;
  static constexpr int NP = PADSHIFT ? N + (N >> PADSHIFT) : N;  // padded transform length
  static constexpr int LD = NP;               // row-mode LDS stride
  static constexpr int BUF = B * NP;          // complex elements per LDS buffer
  static constexpr int NBUF = DB ? 2 : 1;     // LDS buffers (elements: NBUF * BUF)
  static_assert(N % E == 0, "E must divide N");
  static_assert(RL::product() == N, "radix list must multiply to N");

  __device__ __forceinline__ static int padk(int k) { return PADSHIFT ? k + (k >> PADSHIFT) : k; }
  __device__ __forceinline__ static int lidx(int b, int k) { return COL ? (padk(k) * B + b) : (b * LD + padk(k)); }
  __device__ __forceinline__ static int thread_t() { return COL ? (int)(threadIdx.x / B) : (int)(threadIdx.x % TPT); }
  __device__ __forceinline__ static int thread_b() { return COL ? (int)(threadIdx.x % B) : (int)(threadIdx.x / TPT); }
  __device__ __forceinline__ static int elem(int t, int j) { return t + j * TPT; }

  // Twiddle factors this thread needs, preloaded into registers once
  // (stages >= 1; stage 0 has span 1 and no twiddles).  Forward and inverse
  // transforms of the same length share them (the inverse conjugates).
  static constexpr int tw_offset(int S) {
    int c = 0;
    for (int s = 1; s < S && s < RL::count; ++s) c += (E / RL::values[s]) * (RL::values[s] - 1);
    return c;
  }
  static constexpr int NTW = tw_offset(RL::count) > 0 ? tw_offset(RL::count) : 1;
  // The sixteen-element shape reads each stage's twiddles from the table at
  // that stage instead (its 29 would not fit in registers beside the data).
  static constexpr bool LAZY_TW = E_ >= 16;
  struct TableTw {
    const float2* p;  // the table, offset to this thread
  };
  using Twiddles = typename std::conditional<LAZY_TW, TableTw, float2[NTW]>::type;

  // tw: this shape's thread-order twiddle table, entry i * TPT + t = twiddle
  // slot i of thread t (so each load instruction reads consecutive entries),
  // values exp(-2 pi i e/N) rounded from float64 (see for_each_twiddle).
  __device__ __forceinline__ static void load_twiddles(Twiddles& w, const float2* __restrict__ tw, int t) {
    if constexpr (LAZY_TW) {
      w.p = tw + t;
    } else {
#pragma unroll
      for (int i = 0; i < NTW; ++i) w[i] = tw[i * TPT + t];
    }
  }

  // Host: calls f(slot, t, e) for every twiddle slot of every thread, where
  // slot i of thread t holds exp(-2 pi i e/N).  Stage S >= 1 (span P, radix R)
  // multiplies input r of butterfly q by w^(r k), k = (t + q TPT) mod P,
  // w = exp(-2 pi i/(P R)), i.e. e = r k N/(P R).
  template <class F>
  static void for_each_twiddle(F&& f) {
    twiddle_stage<1>(f);
  }

  // Forward (INV=false) or inverse (INV=true) unscaled DFT of the B transforms.
  // v: canonical registers in, canonical registers out.  lds: two buffers of
  // BUF elements; `phase` selects which buffer the first exchange writes and
  // is advanced so that consecutive transforms keep alternating buffers.
  template <bool INV>
  __device__ __forceinline__ static void fft(float2 (&v)[E], float2* lds, int& phase, const Twiddles& w, int t,
                                             int b) {
    stage<INV, 0>(v, lds, phase, w, t, b);
  }

 private:
  template <int S, class F>
  static void twiddle_stage(F& f) {
    if constexpr (S < RL::count) {
      constexpr int R = RL::values[S];
      constexpr int P = RL::span(S);
      constexpr int Q = E / R;
      constexpr int STRIDE = N / (P * R);
      for (int t = 0; t < TPT; ++t)
        for (int q = 0; q < Q; ++q) {
          const int k = (t + q * TPT) % P;
          for (int r = 1; r < R; ++r) f(tw_offset(S) + q * (R - 1) + (r - 1), t, r * k * STRIDE);
        }
      twiddle_stage<S + 1>(f);
    }
  }

  // Fence between the LDS writes of one stage and the reads of the next: a
  // workgroup barrier, or, when the whole tile is one wavefront, only a
  // wavefront-scope fence (the LDS operations of one wavefront complete in
  // issue order, so nothing waits on other waves).
  __device__ __forceinline__ static void xsync() {
    if constexpr (THREADS <= 64) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
      __syncthreads();
    }
  }

  template <bool INV, int S>
  __device__ __forceinline__ static void stage(float2 (&v)[E], float2* lds, int& phase, const Twiddles& w, int t,
                                               int b) {
    if constexpr (S < RL::count) {
      constexpr int R = RL::values[S];
      constexpr int P = RL::span(S);
      constexpr int Q = E / R;  // butterflies per thread in this stage
      static_assert(E % R == 0, "radix must divide elements per thread");
      // this stage's twiddles (from registers, or loaded from the table now,
      // in flight across the exchange below)
      constexpr int NS = S > 0 ? Q * (R - 1) : 1;
      float2 ws[NS];
      if constexpr (S > 0) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          if constexpr (LAZY_TW) ws[i] = w.p[(tw_offset(S) + i) * TPT];
          else ws[i] = w[tw_offset(S) + i];
        }
      }
      if constexpr (S > 0) {
        // inputs of this stage: canonical positions in the buffer written last
        xsync();
        float2* src = DB ? lds + (phase ^ 1) * BUF : lds;
#pragma unroll
        for (int j = 0; j < E; ++j) v[j] = src[lidx(b, elem(t, j))];
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        float2 u[R];
#pragma unroll
        for (int r = 0; r < R; ++r) u[r] = v[q + r * Q];
        const int i = t + q * TPT;
        const int k = i % P;
        if constexpr (S > 0) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const float2 tf = ws[q * (R - 1) + (r - 1)];
            u[r] = INV ? cmulc(u[r], tf) : cmul(u[r], tf);
          }
        }
        Dft<R, INV>::run(u);
        if constexpr (S + 1 < RL::count) {
          if constexpr (!DB) {
            // single buffer: every thread must be done reading it (this stage's
            // loads, or an earlier transform's) before anyone overwrites it
            if (q == 0) xsync();
          }
          float2* dst = DB ? lds + phase * BUF : lds;
          const int base = (i / P) * P * R + k;
#pragma unroll
          for (int r = 0; r < R; ++r) dst[lidx(b, base + r * P)] = u[r];
        } else {
#pragma unroll
          for (int r = 0; r < R; ++r) v[q + r * Q] = u[r];
        }
      }
      if constexpr (S + 1 < RL::count) phase ^= 1;
      stage<INV, S + 1>(v, lds, phase, w, t, b);
    }
  }
};

// Tile of shape variant EV: 0 = the length's default shape, 1 = narrow,
// 2 = wide.
template <int N, int B, bool COL, bool DB, int EV>
struct TileSel {
  using type = Tile<N, B, COL, DB>;
};
template <int N, int B, bool COL, bool DB>
struct TileSel<N, B, COL, DB, 1> {
  using type = Tile<N, B, COL, DB, 4, typename FftNarrow<N>::R>;
};
template <int N, int B, bool COL, bool DB>
struct TileSel<N, B, COL, DB, 2> {
  using type = Tile<N, B, COL, DB, 16, typename FftWide<N>::R>;
};
template <int N, int B, bool COL, bool DB = true, int EV = 0>
using TileV = typename TileSel<N, B, COL, DB, EV>::type;

}  // namespace sr
