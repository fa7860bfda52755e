// Instantiations and launcher of the persistent cooperative solver kernels.
#include "launch.hpp"
#include "persist.hpp"

namespace sr {

namespace {

__global__ void zero_sync_kernel(unsigned* bar, int* err) {
  if (threadIdx.x == 0) {
    *bar = 0u;
    *err = 0;
  }
}

template <int N, int B, int OP>
hipError_t go(const PersistArgs& pa, int grid, hipStream_t s) {
  auto kern = persistent_kernel<N, B, OP>;
  constexpr int threads = Tile<N, B, true>::THREADS;
  const size_t lds = 2 * sizeof(float2) * (size_t)Tile<N, B, true>::BUF;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds);
  if (e != hipSuccess) return e;
  int dev = 0, cus = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  const int cap = per_cu * cus;
  if (cap <= 0) return hipErrorInvalidConfiguration;
  if (grid > cap) grid = cap;
  hipLaunchKernelGGL(zero_sync_kernel, dim3(1), dim3(64), 0, s, pa.bar, pa.err);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  void* args[] = {(void*)&pa};
  return hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(threads), args, (unsigned)lds, s);
}

template <int N, int OP>
hipError_t by_b(int B, const PersistArgs& pa, int grid, hipStream_t s) {
  switch (B) {
    case 2: return go<N, 2, OP>(pa, grid, s);
    case 4: return go<N, 4, OP>(pa, grid, s);
    case 8: return go<N, 8, OP>(pa, grid, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool persistent_supported(int N, int B) {
  return (N == 256 || N == 512) && (B == 2 || B == 4 || B == 8);
}

hipError_t launch_persistent(int N, int B, int op, const PersistArgs& pa, int grid, hipStream_t s) {
  if (N == 512) return op == PO_GD ? by_b<512, PO_GD>(B, pa, grid, s) : by_b<512, PO_SPEC>(B, pa, grid, s);
  if (N == 256) return op == PO_GD ? by_b<256, PO_GD>(B, pa, grid, s) : by_b<256, PO_SPEC>(B, pa, grid, s);
  return hipErrorInvalidValue;
}

}  // namespace sr
