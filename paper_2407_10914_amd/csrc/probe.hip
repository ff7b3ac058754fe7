// Streaming reference kernels for the HBM roofline: the best rate that plain
// read, write and copy streams reach on this device is the practical ceiling
// a bandwidth-bound kernel is compared with (beside the published peak).
//
// Each kernel walks a float4 array with a grid-stride loop, four elements in
// flight per thread and iteration (all loads of an iteration issued before any
// use).  The read kernel folds what it reads into one value that it stores
// only when it equals an impossible sentinel, so the loads stay live without
// adding write traffic.  Non-temporal variants mark every access as streaming.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/cg_lbm.h"

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ v4f ld(const v4f* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <bool NT>
__device__ __forceinline__ void st(v4f* p, v4f v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// kind 0: read, 1: write, 2: copy
template <int Kind, bool NT>
__global__ void __launch_bounds__(1024) k_stream(const v4f* __restrict__ a, v4f* __restrict__ b, size_t n4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  const v4f one = {1.f, 1.f, 1.f, 1.f};
  for (; i + 3 * stride < n4; i += 4 * stride) {
    if constexpr (Kind == 1) {
      st<NT>(b + i, one);
      st<NT>(b + i + stride, one);
      st<NT>(b + i + 2 * stride, one);
      st<NT>(b + i + 3 * stride, one);
    } else {
      const v4f x0 = ld<NT>(a + i), x1 = ld<NT>(a + i + stride), x2 = ld<NT>(a + i + 2 * stride),
                x3 = ld<NT>(a + i + 3 * stride);
      if constexpr (Kind == 0) {
        acc += (x0 + x1) + (x2 + x3);
      } else {
        st<NT>(b + i, x0);
        st<NT>(b + i + stride, x1);
        st<NT>(b + i + 2 * stride, x2);
        st<NT>(b + i + 3 * stride, x3);
      }
    }
  }
  for (; i < n4; i += stride) {
    if constexpr (Kind == 1) {
      st<NT>(b + i, one);
    } else {
      const v4f x = ld<NT>(a + i);
      if constexpr (Kind == 0)
        acc += x;
      else
        st<NT>(b + i, x);
    }
  }
  if constexpr (Kind == 0) {
    if (acc.x + acc.y + acc.z + acc.w == -1.25e30f) b[0] = acc;
  }
}

template <int Kind, bool NT>
void launch(const void* a, void* b, size_t n4, int grid, int block, hipStream_t s) {
  hipLaunchKernelGGL((k_stream<Kind, NT>), dim3(grid), dim3(block), 0, s, (const v4f*)a, (v4f*)b, n4);
}

}  // namespace

extern "C" cg_status cg_stream_probe(int kind, const void* src, void* dst, size_t bytes, int grid, int block,
                                     int nontemporal, void* stream, int reps, float* ms_per_launch) {
  if (kind < 0 || kind > 2 || grid < 1 || block < 64 || block > 1024 || (block & 63) || reps < 1 ||
      !ms_per_launch || bytes < 16 || (bytes & 15))
    return CG_EINVAL;
  if ((kind != 1 && !src) || (kind != 0 && !dst) || (kind == 0 && !dst)) return CG_EINVAL;
  if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return CG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const size_t n4 = bytes / 16;
  auto go = [&]() {
    switch (kind * 2 + (nontemporal ? 1 : 0)) {
      case 0: launch<0, false>(src, dst, n4, grid, block, s); break;
      case 1: launch<0, true>(src, dst, n4, grid, block, s); break;
      case 2: launch<1, false>(src, dst, n4, grid, block, s); break;
      case 3: launch<1, true>(src, dst, n4, grid, block, s); break;
      case 4: launch<2, false>(src, dst, n4, grid, block, s); break;
      default: launch<2, true>(src, dst, n4, grid, block, s); break;
    }
  };
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return CG_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return CG_EHIP;
  }
  go();  // warm-up
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) go();
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) e = hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return CG_EHIP;
  *ms_per_launch = ms / (float)reps;
  return CG_OK;
}
