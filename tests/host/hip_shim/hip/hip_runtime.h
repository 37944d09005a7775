// Host stand-in for the part of the HIP runtime that the XCTS solver
// (csrc/xcts.hip) uses, so that a g++ build of the same source can run on the
// CPU (tests/host/xcts_harness.cpp).  A kernel launch runs its blocks one after
// another; the threads of a block run on a pool of host threads, one per GPU
// thread, which meet at __syncthreads.  Device memory is host memory, copies
// are memmove, streams do nothing.
#pragma once
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <functional>

typedef unsigned short __bf16;
#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(x)
// one block runs at a time, so a block's shared arrays are plain statics
#define __shared__ static

typedef int hipError_t;
typedef void* hipStream_t;
typedef void* hipEvent_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorNotReady = 600 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyHostToHost };

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
extern dim3 blockIdx, blockDim, gridDim;  // the block being run
extern thread_local dim3 threadIdx;       // each pool thread's own index

namespace hipshim {
// Runs body once on each of blockDim.x pool threads (threadIdx.x = 0 ..);
// returns when all have finished.
void run_block(const std::function<void()>& body);
// __syncthreads: every thread of the running block waits for the others.
void syncthreads();
}  // namespace hipshim
#define __syncthreads() hipshim::syncthreads()

inline hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  if (n) memmove(d, s, n);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "host stand-in"; }

#define hipLaunchKernelGGL(K, G, B, SH, S, ...)                                    \
  do {                                                                             \
    const dim3 g_ = (G), b_ = (B);                                                 \
    gridDim = g_;                                                                  \
    blockDim = b_;                                                                 \
    for (unsigned bz = 0; bz < g_.z; ++bz)                                         \
      for (unsigned by = 0; by < g_.y; ++by)                                       \
        for (unsigned bx = 0; bx < g_.x; ++bx) {                                   \
          blockIdx = dim3(bx, by, bz);                                             \
          hipshim::run_block([&] { K(__VA_ARGS__); });                             \
        }                                                                          \
  } while (0)
