// Host stand-in for <hip/hip_runtime.h>, used only to run the library's
// vector-ALU kernels on the CPU for checking (every work item an OS thread,
// workgroup barriers real barriers, __shared__ arrays one static copy used by
// one workgroup at a time).  Test infrastructure: never part of the library.
#pragma once

#include <barrier>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static

struct dim3 {
  unsigned x, y, z;
  constexpr dim3(unsigned x_ = 1, unsigned y_ = 1, unsigned z_ = 1) : x(x_), y(y_), z(z_) {}
};
struct emu_idx {
  unsigned x = 0, y = 0, z = 0;
};

namespace emu {
inline thread_local emu_idx t_thread, t_block;
inline dim3 g_block, g_grid;
inline std::barrier<>* g_bar = nullptr;
inline int g_checked = 0;
}  // namespace emu

#define threadIdx (emu::t_thread)
#define blockIdx (emu::t_block)
#define blockDim (emu::g_block)
#define gridDim (emu::g_grid)

inline void __syncthreads() { emu::g_bar->arrive_and_wait(); }
// scheduling hints of the device compiler: nothing to do on the host
#define __builtin_amdgcn_sched_barrier(mask) ((void)(mask))

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorInvalidConfiguration = 9 };
typedef void* hipStream_t;
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "emulated"; }
struct hipFuncAttributes {
  size_t sharedSizeBytes = 0, localSizeBytes = 0, constSizeBytes = 0;
  int maxThreadsPerBlock = 1024, numRegs = 0;
};
struct hipDeviceProp_t {
  size_t sharedMemPerBlock = 160 * 1024;
};
inline hipError_t hipFuncGetAttributes(hipFuncAttributes* a, const void*) {
  *a = hipFuncAttributes{};
  return hipSuccess;
}
inline hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  *p = hipDeviceProp_t{};
  return hipSuccess;
}

namespace emu {
// Runs fn once per work item of the grid: blockDim.x threads, each walking
// the blocks in order with a barrier after every block (so the static
// __shared__ arrays serve one block at a time).  With EMU_EDGE_BLOCKS=n in
// the environment only the first and last n blocks of each grid run (an
// index check of huge grids in reasonable time; the other blocks' outputs
// are left as they were).
inline void launch(dim3 grid, dim3 block, const std::function<void()>& fn) {
  unsigned edge = 0;
  if (const char* v = std::getenv("EMU_EDGE_BLOCKS")) edge = (unsigned)std::strtoul(v, nullptr, 10);
  if (block.y != 1 || block.z != 1 || grid.y != 1 || grid.z != 1) {
    std::fprintf(stderr, "emulated launch: 1-D grids only\n");
    std::abort();
  }
  g_grid = grid;
  g_block = block;
  std::barrier<> bar((std::ptrdiff_t)block.x);
  g_bar = &bar;
  std::vector<std::thread> th;
  th.reserve(block.x);
  for (unsigned t = 0; t < block.x; ++t)
    th.emplace_back([&, t]() {
      t_thread.x = t;
      for (unsigned b = 0; b < grid.x; ++b) {
        if (edge && b >= edge && b + edge < grid.x) b = grid.x - edge;
        t_block.x = b;
        fn();
        bar.arrive_and_wait();
      }
    });
  for (auto& x : th) x.join();
  g_bar = nullptr;
}
}  // namespace emu

#define hipLaunchKernelGGL(kernel, grid, block, shm, stream, ...) \
  emu::launch((grid), (block), [&]() { kernel(__VA_ARGS__); })
