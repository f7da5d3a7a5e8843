// Timing of selected kernel launches (diagnostics).  When a timer is
// installed for the calling thread, every stride-th launch of each timed
// kernel class goes through hipExtLaunchKernelGGL with a start and a stop
// event, which the runtime records at the start and the end of that kernel's
// execution on its stream; the other launches go out plain (events on every
// launch would add their own host cost to the run being measured).
// collect() (after the stream has been synchronised) adds up the sampled
// times; the per-class time is the sampled mean times the number of
// launches, and the algorithmic work covers every launch.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace sctm {

enum KernelClass : int {
  KC_GEMM_F64 = 0,
  KC_GEMM_F32 = 1,
  KC_GEMM_BF16X3 = 2,
  KC_JACOBI_GRAM = 3,    // pair kernel: Gram matrix + 32 x 32 eigensolve
  KC_JACOBI_SOLVE = 4,   // unused (the eigensolve runs in the pair kernel)
  KC_JACOBI_ROTATE = 5,
  KC_GEMM_BF16X6 = 6,
  KC_COUNT = 7
};

struct KernelTimer {
  struct Rec {
    int kind;
    hipEvent_t a, b;
  };
  int stride = 1;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> pending;
  double sampled_ms[KC_COUNT] = {};
  double sampled[KC_COUNT] = {};
  double flops[KC_COUNT] = {};
  double bytes[KC_COUNT] = {};
  double launches[KC_COUNT] = {};

  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  // counts the launch and its work; true (with the two events) when it is sampled
  bool events(int kind, double f, double by, hipEvent_t& a, hipEvent_t& b) {
    flops[kind] += f;
    bytes[kind] += by;
    const long k = (long)launches[kind];
    launches[kind] += 1;
    if (k % stride != 0) return false;
    a = next();
    b = next();
    if (!a || !b) return false;
    pending.push_back({kind, a, b});
    return true;
  }
  void add(int kind, double f, double by) {
    flops[kind] += f;
    bytes[kind] += by;
  }
  void collect() {
    for (const Rec& r : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        sampled_ms[r.kind] += t;
        sampled[r.kind] += 1;
      }
    }
    pending.clear();
    used = 0;
  }
  // estimated total kernel time of a class: sampled mean x launches
  double ms(int kind) const { return sampled[kind] > 0 ? sampled_ms[kind] / sampled[kind] * launches[kind] : 0.0; }
  void reset() {
    pending.clear();
    used = 0;
    for (int k = 0; k < KC_COUNT; ++k) sampled_ms[k] = sampled[k] = flops[k] = bytes[k] = launches[k] = 0;
  }
  ~KernelTimer() {
    for (hipEvent_t e : pool) hipEventDestroy(e);
  }
};

// timer of the calling thread (nullptr: no timing)
KernelTimer*& kernel_timer();

// Launch `kernel`; when a timer is installed, with start / stop events of
// class `kind` carrying the given algorithmic flops and bytes.
template <typename F, typename... Args>
inline void launch_timed(int kind, double flops, double bytes, F kernel, dim3 grid, dim3 block, uint32_t shmem,
                         hipStream_t s, Args... args) {
  KernelTimer* tm = kernel_timer();
  hipEvent_t a, b;
  if (tm && tm->events(kind, flops, bytes, a, b))
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, a, b, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
}

}  // namespace sctm
