// HIP-event timing of selected kernel launches (diagnostics).  When a timer is
// installed for the calling thread, every launch of a timed kernel class is
// bracketed by two events on its stream; collect() (after the stream has been
// synchronised) adds the elapsed times and the algorithmic work of the
// launches to per-class totals.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace sctm {

enum KernelClass : int { KC_GEMM_F64 = 0, KC_GEMM_F32 = 1, KC_GEMM_BF16X3 = 2, KC_JACOBI = 3, KC_COUNT = 4 };

struct KernelTimer {
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double work;
  };
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> pending;
  double ms[KC_COUNT] = {0, 0, 0, 0};
  double work[KC_COUNT] = {0, 0, 0, 0};
  double launches[KC_COUNT] = {0, 0, 0, 0};

  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(hipStream_t s, int kind, double w) {
    hipEvent_t a = next(), b = next();
    if (!a || !b) return;
    hipEventRecord(a, s);
    pending.push_back({kind, a, b, w});
  }
  void end(hipStream_t s) {
    if (!pending.empty()) hipEventRecord(pending.back().b, s);
  }
  void collect() {
    for (const Rec& r : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.kind] += t;
        work[r.kind] += r.work;
        launches[r.kind] += 1;
      }
    }
    pending.clear();
    used = 0;
  }
  void reset() {
    pending.clear();
    used = 0;
    for (int k = 0; k < KC_COUNT; ++k) ms[k] = work[k] = launches[k] = 0;
  }
  ~KernelTimer() {
    for (hipEvent_t e : pool) hipEventDestroy(e);
  }
};

// timer of the calling thread (nullptr: no timing)
KernelTimer*& kernel_timer();

}  // namespace sctm
