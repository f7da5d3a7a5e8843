// Tensor engine of the split-CTMRG library: device tensors carved from a
// caller-owned workspace, einsum-style contractions lowered to permutes and
// MFMA GEMMs, and a tape that records every op so that the hand-written
// adjoints can run the reverse pass (the gradient dE/dA of Sec. III is
// reverse mode through the whole environment update).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "kernels.hpp"

namespace sctm {

enum DType : int { F64 = 0, F32 = 1 };

struct Ten {
  void* p = nullptr;
  int dt = F64;
  int r = 0;
  long d[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  int id = -1;
  long n() const {
    long k = 1;
    for (int i = 0; i < r; ++i) k *= d[i];
    return k;
  }
  size_t esize() const { return dt == F64 ? 8 : 4; }
  size_t bytes() const { return n() * esize(); }
  double* f64() const { return (double*)p; }
  float* f32() const { return (float*)p; }
};

// Bump allocator over a caller-owned device buffer.  In dry mode nothing is
// touched: the allocator only records the peak, which sizes the workspace.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, top = 0, peak = 0;
  bool dry = false;
  bool overflow = false;
  void* alloc(size_t bytes) {
    size_t b = (bytes + 255) & ~size_t(255);
    size_t o = top;
    top += b;
    if (top > peak) peak = top;
    if (dry) return (void*)(uintptr_t)(0x1000 + o);   // never dereferenced
    if (top > cap) {
      overflow = true;
      return nullptr;
    }
    return base + o;
  }
  size_t mark() const { return top; }
  void release(size_t m) { top = m; }
};

enum OpKind : int { OP_CONTRACT, OP_PERMUTE, OP_COPY, OP_CAST, OP_NORMALIZE, OP_PROJ, OP_BOND };

struct ProjSaved {
  Ten rT, rB;          // FP64 copies of the half networks (na x nb)
  Ten U, S, V, X, Y;   // SVD of M (or of its core, rk > 0) and the scaled truncated factors (nb x chi)
  Ten QLt, QRt;        // rk > 0: M = Q_L (U S V^T) Q_R^T with Q_L^T, Q_R^T (rk x nb) orthonormal rows
  Ten sgn;             // sign of every projector column
  Ten kr;              // device ints: [k, r]
  int na = 0, nb = 0, chi = 0;
  int rk = 0;          // > 0: M has rank <= rk and U, S, V are those of the rk x rk core
  bool rows = true;    // truncated legs are the rows of rho (else the columns)
};

struct ProjReq {
  Ten rT, rB;
  int n_a;
  bool rows;
  int chi;
  std::vector<double>* spectrum_out;
  // optional factorisation rho_T = fX^T fZ through a bond of dimension r0
  // (fX: a-legs x r0, fZ: r0 x b-legs; rows layout only): M = (fX^T rho_B)^T fZ
  // then has rank <= r0 and is decomposed through that core.
  Ten fX, fZ;
};

struct PlanStep {
  int i, j;            // operands: inputs 0..n-1, then intermediates in step order
  std::string keep;    // labels of the result
};
struct ContractionPlan {
  std::vector<PlanStep> steps;
  double flops = 0;
};

struct TapeRec {
  OpKind kind;
  std::vector<Ten> in, out;
  std::string spec;
  ProjSaved proj;
  Ten aux;             // normalize: [nrm2] FP64 device scalar; bond: [e, den]; permute: not used
  Ten h;               // bond: Hamiltonian (FP64, p^2 x p^2)
  int p = 0;
};

struct Engine {
  hipStream_t s = nullptr;
  // second stream (default priority) for work off the critical path: the Q
  // factors of the QRs, formed while s goes on; every use joins back into s
  // before the call that issued it returns.  Null: everything runs on s.
  hipStream_t aux = nullptr;
  hipEvent_t aux_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  Arena ar;
  Prec prec = Prec::F64;
  int cdt = F64;                 // dtype of contraction tensors
  bool taping = false;
  bool dry = false;
  hipError_t err = hipSuccess;
  int status = 0;                // first library-level failure (ctm_status code)
  int next_id = 0;
  double svd_tol = 0.0;            // <= 0: sqrt(n) * 1.2e-16
  int svd_max_sweeps = 40;
  double cutoff = 1e-12;
  double adj_eps = 1e-12;
  double* partial = nullptr;     // reduction scratch (reduce_partials() doubles)
  int* host_flags = nullptr;     // host buffer for SVD convergence flags
  int host_flags_n = 0;
  std::vector<TapeRec> tape;
  std::unordered_set<int> needs_grad;
  std::unordered_map<int, Ten> grads;
  long flops_gemm = 0;           // algorithmic flops of the GEMMs issued (statistics)
  long svd_sweeps_total = 0;

  bool ok() const { return err == hipSuccess && status == 0 && !ar.overflow; }
  void check(hipError_t e) {
    if (e != hipSuccess && err == hipSuccess) err = e;
  }

  Ten alloc(int dt, const std::vector<long>& dims);
  Ten alloc_like(const Ten& t) {
    std::vector<long> d(t.d, t.d + t.r);
    return alloc(t.dt, d);
  }
  void zero(const Ten& t);
  void mark_input(const Ten& t) { needs_grad.insert(t.id); }
  bool ng(const Ten& t) const { return needs_grad.count(t.id) != 0; }

  // ---- forward ops (taped when `taping`) ----
  Ten contract(const std::string& spec, const Ten& A, const Ten& B);
  Ten ncon(const std::string& spec, const std::vector<Ten>& ops);
  Ten permute(const Ten& A, const std::string& spec);   // "abc->cab"
  Ten copy(const Ten& A);
  Ten cast(const Ten& A, int dt);
  Ten normalize(const Ten& A);                          // A / |A|_F
  // Projector pair from the half networks (Fig. proj_plots_green recipe).
  // rT, rB: same shape; the first n_a legs (rows=true) or the last n_a legs
  // (rows=false) are the legs to truncate.  Returns {P_T, P_B} with shape
  // a_shape + (chi), in the contraction dtype; columns >= k are zero.
  std::vector<Ten> projectors(const Ten& rT, const Ten& rB, int n_a, bool rows, int chi,
                              std::vector<double>* spectrum_out = nullptr);
  std::vector<std::vector<Ten>> projectors_batch(const std::vector<ProjReq>& reqs);
  long svd_calls = 0;
  bool lowrank_svd = true;           // decompose rank-limited M through its r0 x r0 core
  // Record / replay of projector SVDs per move of a checkpoint block: the
  // recomputation of a move rebuilds bit-identical matrices M, so the U, S, V
  // recorded when the move first ran are reused instead of recomputed.
  struct SvdCacheSlot {
    long cap = 0, used = 0;
    bool valid = false;
    std::vector<long> off, nb, g, rk;
  };
  Ten svdc_buf;                      // FP64, nslots * per_slot elements
  long svdc_per_slot = 0;
  std::vector<SvdCacheSlot> svdc_slots;
  int svdc_mode = 0;                 // 0 off, 1 record, 2 replay
  int svdc_slot = -1;
  size_t svdc_cursor = 0;
  void svdc_setup(const Ten& buf, int nslots, long per_slot_elems) {
    svdc_buf = buf;
    svdc_per_slot = per_slot_elems;
    svdc_slots.assign(nslots, SvdCacheSlot{});
    for (auto& sl : svdc_slots) sl.cap = per_slot_elems;
    svdc_mode = 0;
    svdc_slot = -1;
  }
  void svdc_select(int slot, int mode) {
    svdc_slot = (slot >= 0 && slot < (int)svdc_slots.size()) ? slot : -1;
    svdc_mode = svdc_slot >= 0 ? mode : 0;
    svdc_cursor = 0;
    if (svdc_mode == 1) {
      SvdCacheSlot& sl = svdc_slots[svdc_slot];
      sl.used = 0;
      sl.valid = true;
      sl.off.clear();
      sl.nb.clear();
      sl.g.clear();
      sl.rk.clear();
    }
  }
  void svdc_reset() {
    svdc_slots.clear();
    svdc_mode = 0;
    svdc_slot = -1;
  }
  Ten bond_energy(const Ten& rho, const Ten& h64, int p);   // -> FP64 [2] (e, den)

  // ---- low level ----
  void contract_into(const std::string& spec, const Ten& A, const Ten& B, const Ten& C, bool accumulate);
  void permute_into(const Ten& A, const std::string& spec, const Ten& out, bool accumulate);
  void gemm(bool tA, bool tB, int M, int N, int K, double alpha, const Ten& A, long offA, long lda,
            const Ten& B, long offB, long ldb, double beta, const Ten& C, long offC, long ldc);
  // the product on its route (pre-split BF16X3, split-K or plain); returns the route's name
  const char* gemm_route(bool tA, bool tB, int M, int N, int K, double alpha, const Ten& A, long offA, long lda,
                         const Ten& B, long offB, long ldb, double beta, const Ten& C, long offC, long ldc);
  void add_into(const Ten& src, const Ten& dst);         // dst += src (same dtype/size)

  // ---- reverse pass ----
  Ten grad(const Ten& t);                                // zero-initialised on first use
  bool has_grad(const Ten& t) const { return grads.count(t.id) != 0; }
  void backward();                                       // walk the tape in reverse
  void clear_tape() {
    tape.clear();
    grads.clear();
    needs_grad.clear();
  }
  void record(TapeRec&& r);

 private:
  void proj_backward(TapeRec& r);
};

}  // namespace sctm
