// Engine implementation: contraction planning, ops, and their adjoints.
#include "engine.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "adj_kernels.hpp"

namespace sctm {

// ---------------------------------------------------------------------------
// allocation
// ---------------------------------------------------------------------------
Ten Engine::alloc(int dt, const std::vector<long>& dims) {
  Ten t;
  t.dt = dt;
  if (dims.size() > 12) {   // rank beyond what Ten and the permute kernel hold
    status = 1;
    t.r = 0;
    return t;
  }
  t.r = (int)dims.size();
  for (int i = 0; i < t.r; ++i) t.d[i] = dims[i];
  t.id = next_id++;
  t.p = ar.alloc(t.bytes() ? t.bytes() : 8);
  if (!t.p && !dry) status = 2;   // workspace exhausted
  return t;
}

void Engine::zero(const Ten& t) {
  if (dry || !ok()) return;
  if (t.dt == F64)
    check(fill_f64(s, t.f64(), 0.0, t.n()));
  else
    check(fill_f32(s, t.f32(), 0.f, t.n()));
}

void Engine::record(TapeRec&& r) { tape.push_back(std::move(r)); }

Ten Engine::grad(const Ten& t) {
  auto it = grads.find(t.id);
  if (it != grads.end()) return it->second;
  Ten g = alloc_like(t);
  zero(g);
  return grads[t.id] = g;
}

// ---------------------------------------------------------------------------
// permutations
// ---------------------------------------------------------------------------
static void parse_arrow(const std::string& spec, std::string& lhs, std::string& rhs) {
  size_t a = spec.find("->");
  lhs = spec.substr(0, a);
  rhs = spec.substr(a + 2);
}

void Engine::permute_into(const Ten& A, const std::string& spec, const Ten& out, bool accumulate) {
  std::string li, lo;
  parse_arrow(spec, li, lo);
  if ((int)li.size() != A.r || (int)lo.size() != A.r) {
    status = 1;
    return;
  }
  int perm[12];
  for (int i = 0; i < A.r; ++i) {
    size_t k = li.find(lo[i]);
    if (k == std::string::npos) {
      status = 1;
      return;
    }
    perm[i] = (int)k;
  }
  // input strides
  long st[12];
  st[A.r - 1] = 1;
  for (int i = A.r - 2; i >= 0; --i) st[i] = st[i + 1] * A.d[i + 1];
  // merge output axes that stay adjacent and in order in the input
  PermDesc d;
  d.rank = 0;
  for (int i = 0; i < A.r; ++i) {
    if (A.d[perm[i]] == 1) continue;
    d.out_dims[d.rank] = A.d[perm[i]];
    d.in_strides_perm[d.rank] = st[perm[i]];
    ++d.rank;
  }
  // merge pass: axis k and k+1 merge when stride[k] == stride[k+1] * dim[k+1]
  PermDesc m;
  m.rank = 0;
  for (int i = 0; i < d.rank; ++i) {
    if (m.rank > 0 && m.in_strides_perm[m.rank - 1] == d.in_strides_perm[i] * d.out_dims[i]) {
      m.out_dims[m.rank - 1] *= d.out_dims[i];
      m.in_strides_perm[m.rank - 1] = d.in_strides_perm[i];
    } else {
      m.out_dims[m.rank] = d.out_dims[i];
      m.in_strides_perm[m.rank] = d.in_strides_perm[i];
      ++m.rank;
    }
  }
  if (m.rank == 0) {
    m.rank = 1;
    m.out_dims[0] = 1;
    m.in_strides_perm[0] = 1;
  }
  if (dry || !ok()) return;
  if (m.rank == 1 && m.in_strides_perm[0] == 1) {   // identity
    if (accumulate)
      add_into(A, out);
    else
      check(hipMemcpyAsync(out.p, A.p, A.bytes(), hipMemcpyDeviceToDevice, s));
    return;
  }
  check(sctm::permute(s, (int)A.esize(), A.p, out.p, m, A.n(), accumulate));
}

Ten Engine::permute(const Ten& A, const std::string& spec) {
  std::string li, lo;
  parse_arrow(spec, li, lo);
  std::vector<long> dims;
  for (char c : lo) dims.push_back(A.d[li.find(c)]);
  Ten out = alloc(A.dt, dims);
  permute_into(A, spec, out, false);
  if (taping && ng(A)) {
    TapeRec r;
    r.kind = OP_PERMUTE;
    r.in = {A};
    r.out = {out};
    r.spec = spec;
    record(std::move(r));
    needs_grad.insert(out.id);
  }
  return out;
}

void Engine::add_into(const Ten& src, const Ten& dst) {
  if (dry || !ok()) return;
  if (src.dt == dst.dt) {
    if (src.dt == F64)
      check(axpy_f64(s, 1.0, src.f64(), dst.f64(), src.n()));
    else
      check(axpy_f32(s, 1.f, src.f32(), dst.f32(), src.n()));
    return;
  }
  check(add_cast(s, src.p, src.dt == F64, dst.p, dst.dt == F64, src.n()));
}

Ten Engine::copy(const Ten& A) {
  Ten out = alloc_like(A);
  if (!dry && ok()) check(hipMemcpyAsync(out.p, A.p, A.bytes(), hipMemcpyDeviceToDevice, s));
  if (taping && ng(A)) {
    TapeRec r;
    r.kind = OP_COPY;
    r.in = {A};
    r.out = {out};
    record(std::move(r));
    needs_grad.insert(out.id);
  }
  return out;
}

Ten Engine::cast(const Ten& A, int dt) {
  if (A.dt == dt) return A;
  std::vector<long> dims(A.d, A.d + A.r);
  Ten out = alloc(dt, dims);
  if (!dry && ok()) {
    if (dt == F64)
      check(cast_f32_to_f64(s, A.f32(), out.f64(), A.n()));
    else
      check(cast_f64_to_f32(s, A.f64(), out.f32(), A.n()));
  }
  if (taping && ng(A)) {
    TapeRec r;
    r.kind = OP_CAST;
    r.in = {A};
    r.out = {out};
    record(std::move(r));
    needs_grad.insert(out.id);
  }
  return out;
}

Ten Engine::normalize(const Ten& A) {
  Ten nrm2 = alloc(F64, {1});
  Ten out = alloc_like(A);
  if (!dry && ok()) {
    if (A.dt == F64) {
      check(sumsq_f64(s, A.f64(), A.n(), partial, nrm2.f64()));
      check(scale_by_rsqrt_f64(s, A.f64(), out.f64(), nrm2.f64(), A.n()));
    } else {
      check(sumsq_f32(s, A.f32(), A.n(), partial, nrm2.f64()));
      check(scale_by_rsqrt_f32(s, A.f32(), out.f32(), nrm2.f64(), A.n()));
    }
  }
  if (taping && ng(A)) {
    TapeRec r;
    r.kind = OP_NORMALIZE;
    r.in = {A};
    r.out = {out};
    r.aux = nrm2;
    record(std::move(r));
    needs_grad.insert(out.id);
  }
  return out;
}

// ---------------------------------------------------------------------------
// GEMM dispatch
// ---------------------------------------------------------------------------
void Engine::gemm(bool tA, bool tB, int M, int N, int K, double alpha, const Ten& A, long offA, long lda,
                  const Ten& B, long offB, long ldb, double beta, const Ten& C, long offC, long ldc) {
  flops_gemm += 2L * M * N * K;
  if (dry || !ok()) return;
  if (M <= 0 || N <= 0) return;
  if (K <= 0) {   // C = beta C
    if (beta == 0.0) {
      // zero the M x N block row by row (contiguous when ldc == N)
      if (ldc == N) {
        if (C.dt == F64)
          check(fill_f64(s, C.f64() + offC, 0.0, (long)M * N));
        else
          check(fill_f32(s, C.f32() + offC, 0.f, (long)M * N));
      }
    }
    return;
  }
  if (C.dt == F64)
    check(gemm_f64(s, tA, tB, M, N, K, alpha, A.f64() + offA, lda, 0, B.f64() + offB, ldb, 0, beta,
                   C.f64() + offC, ldc, 0, 1));
  else
    check(gemm_f32(s, prec == Prec::BF16X3 ? Prec::BF16X3 : Prec::F32, tA, tB, M, N, K, (float)alpha,
                   A.f32() + offA, lda, 0, B.f32() + offB, ldb, 0, (float)beta, C.f32() + offC, ldc, 0, 1));
}

// ---------------------------------------------------------------------------
// pairwise contraction: permute operands (only when needed) + one GEMM
// ---------------------------------------------------------------------------
static std::string filt(const std::string& src, const std::string& keep_in, bool in) {
  std::string o;
  for (char c : src)
    if ((keep_in.find(c) != std::string::npos) == in) o += c;
  return o;
}

void Engine::contract_into(const std::string& spec, const Ten& A, const Ten& B, const Ten& C, bool accumulate) {
  std::string lhs, lc;
  parse_arrow(spec, lhs, lc);
  size_t comma = lhs.find(',');
  std::string la = lhs.substr(0, comma), lb = lhs.substr(comma + 1);
  if ((int)la.size() != A.r || (int)lb.size() != B.r || (int)lc.size() != C.r || A.dt != B.dt || A.dt != C.dt) {
    status = 1;
    return;
  }
  auto dim = [&](char c) -> long {
    size_t i = la.find(c);
    if (i != std::string::npos) return A.d[i];
    return B.d[lb.find(c)];
  };
  std::string fa = filt(la, lc, true), fb = filt(lb, lc, true);
  std::string ka = filt(la, lc, false), kb = filt(lb, lc, false);
  // every label must be either contracted (in both) or free (in one + output)
  for (char c : ka)
    if (lb.find(c) == std::string::npos) status = 1;
  for (char c : fa)
    if (lb.find(c) != std::string::npos) status = 1;   // batch labels unsupported
  if (status) return;
  long M = 1, N = 1, K = 1;
  for (char c : fa) M *= dim(c);
  for (char c : fb) N *= dim(c);
  for (char c : ka) K *= dim(c);
  // choose the contracted order that needs the fewest operand permutes
  struct Plan {
    std::string ko;
    bool pa, pb, ta, tb;
    long cost;
  } best{};
  best.cost = -1;
  for (int opt = 0; opt < 2; ++opt) {
    std::string ko = opt == 0 ? ka : kb;
    Plan p{ko, false, false, false, false, 0};
    if (la == fa + ko)
      p.ta = false;
    else if (la == ko + fa)
      p.ta = true;
    else {
      p.pa = true;
      p.cost += A.n();
    }
    if (lb == ko + fb)
      p.tb = false;
    else if (lb == fb + ko)
      p.tb = true;
    else {
      p.pb = true;
      p.cost += B.n();
    }
    if (best.cost < 0 || p.cost < best.cost) best = p;
  }
  size_t mk = ar.mark();
  Ten Aop = A, Bop = B;
  if (best.pa) {
    std::string want = fa + best.ko;
    std::vector<long> d;
    for (char c : want) d.push_back(dim(c));
    Aop = alloc(A.dt, d);
    permute_into(A, la + "->" + want, Aop, false);
    best.ta = false;
  }
  if (best.pb) {
    std::string want = best.ko + fb;
    std::vector<long> d;
    for (char c : want) d.push_back(dim(c));
    Bop = alloc(B.dt, d);
    permute_into(B, lb + "->" + want, Bop, false);
    best.tb = false;
  }
  const long lda = best.ta ? M : K, ldb = best.tb ? K : N;
  if (lc == fa + fb) {
    gemm(best.ta, best.tb, (int)M, (int)N, (int)K, 1.0, Aop, 0, lda, Bop, 0, ldb, accumulate ? 1.0 : 0.0, C, 0, N);
  } else if (lc == fb + fa) {
    // C^T = op(B)^T op(A)^T
    gemm(!best.tb, !best.ta, (int)N, (int)M, (int)K, 1.0, Bop, 0, ldb, Aop, 0, lda, accumulate ? 1.0 : 0.0, C, 0, M);
  } else {
    std::string nat = fa + fb;
    std::vector<long> d;
    for (char c : nat) d.push_back(dim(c));
    Ten T = alloc(C.dt, d);
    gemm(best.ta, best.tb, (int)M, (int)N, (int)K, 1.0, Aop, 0, lda, Bop, 0, ldb, 0.0, T, 0, N);
    permute_into(T, nat + "->" + lc, C, accumulate);
  }
  // temporaries are dead once the kernels are enqueued in stream order, but
  // the stack allocator may only release what sits above C: C was allocated
  // before the temporaries, so releasing to the mark is safe.
  ar.release(mk);
}

Ten Engine::contract(const std::string& spec, const Ten& A, const Ten& B) {
  std::string lhs, lc;
  parse_arrow(spec, lhs, lc);
  size_t comma = lhs.find(',');
  std::string la = lhs.substr(0, comma), lb = lhs.substr(comma + 1);
  std::vector<long> dims;
  for (char c : lc) {
    size_t i = la.find(c);
    dims.push_back(i != std::string::npos ? A.d[i] : B.d[lb.find(c)]);
  }
  Ten C = alloc(A.dt, dims);
  contract_into(spec, A, B, C, false);
  if (taping && (ng(A) || ng(B))) {
    TapeRec r;
    r.kind = OP_CONTRACT;
    r.in = {A, B};
    r.out = {C};
    r.spec = spec;
    record(std::move(r));
    needs_grad.insert(C.id);
  }
  return C;
}

// Greedy pairwise contraction of a tensor network given as one einsum string.
// At every step the pair sharing an index with the fewest multiply-adds is
// contracted; its result keeps the free labels of the first operand followed
// by those of the second (the GEMM's natural output order, so no permute).
Ten Engine::ncon(const std::string& spec, const std::vector<Ten>& ops) {
  std::string lhs, out;
  parse_arrow(spec, lhs, out);
  std::vector<std::string> terms;
  size_t st = 0;
  while (true) {
    size_t c = lhs.find(',', st);
    terms.push_back(lhs.substr(st, c == std::string::npos ? std::string::npos : c - st));
    if (c == std::string::npos) break;
    st = c + 1;
  }
  if (terms.size() != ops.size()) {
    status = 1;
    return ops[0];
  }
  long dims[128];
  for (int i = 0; i < 128; ++i) dims[i] = 0;
  for (size_t i = 0; i < terms.size(); ++i) {
    if ((int)terms[i].size() != ops[i].r) {
      status = 1;
      return ops[0];
    }
    for (int k = 0; k < ops[i].r; ++k) {
      unsigned char c = terms[i][k];
      if (dims[c] && dims[c] != ops[i].d[k]) status = 1;
      dims[c] = ops[i].d[k];
    }
  }
  if (status) return ops[0];
  std::vector<std::pair<std::string, Ten>> items;
  for (size_t i = 0; i < terms.size(); ++i) items.push_back({terms[i], ops[i]});
  while (items.size() > 1) {
    int bi = -1, bj = -1;
    double bflops = 0, bsize = 0;
    bool bshared = false;
    std::string bkeep;
    for (size_t i = 0; i < items.size(); ++i)
      for (size_t j = i + 1; j < items.size(); ++j) {
        const std::string &ti = items[i].first, &tj = items[j].first;
        std::string rest = out;
        for (size_t k = 0; k < items.size(); ++k)
          if (k != i && k != j) rest += items[k].first;
        bool shared = false;
        double flops = 1.0, size = 1.0;
        std::string keep;
        for (char c : ti) {
          flops *= dims[(unsigned char)c];
          if (tj.find(c) != std::string::npos) shared = true;
          if (rest.find(c) != std::string::npos) {
            keep += c;
            size *= dims[(unsigned char)c];
          }
        }
        for (char c : tj) {
          if (ti.find(c) == std::string::npos) flops *= dims[(unsigned char)c];
          if (ti.find(c) == std::string::npos && rest.find(c) != std::string::npos) {
            keep += c;
            size *= dims[(unsigned char)c];
          }
        }
        bool better = bi < 0 || (shared && !bshared) ||
                      (shared == bshared && (flops < bflops || (flops == bflops && size < bsize)));
        if (better) {
          bi = (int)i;
          bj = (int)j;
          bflops = flops;
          bsize = size;
          bshared = shared;
          bkeep = keep;
        }
      }
    Ten r = contract(items[bi].first + "," + items[bj].first + "->" + bkeep, items[bi].second, items[bj].second);
    std::vector<std::pair<std::string, Ten>> nx;
    for (size_t k = 0; k < items.size(); ++k)
      if ((int)k != bi && (int)k != bj) nx.push_back(items[k]);
    nx.push_back({bkeep, r});
    items.swap(nx);
  }
  if (items[0].first == out) return items[0].second;
  return permute(items[0].second, items[0].first + "->" + out);
}

// ---------------------------------------------------------------------------
// projectors
// ---------------------------------------------------------------------------
std::vector<Ten> Engine::projectors(const Ten& rT, const Ten& rB, int n_a, bool rows, int chi,
                                    std::vector<double>* spectrum_out) {
  long na = 1, nb = 1;
  std::vector<long> a_shape;
  if (rows) {
    for (int i = 0; i < n_a; ++i) {
      na *= rT.d[i];
      a_shape.push_back(rT.d[i]);
    }
    nb = rT.n() / na;
  } else {
    for (int i = rT.r - n_a; i < rT.r; ++i) {
      na *= rT.d[i];
      a_shape.push_back(rT.d[i]);
    }
    nb = rT.n() / na;
  }
  ProjSaved ps;
  ps.na = (int)na;
  ps.nb = (int)nb;
  ps.chi = chi;
  ps.rows = rows;
  // FP64 copies of the half networks (the SVD side of the path is FP64)
  ps.rT = alloc(F64, {rows ? na : nb, rows ? nb : na});
  ps.rB = alloc(F64, {rows ? na : nb, rows ? nb : na});
  if (!dry && ok()) {
    if (rT.dt == F64) {
      check(hipMemcpyAsync(ps.rT.p, rT.p, rT.bytes(), hipMemcpyDeviceToDevice, s));
      check(hipMemcpyAsync(ps.rB.p, rB.p, rB.bytes(), hipMemcpyDeviceToDevice, s));
    } else {
      check(cast_f32_to_f64(s, rT.f32(), ps.rT.f64(), rT.n()));
      check(cast_f32_to_f64(s, rB.f32(), ps.rB.f64(), rB.n()));
    }
  }
  Ten Mm = alloc(F64, {nb, nb});
  if (rows)   // M = rho_B^T rho_T  (b x b)
    gemm(true, false, (int)nb, (int)nb, (int)na, 1.0, ps.rB, 0, nb, ps.rT, 0, nb, 0.0, Mm, 0, nb);
  else        // M = rho_B rho_T^T
    gemm(false, true, (int)nb, (int)nb, (int)na, 1.0, ps.rB, 0, na, ps.rT, 0, na, 0.0, Mm, 0, nb);
  ps.U = alloc(F64, {nb, nb});
  ps.S = alloc(F64, {nb});
  ps.V = alloc(F64, {nb, nb});
  {
    size_t mk = ar.mark();
    void* work = ar.alloc(svd_work_bytes((int)nb, 1));
    if (!dry && ok()) {
      int sweeps = 0;
      check(svd_f64(s, (int)nb, 1, Mm.f64(), ps.U.f64(), ps.S.f64(), ps.V.f64(), work, svd_max_sweeps, svd_tol,
                    host_flags, &sweeps));
      svd_sweeps_total += sweeps;
    }
    ar.release(mk);
  }
  ps.kr = alloc(F64, {2});   // holds two ints (k, r) in its first 8 bytes
  ps.X = alloc(F64, {nb, chi});
  ps.Y = alloc(F64, {nb, chi});
  if (!dry && ok()) {
    int* kr = (int*)ps.kr.p;
    check(trunc_scale(s, (int)nb, (int)nb, chi, ps.U.f64(), ps.S.f64(), cutoff, ps.X.f64(), kr, 1));
    check(trunc_scale(s, (int)nb, (int)nb, chi, ps.V.f64(), ps.S.f64(), cutoff, ps.Y.f64(), kr, 1));
    check(rank_count(s, (int)nb, ps.S.f64(), 1e-14, kr + 1));
  }
  Ten PT64 = alloc(F64, {na, chi}), PB64 = alloc(F64, {na, chi});
  if (rows) {   // P_T = rho_B X, P_B = rho_T Y
    gemm(false, false, (int)na, chi, (int)nb, 1.0, ps.rB, 0, nb, ps.X, 0, chi, 0.0, PT64, 0, chi);
    gemm(false, false, (int)na, chi, (int)nb, 1.0, ps.rT, 0, nb, ps.Y, 0, chi, 0.0, PB64, 0, chi);
  } else {      // P_T = rho_B^T X, P_B = rho_T^T Y
    gemm(true, false, (int)na, chi, (int)nb, 1.0, ps.rB, 0, na, ps.X, 0, chi, 0.0, PT64, 0, chi);
    gemm(true, false, (int)na, chi, (int)nb, 1.0, ps.rT, 0, na, ps.Y, 0, chi, 0.0, PB64, 0, chi);
  }
  ps.sgn = alloc(F64, {chi});
  if (!dry && ok()) check(sign_fix(s, (int)na, chi, PT64.f64(), PB64.f64(), ps.sgn.f64(), 1));
  if (spectrum_out && !dry && ok()) {
    spectrum_out->resize(nb);
    check(hipMemcpyAsync(spectrum_out->data(), ps.S.p, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    check(hipStreamSynchronize(s));
  }
  std::vector<long> pshape = a_shape;
  pshape.push_back(chi);
  Ten PT, PB;
  if (cdt == F64) {
    PT = PT64;
    PB = PB64;
  } else {
    PT = alloc(F32, {na, chi});
    PB = alloc(F32, {na, chi});
    if (!dry && ok()) {
      check(cast_f64_to_f32(s, PT64.f64(), PT.f32(), na * chi));
      check(cast_f64_to_f32(s, PB64.f64(), PB.f32(), na * chi));
    }
  }
  PT.r = PB.r = (int)pshape.size();
  for (size_t i = 0; i < pshape.size(); ++i) PT.d[i] = PB.d[i] = pshape[i];
  if (taping && (ng(rT) || ng(rB))) {
    TapeRec r;
    r.kind = OP_PROJ;
    r.in = {rT, rB};
    r.out = {PT, PB};
    r.proj = ps;
    record(std::move(r));
    needs_grad.insert(PT.id);
    needs_grad.insert(PB.id);
  }
  return {PT, PB};
}

Ten Engine::bond_energy(const Ten& rho, const Ten& h64, int p) {
  Ten r64 = cast(rho, F64);
  Ten e = alloc(F64, {2});
  if (!dry && ok()) check(sctm::bond_energy(s, p, r64.f64(), h64.f64(), e.f64()));
  if (taping && ng(r64)) {
    TapeRec r;
    r.kind = OP_BOND;
    r.in = {r64};
    r.out = {e};
    r.h = h64;
    r.p = p;
    record(std::move(r));
    needs_grad.insert(e.id);
  }
  return e;
}

// ---------------------------------------------------------------------------
// reverse pass
// ---------------------------------------------------------------------------
void Engine::backward() {
  bool saved = taping;
  taping = false;
  for (int i = (int)tape.size() - 1; i >= 0 && ok(); --i) {
    TapeRec& r = tape[i];
    bool any = false;
    for (auto& o : r.out) any = any || has_grad(o);
    if (!any) continue;
    switch (r.kind) {
      case OP_CONTRACT: {
        std::string lhs, lc;
        parse_arrow(r.spec, lhs, lc);
        size_t comma = lhs.find(',');
        std::string la = lhs.substr(0, comma), lb = lhs.substr(comma + 1);
        Ten Cb = grad(r.out[0]);
        if (ng(r.in[0])) contract_into(lc + "," + lb + "->" + la, Cb, r.in[1], grad(r.in[0]), true);
        if (ng(r.in[1])) contract_into(la + "," + lc + "->" + lb, r.in[0], Cb, grad(r.in[1]), true);
        break;
      }
      case OP_PERMUTE: {
        std::string li, lo;
        parse_arrow(r.spec, li, lo);
        permute_into(grad(r.out[0]), lo + "->" + li, grad(r.in[0]), true);
        break;
      }
      case OP_COPY:
        add_into(grad(r.out[0]), grad(r.in[0]));
        break;
      case OP_CAST:
        add_into(grad(r.out[0]), grad(r.in[0]));
        break;
      case OP_NORMALIZE: {
        Ten yb = grad(r.out[0]);
        Ten xb = grad(r.in[0]);
        Ten yd = alloc(F64, {1});
        if (!dry && ok()) {
          if (yb.dt == F64) {
            check(dot_f64(s, r.out[0].f64(), yb.f64(), yb.n(), partial, yd.f64()));
            check(normalize_adjoint_f64(s, r.out[0].f64(), yb.f64(), r.aux.f64(), yd.f64(), xb.f64(), yb.n()));
          } else {
            check(dot_f32(s, r.out[0].f32(), yb.f32(), yb.n(), partial, yd.f64()));
            check(normalize_adjoint_f32(s, r.out[0].f32(), yb.f32(), r.aux.f64(), yd.f64(), xb.f32(), yb.n()));
          }
        }
        break;
      }
      case OP_PROJ:
        proj_backward(r);
        break;
      case OP_BOND: {
        Ten eb = grad(r.out[0]);
        Ten rb = grad(r.in[0]);
        if (!dry && ok()) check(bond_energy_adjoint(s, r.p, r.h.f64(), r.out[0].f64(), eb.f64(), rb.f64()));
        break;
      }
    }
  }
  taping = saved;
}

// Reverse mode of the projector recipe.  With M = U S V^T (b x b), the kept
// k columns, X = U_k S_k^{-1/2}, Y = V_k S_k^{-1/2}, P_T = rho_B X sg,
// P_B = rho_T Y sg (sg = column signs):
//   Xbar = rho_B^T Pbar_T sg, Ybar = rho_T^T Pbar_B sg,
//   Ubar_k = Xbar S^{-1/2}, Vbar_k = Ybar S^{-1/2},
//   Sbar_k = -1/2 S^{-3/2} diag(U_k^T Xbar + V_k^T Ybar),
//   Mbar by the thin-SVD adjoint over the r = #{s > 1e-14 s_1} leading
//   triplets with the Lorentzian-broadened F (eps_F = (adj_eps s_1^2)^2):
//   Mbar = U [F o (G_U - G_U^T) S + S F o (G_V - G_V^T) + diag(Sbar)] V^T
//          + (Ubar - U G_U) S^{-1} V^T + U S^{-1} (Vbar - V G_V)^T,
//   G_U = U_r^T Ubar, G_V = V_r^T Vbar; then rho_Bbar += rho_T Mbar^T,
//   rho_Tbar += rho_B Mbar (rows case; the columns case is transposed).
// Ubar and Vbar have only chi nonzero columns, so every product is
// O(b^2 chi) except none: the inner matrix is split into its first chi rows
// and first chi columns.
void Engine::proj_backward(TapeRec& r) {
  ProjSaved& ps = r.proj;
  const int na = ps.na, nb = ps.nb, chi = ps.chi;
  const bool rows = ps.rows;
  const Ten PTg = grad(r.out[0]);
  const Ten PBg = grad(r.out[1]);
  Ten PTb = alloc(F64, {na, chi}), PBb = alloc(F64, {na, chi});
  if (!dry && ok()) {
    check(scale_cols_from(s, PTg.p, PTg.dt == F64, PTb.f64(), na, chi, ps.sgn.f64()));
    check(scale_cols_from(s, PBg.p, PBg.dt == F64, PBb.f64(), na, chi, ps.sgn.f64()));
  }
  Ten rTb = alloc(F64, {ps.rT.d[0], ps.rT.d[1]}), rBb = alloc(F64, {ps.rB.d[0], ps.rB.d[1]});
  zero(rTb);
  zero(rBb);
  Ten Xb = alloc(F64, {nb, chi}), Yb = alloc(F64, {nb, chi});
  if (rows) {
    gemm(false, true, na, nb, chi, 1.0, PTb, 0, chi, ps.X, 0, chi, 1.0, rBb, 0, nb);   // rBb += PTb X^T
    gemm(true, false, nb, chi, na, 1.0, ps.rB, 0, nb, PTb, 0, chi, 0.0, Xb, 0, chi);   // Xb = rB^T PTb
    gemm(false, true, na, nb, chi, 1.0, PBb, 0, chi, ps.Y, 0, chi, 1.0, rTb, 0, nb);
    gemm(true, false, nb, chi, na, 1.0, ps.rT, 0, nb, PBb, 0, chi, 0.0, Yb, 0, chi);
  } else {
    gemm(false, true, nb, na, chi, 1.0, ps.X, 0, chi, PTb, 0, chi, 1.0, rBb, 0, na);   // rBb += X PTb^T
    gemm(false, false, nb, chi, na, 1.0, ps.rB, 0, na, PTb, 0, chi, 0.0, Xb, 0, chi);  // Xb = rB PTb
    gemm(false, true, nb, na, chi, 1.0, ps.Y, 0, chi, PBb, 0, chi, 1.0, rTb, 0, na);
    gemm(false, false, nb, chi, na, 1.0, ps.rT, 0, na, PBb, 0, chi, 0.0, Yb, 0, chi);
  }
  // Ubar, Vbar, Sbar
  Ten Ub = alloc(F64, {nb, chi}), Vb = alloc(F64, {nb, chi}), Sb = alloc(F64, {chi});
  if (!dry && ok())
    check(svd_adj_prep(s, nb, chi, ps.U.f64(), ps.V.f64(), ps.S.f64(), (const int*)ps.kr.p, Xb.f64(), Yb.f64(),
                       Ub.f64(), Vb.f64(), Sb.f64()));
  // G_U = U^T Ubar, G_V = V^T Vbar (b x chi), rows >= r zeroed
  Ten GU = alloc(F64, {nb, chi}), GV = alloc(F64, {nb, chi});
  gemm(true, false, nb, chi, nb, 1.0, ps.U, 0, nb, Ub, 0, chi, 0.0, GU, 0, chi);
  gemm(true, false, nb, chi, nb, 1.0, ps.V, 0, nb, Vb, 0, chi, 0.0, GV, 0, chi);
  if (!dry && ok()) check(zero_rows_from(s, nb, chi, GU.f64(), GV.f64(), (const int*)ps.kr.p + 1));
  // inner blocks: top = inner[0:chi, :] (chi x b), left = inner[chi:, 0:chi] ((b-chi) x chi)
  const int c2 = std::min(chi, nb);
  Ten Itop = alloc(F64, {c2, nb});
  Ten Ileft = alloc(F64, {std::max(nb - c2, 1), c2});
  if (!dry && ok())
    check(svd_adj_inner(s, nb, c2, chi, ps.S.f64(), Sb.f64(), GU.f64(), GV.f64(), (const int*)ps.kr.p, adj_eps,
                        Itop.f64(), Ileft.f64()));
  // C1 = (Ubar - U G_U) S^{-1}, C2 = (Vbar - V G_V) S^{-1}   (b x chi)
  Ten C1 = alloc(F64, {nb, chi}), C2 = alloc(F64, {nb, chi});
  if (!dry && ok()) {
    check(hipMemcpyAsync(C1.p, Ub.p, Ub.bytes(), hipMemcpyDeviceToDevice, s));
    check(hipMemcpyAsync(C2.p, Vb.p, Vb.bytes(), hipMemcpyDeviceToDevice, s));
  }
  gemm(false, false, nb, chi, nb, -1.0, ps.U, 0, nb, GU, 0, chi, 1.0, C1, 0, chi);
  gemm(false, false, nb, chi, nb, -1.0, ps.V, 0, nb, GV, 0, chi, 1.0, C2, 0, chi);
  if (!dry && ok()) check(scale_cols_inv_s(s, nb, chi, C1.f64(), C2.f64(), ps.S.f64(), (const int*)ps.kr.p));
  // Q1 = Itop V^T + C2^T  (c2 x b);  Q2 = U[:, c2:] Ileft + C1[:, :c2]  (b x c2)
  Ten Q1 = alloc(F64, {c2, nb}), Q2 = alloc(F64, {nb, c2});
  gemm(false, true, c2, nb, nb, 1.0, Itop, 0, nb, ps.V, 0, nb, 0.0, Q1, 0, nb);
  if (!dry && ok()) check(add_transposed(s, nb, chi, c2, C2.f64(), Q1.f64()));   // Q1[c][b] += C2[b][c]
  if (!dry && ok()) check(copy_cols(s, nb, chi, c2, C1.f64(), Q2.f64()));         // Q2 = C1[:, :c2]
  if (nb > c2) gemm(false, false, nb, c2, nb - c2, 1.0, ps.U, c2, nb, Ileft, 0, c2, 1.0, Q2, 0, c2);
  // Mbar = U[:, :c2] Q1 + Q2 V[:, :c2]^T
  Ten Mb = alloc(F64, {nb, nb});
  gemm(false, false, nb, nb, c2, 1.0, ps.U, 0, nb, Q1, 0, nb, 0.0, Mb, 0, nb);
  gemm(false, true, nb, nb, c2, 1.0, Q2, 0, c2, ps.V, 0, nb, 1.0, Mb, 0, nb);
  // rho bars from M
  if (rows) {   // M = rB^T rT  (rho: na x nb)
    gemm(false, true, na, nb, nb, 1.0, ps.rT, 0, nb, Mb, 0, nb, 1.0, rBb, 0, nb);   // rBb += rT Mb^T
    gemm(false, false, na, nb, nb, 1.0, ps.rB, 0, nb, Mb, 0, nb, 1.0, rTb, 0, nb);  // rTb += rB Mb
  } else {      // M = rB rT^T  (rho: nb x na)
    gemm(false, false, nb, na, nb, 1.0, Mb, 0, nb, ps.rT, 0, na, 1.0, rBb, 0, na);  // rBb += Mb rT
    gemm(true, false, nb, na, nb, 1.0, Mb, 0, nb, ps.rB, 0, na, 1.0, rTb, 0, na);   // rTb += Mb^T rB
  }
  Ten gT = grad(r.in[0]);
  Ten gB = grad(r.in[1]);
  add_into(rTb, gT);
  add_into(rBb, gB);
}

}  // namespace sctm
