// Engine implementation: contraction planning, ops, and their adjoints.
#include "engine.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>

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
static bool trace_contractions() {
  static const bool on = getenv("SPLITCTM_TRACE") != nullptr;
  return on;
}

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
  // SPLITCTM_TRACE >= 2: every product synchronised and timed on the host,
  // with its shape and route (diagnostics; distorts the run's own timing)
  static const bool timed = [] {
    const char* e = getenv("SPLITCTM_TRACE");
    return e && atoi(e) >= 2;
  }();
  if (!timed || dry) {
    gemm_route(tA, tB, M, N, K, alpha, A, offA, lda, B, offB, ldb, beta, C, offC, ldc);
    return;
  }
  // us: device time of the product's kernels (events on the stream); host_us:
  // the same on the host clock, with launch and synchronisation overheads
  static hipEvent_t ev[2] = {nullptr, nullptr};
  if (!ev[0]) {
    check(hipEventCreate(&ev[0]));
    check(hipEventCreate(&ev[1]));
  }
  check(hipStreamSynchronize(s));
  const auto t0 = std::chrono::steady_clock::now();
  check(hipEventRecord(ev[0], s));
  const char* route = gemm_route(tA, tB, M, N, K, alpha, A, offA, lda, B, offB, ldb, beta, C, offC, ldc);
  check(hipEventRecord(ev[1], s));
  check(hipStreamSynchronize(s));
  const double hus = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  float ms = 0.f;
  check(hipEventElapsedTime(&ms, ev[0], ev[1]));
  fprintf(stderr, "[gemm] route=%s dt=%d tA=%d tB=%d M=%d N=%d K=%d lda=%ld ldb=%ld ldc=%ld beta=%g us=%.1f host_us=%.1f\n",
          route, C.dt, (int)tA, (int)tB, M, N, K, lda, ldb, ldc, beta, 1e3 * ms, hus);
}

const char* Engine::gemm_route(bool tA, bool tB, int M, int N, int K, double alpha, const Ten& A, long offA,
                               long lda, const Ten& B, long offB, long ldb, double beta, const Ten& C, long offC,
                               long ldc) {
  flops_gemm += 2L * M * N * K;
  // large BF16X3 products: operands split once into bf16 planes (scratch from the arena)
  if (C.dt == F32 && prec == Prec::BF16X3) {
    const size_t bb = bf16x3_big_scratch_bytes(M, N, K);
    if (bb > 0) {
      size_t mk = ar.mark();
      void* w = ar.alloc(bb);
      if (!dry && ok() && w)
        check(gemm_bf16x3_big(s, tA, tB, M, N, K, (float)alpha, A.f32() + offA, lda, B.f32() + offB, ldb,
                              (float)beta, C.f32() + offC, ldc, w));
      if (!w && !dry) status = 2;   // workspace exhausted
      ar.release(mk);
      return "presplit";
    }
  }
  // Split-K (long K, few output tiles): the scratch for the slices comes from the arena
  const long sk = splitk_scratch_elems(M, N, K);
  if (sk > 0) {
    size_t mk = ar.mark();
    Ten P = alloc(C.dt, {sk});
    if (!dry && ok()) {
      if (C.dt == F64)
        check(gemm_f64_splitk(s, tA, tB, M, N, K, alpha, A.f64() + offA, lda, B.f64() + offB, ldb, beta,
                              C.f64() + offC, ldc, P.f64()));
      else
        check(gemm_f32_splitk(s, prec, tA, tB, M, N, K, (float)alpha,
                              A.f32() + offA, lda, B.f32() + offB, ldb, (float)beta, C.f32() + offC, ldc, P.f32()));
    }
    ar.release(mk);
    return "splitk";
  }
  if (dry || !ok()) return "none";
  if (M <= 0 || N <= 0) return "none";
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
    return "none";
  }
  if (C.dt == F64)
    check(gemm_f64(s, tA, tB, M, N, K, alpha, A.f64() + offA, lda, 0, B.f64() + offB, ldb, 0, beta,
                   C.f64() + offC, ldc, 0, 1));
  else
    check(gemm_f32(s, prec, tA, tB, M, N, K, (float)alpha,
                   A.f32() + offA, lda, 0, B.f32() + offB, ldb, 0, (float)beta, C.f32() + offC, ldc, 0, 1));
  return "plain";
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
  if (trace_contractions()) fprintf(stderr, "[contract] %s M=%ld N=%ld K=%ld GF=%.3f\n", spec.c_str(), M, N, K, 2e-9 * M * N * K);
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
// Pairwise contraction order of a tensor network: exhaustive dynamic
// programming over subsets of the operands, minimising the total multiply-add
// count (ties: the smaller largest intermediate).  Every label occurs in two
// operands, or in one operand and the output, so each pairwise step is a plain
// GEMM-shaped contraction.  Plans are cached per (spec, dims).
struct PlanKey {
  std::string spec;
  std::vector<long> dims;
  bool operator==(const PlanKey& o) const { return spec == o.spec && dims == o.dims; }
};
struct PlanKeyHash {
  size_t operator()(const PlanKey& k) const {
    size_t h = std::hash<std::string>()(k.spec);
    for (long d : k.dims) h = h * 1000003u ^ std::hash<long>()(d);
    return h;
  }
};

static const ContractionPlan& plan_for(const std::string& spec, const std::vector<std::string>& terms,
                                       const std::string& out, const long* dims) {
  static std::unordered_map<PlanKey, ContractionPlan, PlanKeyHash> cache;
  PlanKey key{spec, {}};
  for (const auto& t : terms)
    for (char c : t) key.dims.push_back(dims[(unsigned char)c]);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;

  const int n = (int)terms.size();
  const int full = (1 << n) - 1;
  // labels of each operand as bit sets over the distinct labels
  std::string labels;
  for (const auto& t : terms)
    for (char c : t)
      if (labels.find(c) == std::string::npos) labels += c;
  const int nl = (int)labels.size();
  std::vector<unsigned long long> lab(n, 0ull);
  for (int i = 0; i < n; ++i)
    for (char c : terms[i]) lab[i] |= 1ull << labels.find(c);
  unsigned long long outl = 0;
  for (char c : out) outl |= 1ull << labels.find(c);
  std::vector<double> ld(nl);
  for (int k = 0; k < nl; ++k) ld[k] = (double)dims[(unsigned char)labels[k]];
  auto vol = [&](unsigned long long m) {
    double v = 1.0;
    for (int k = 0; k < nl; ++k)
      if (m >> k & 1) v *= ld[k];
    return v;
  };
  // open legs of every subset: labels of the subset also present outside it
  std::vector<unsigned long long> inner(full + 1, 0ull), legs(full + 1, 0ull);
  for (int S = 1; S <= full; ++S) {
    unsigned long long in = 0, outside = outl;
    for (int i = 0; i < n; ++i) (S >> i & 1 ? in : outside) |= lab[i];
    inner[S] = in;
    legs[S] = in & outside;
  }
  std::vector<double> cost(full + 1, 0.0), peak(full + 1, 0.0);
  std::vector<int> split(full + 1, 0);
  for (int S = 1; S <= full; ++S) {
    if ((S & (S - 1)) == 0) {
      cost[S] = 0.0;
      peak[S] = 0.0;
      continue;
    }
    double best = -1.0, bpk = 0.0;
    int bs = 0;
    // enumerate proper submasks S1 containing the lowest operand of S
    const int low = S & -S;
    for (int S1 = (S - 1) & S; S1 > 0; S1 = (S1 - 1) & S) {
      if (!(S1 & low)) continue;
      const int S2 = S ^ S1;
      const double f = vol(legs[S1] | legs[S2]);
      const double c = cost[S1] + cost[S2] + f;
      const double pk = std::max(std::max(peak[S1], peak[S2]), vol(legs[S]));
      if (best < 0 || c < best * (1 - 1e-12) || (c <= best * (1 + 1e-12) && pk < bpk)) {
        best = c;
        bpk = pk;
        bs = S1;
      }
    }
    cost[S] = best;
    peak[S] = bpk;
    split[S] = bs;
  }
  // emit the steps bottom-up; the label order of an intermediate is the kept
  // labels of its left part followed by those of its right part
  ContractionPlan plan;
  std::vector<std::string> names(terms);
  std::function<int(int)> emit = [&](int S) -> int {
    if ((S & (S - 1)) == 0) return __builtin_ctz(S);
    const int S1 = split[S], S2 = S ^ S1;
    const int a = emit(S1), b = emit(S2);
    std::string keep;
    for (char c : names[a])
      if (legs[S] >> labels.find(c) & 1) keep += c;
    for (char c : names[b])
      if ((legs[S] >> labels.find(c) & 1) && names[a].find(c) == std::string::npos) keep += c;
    plan.steps.push_back({a, b, keep});
    names.push_back(keep);
    return (int)names.size() - 1;
  };
  emit(full);
  plan.flops = 2.0 * cost[full];
  return cache.emplace(key, std::move(plan)).first->second;
}

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
  const ContractionPlan& plan = plan_for(spec, terms, out, dims);
  std::vector<std::pair<std::string, Ten>> items;
  for (size_t i = 0; i < terms.size(); ++i) items.push_back({terms[i], ops[i]});
  for (const auto& st : plan.steps) {
    auto& a = items[st.i];
    auto& b = items[st.j];
    Ten r = contract(a.first + "," + b.first + "->" + st.keep, a.second, b.second);
    items.push_back({st.keep, r});
  }
  items[0] = items.back();
  items.resize(1);
  if (items[0].first == out) return items[0].second;
  return permute(items[0].second, items[0].first + "->" + out);
}

// ---------------------------------------------------------------------------
// projectors
// ---------------------------------------------------------------------------
std::vector<Ten> Engine::projectors(const Ten& rT, const Ten& rB, int n_a, bool rows, int chi,
                                    std::vector<double>* spectrum_out) {
  ProjReq q{rT, rB, n_a, rows, chi, spectrum_out};
  return projectors_batch({q})[0];
}

static Ten view_of(Engine& E, const Ten& base, long off_elems, const std::vector<long>& dims) {
  Ten t;
  t.dt = base.dt;
  t.r = (int)dims.size();
  for (int i = 0; i < t.r; ++i) t.d[i] = dims[i];
  t.p = (char*)base.p + off_elems * base.esize();
  t.id = E.next_id++;
  return t;
}

// Projector pairs for several cuts at once.  All matrices handed to the
// Jacobi SVD that have the same size (the matrices M of the full-rank
// requests and the cores of the rank-limited ones) share one batched SVD:
// one launch per round for all of them.
std::vector<std::vector<Ten>> Engine::projectors_batch(const std::vector<ProjReq>& reqs) {
  const size_t nr = reqs.size();
  std::vector<std::vector<Ten>> result(nr);
  std::vector<ProjSaved> ps(nr);
  std::vector<std::vector<long>> a_shapes(nr);
  for (size_t i = 0; i < nr; ++i) {
    const ProjReq& q = reqs[i];
    long na = 1;
    if (q.rows) {
      for (int k = 0; k < q.n_a; ++k) {
        na *= q.rT.d[k];
        a_shapes[i].push_back(q.rT.d[k]);
      }
    } else {
      for (int k = q.rT.r - q.n_a; k < q.rT.r; ++k) {
        na *= q.rT.d[k];
        a_shapes[i].push_back(q.rT.d[k]);
      }
    }
    ps[i].na = (int)na;
    ps[i].nb = (int)(q.rT.n() / na);
    ps[i].chi = q.chi;
    ps[i].rows = q.rows;
  }
  // Route of every request: r0 > 0 when M = rho_B^T rho_T has rank <= r0 < n_b
  // by construction (r0 = n_a, or the bond of a given factorisation of
  // rho_T); M is then decomposed through an r0 x r0 core (Householder QR of
  // the two r0 x n_b factors, Jacobi SVD of the core).  Else one-sided
  // Jacobi on M itself.
  std::vector<long> r0(nr, 0);
  for (size_t i = 0; i < nr; ++i) {
    const ProjReq& q = reqs[i];
    long r = 0;
    if (q.fX.p && q.fZ.p && q.rows) r = q.fZ.n() / ps[i].nb;
    else if (ps[i].na < ps[i].nb) r = ps[i].na;
    if (r > 0 && r < ps[i].nb && ps[i].nb <= 8192 && lowrank_svd) r0[i] = r;
  }
  // groups of equal (n_b, r0), in request order
  struct Group {
    std::vector<size_t> idx;
    long nb = 0, rk = 0, n = 0;   // n: size of the matrices handed to the Jacobi SVD
    Ten Ub, Sb, Vb;               // n x n factors of M (rk = 0) or of its core (rk > 0)
    bool replayed = false;
    long job0 = 0;                // first entry in the Jacobi batch of size n
    Ten Xq, Rq, Qq;               // low-rank route: factors, R's and Q^T's (Q_L^T then Q_R^T, rk x nb each)
  };
  std::vector<Group> groups;
  {
    std::vector<char> handled(nr, 0);
    for (size_t g0 = 0; g0 < nr; ++g0) {
      if (handled[g0]) continue;
      Group G;
      for (size_t i = g0; i < nr; ++i)
        if (!handled[i] && ps[i].nb == ps[g0].nb && r0[i] == r0[g0]) {
          G.idx.push_back(i);
          handled[i] = 1;
        }
      G.nb = ps[g0].nb;
      G.rk = r0[g0];
      G.n = G.rk ? G.rk : G.nb;
      groups.push_back(std::move(G));
    }
  }
  // FP64 copies of the half networks (kept for the projector formation and the reverse pass)
  for (size_t i = 0; i < nr; ++i) {
    const ProjReq& q = reqs[i];
    ProjSaved& P = ps[i];
    const long na = P.na, nb = P.nb;
    P.rT = alloc(F64, {q.rows ? na : nb, q.rows ? nb : na});
    P.rB = alloc(F64, {q.rows ? na : nb, q.rows ? nb : na});
    if (!dry && ok()) {
      if (q.rT.dt == F64) {
        check(hipMemcpyAsync(P.rT.p, q.rT.p, q.rT.bytes(), hipMemcpyDeviceToDevice, s));
        check(hipMemcpyAsync(P.rB.p, q.rB.p, q.rB.bytes(), hipMemcpyDeviceToDevice, s));
      } else {
        check(cast_f32_to_f64(s, q.rT.f32(), P.rT.f64(), q.rT.n()));
        check(cast_f32_to_f64(s, q.rB.f32(), P.rB.f64(), q.rB.n()));
      }
    }
  }
  // replay of recorded decompositions (same group order as when recorded):
  // U, S, V of size n, and for the low-rank route the Q^T factors
  for (Group& G : groups) {
    const long nb = G.nb, n = G.n, rk = G.rk, g = (long)G.idx.size();
    if (svdc_mode != 2 || svdc_slot < 0) continue;
    SvdCacheSlot& sl = svdc_slots[svdc_slot];
    if (sl.valid && svdc_cursor < sl.off.size() && sl.nb[svdc_cursor] == nb && sl.g[svdc_cursor] == g &&
        sl.rk[svdc_cursor] == rk) {
      G.Ub = alloc(F64, {g, n, n});
      G.Sb = alloc(F64, {g, n});
      G.Vb = alloc(F64, {g, n, n});
      if (rk) G.Qq = alloc(F64, {2 * g, rk, nb});
      if (!dry && ok()) {
        const double* src = svdc_buf.f64() + (long)svdc_slot * svdc_per_slot + sl.off[svdc_cursor];
        const long un = g * n * n, sn = g * n;
        check(hipMemcpyAsync(G.Ub.p, src, sizeof(double) * un, hipMemcpyDeviceToDevice, s));
        check(hipMemcpyAsync(G.Sb.p, src + un, sizeof(double) * sn, hipMemcpyDeviceToDevice, s));
        check(hipMemcpyAsync(G.Vb.p, src + un + sn, sizeof(double) * un, hipMemcpyDeviceToDevice, s));
        if (rk)
          check(hipMemcpyAsync(G.Qq.p, src + 2 * un + sn, sizeof(double) * 2 * g * rk * nb, hipMemcpyDeviceToDevice,
                               s));
      }
      ++svdc_cursor;
      G.replayed = true;
    } else {
      sl.valid = false;   // out of step with the recording: recompute from here on
    }
  }
  // one Jacobi batch per matrix size over all groups still to decompose
  std::vector<long> sizes;
  std::unordered_map<long, long> jobs;       // n -> batch entries
  for (Group& G : groups) {
    if (G.replayed) continue;
    if (!jobs.count(G.n)) sizes.push_back(G.n);
    G.job0 = jobs[G.n];
    jobs[G.n] += (long)G.idx.size();
  }
  std::unordered_map<long, Ten> jU, jS, jV;   // Jacobi outputs (persist: views are kept for the reverse pass)
  for (long n : sizes) {
    jU[n] = alloc(F64, {jobs[n], n, n});
    jS[n] = alloc(F64, {jobs[n], n});
    jV[n] = alloc(F64, {jobs[n], n, n});
  }
  for (Group& G : groups) {
    if (G.replayed) continue;
    const long n = G.n, g = (long)G.idx.size();
    // the Jacobi outputs are the factors themselves (of the core on the
    // low-rank route, whose Q^T factors are kept beside them)
    G.Ub = view_of(*this, jU[n], G.job0 * n * n, {g, n, n});
    G.Sb = view_of(*this, jS[n], G.job0 * n, {g, n});
    G.Vb = view_of(*this, jV[n], G.job0 * n * n, {g, n, n});
    if (G.rk) G.Qq = alloc(F64, {2 * g, G.rk, G.nb});
  }
  size_t mk = ar.mark();   // transient from here: Jacobi inputs, QR buffers, workspaces
  std::unordered_map<long, Ten> jM;
  for (long n : sizes) jM[n] = alloc(F64, {jobs[n], n, n});
  for (Group& G : groups) {
    if (G.replayed) continue;
    const long nb = G.nb, rk = G.rk, g = (long)G.idx.size();
    if (!rk) {   // M = rho_B^T rho_T straight into the Jacobi batch
      for (long j = 0; j < g; ++j) {
        const ProjSaved& P = ps[G.idx[j]];
        const long na = P.na, off = (G.job0 + j) * nb * nb;
        if (P.rows)
          gemm(true, false, (int)nb, (int)nb, (int)na, 1.0, P.rB, 0, nb, P.rT, 0, nb, 0.0, jM[nb], off, nb);
        else
          gemm(false, true, (int)nb, (int)nb, (int)na, 1.0, P.rB, 0, na, P.rT, 0, na, 0.0, jM[nb], off, nb);
      }
      continue;
    }
    // M = L^T R with L, R: r0 x n_b  (entries 0..g-1: L, g..2g-1: R)
    G.Xq = alloc(F64, {2 * g, rk, nb});
    G.Rq = alloc(F64, {2 * g, rk, rk});
    for (long j = 0; j < g; ++j) {
      const ProjReq& q = reqs[G.idx[j]];
      const ProjSaved& P = ps[G.idx[j]];
      const long na = P.na, offL = j * rk * nb, offR = (g + j) * rk * nb;
      if (q.fX.p && q.fZ.p && q.rows && rk == q.fZ.n() / nb) {   // L = fX^T rho_B, R = fZ
        size_t m2 = ar.mark();
        Ten fX = alloc(F64, {na, rk});
        if (!dry && ok()) {
          if (q.fX.dt == F64) {
            check(hipMemcpyAsync(fX.p, q.fX.p, q.fX.bytes(), hipMemcpyDeviceToDevice, s));
            check(hipMemcpyAsync(G.Xq.f64() + offR, q.fZ.p, q.fZ.bytes(), hipMemcpyDeviceToDevice, s));
          } else {
            check(cast_f32_to_f64(s, q.fX.f32(), fX.f64(), q.fX.n()));
            check(cast_f32_to_f64(s, q.fZ.f32(), G.Xq.f64() + offR, q.fZ.n()));
          }
        }
        gemm(true, false, (int)rk, (int)nb, (int)na, 1.0, fX, 0, rk, P.rB, 0, nb, 0.0, G.Xq, offL, nb);
        ar.release(m2);
      } else if (P.rows) {   // L = rho_B, R = rho_T  (n_a x n_b)
        if (!dry && ok()) {
          check(hipMemcpyAsync(G.Xq.f64() + offL, P.rB.p, P.rB.bytes(), hipMemcpyDeviceToDevice, s));
          check(hipMemcpyAsync(G.Xq.f64() + offR, P.rT.p, P.rT.bytes(), hipMemcpyDeviceToDevice, s));
        }
      } else {               // rho stored n_b x n_a: L = rho_B^T, R = rho_T^T
        permute_into(P.rB, "ab->ba", view_of(*this, G.Xq, offL, {rk, nb}), false);
        permute_into(P.rT, "ab->ba", view_of(*this, G.Xq, offR, {rk, nb}), false);
      }
    }
    // Q_L R_L = L^T, Q_R R_R = R^T;  M = Q_L (R_L R_R^T) Q_R^T;  the core goes into the Jacobi batch
    void* qwork = ar.alloc(qr_work_bytes((int)nb, (int)rk, 2 * (int)g));
    if (!dry && ok()) {
      const long rr = rk * rk;
      static const bool qtrace = getenv("SPLITCTM_SVD_TRACE") != nullptr;
      auto q0 = std::chrono::steady_clock::now();
      if (qtrace) check(hipStreamSynchronize(s));
      // the Q factors are read only after the SVD: formed on the second
      // stream (qwork stays allocated until the join below)
      check(qr_f64_factor(s, (int)nb, (int)rk, 2 * (int)g, G.Xq.f64(), G.Rq.f64(), qwork));
      if (aux) {
        check(hipEventRecord(aux_ev[3], s));
        check(hipStreamWaitEvent(aux, aux_ev[3], 0));
        check(qr_f64_form_q(aux, (int)nb, (int)rk, 2 * (int)g, G.Qq.f64(), qwork));
      } else {
        check(qr_f64_form_q(s, (int)nb, (int)rk, 2 * (int)g, G.Qq.f64(), qwork));
      }
      if (qtrace && ok()) {
        check(hipStreamSynchronize(s));
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - q0).count();
        fprintf(stderr, "[qr] m=%ld k=%ld batch=%ld %.1f ms\n", nb, rk, 2 * g, ms);
      }
      check(gemm_f64(s, false, true, (int)rk, (int)rk, (int)rk, 1.0, G.Rq.f64(), rk, rr, G.Rq.f64() + g * rr, rk, rr,
                     0.0, jM[rk].f64() + G.job0 * rr, rk, rr, (int)g));
    }
  }
  for (long n : sizes) {
    void* work = ar.alloc(svd_precond_work_bytes((int)n, (int)jobs[n]));
    if (dry || !ok()) continue;
    int sweeps = 0;
    static const bool trace = getenv("SPLITCTM_SVD_TRACE") != nullptr;
    auto t0 = std::chrono::steady_clock::now();
    if (trace) check(hipStreamSynchronize(s));
    check(svd_precond_f64(s, (int)n, (int)jobs[n], jM[n].f64(), jU[n].f64(), jS[n].f64(), jV[n].f64(), work,
                          svd_max_sweeps, svd_tol, host_flags, &sweeps, aux, aux ? aux_ev : nullptr));
    svd_sweeps_total += sweeps;
    svd_calls += 1;
    if (trace && ok()) {
      check(hipStreamSynchronize(s));
      const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      fprintf(stderr, "[svd] n=%ld batch=%ld sweeps=%d %.1f ms\n", n, jobs[n], sweeps, ms);
      // how far each spectrum reaches: counts of s > 10^-k s_1
      std::vector<double> hs((size_t)jobs[n] * n);
      check(hipMemcpy(hs.data(), jS[n].p, sizeof(double) * hs.size(), hipMemcpyDeviceToHost));
      for (long b = 0; b < jobs[n]; ++b) {
        const double* S = hs.data() + b * n;
        int c[8] = {0};
        for (long i = 0; i < n; ++i)
          for (int k = 0; k < 8; ++k)
            if (S[i] > std::pow(10.0, -2.0 * (k + 1)) * S[0]) ++c[k];
        fprintf(stderr, "[spectrum] n=%ld entry=%ld above 1e-2..1e-16: %d %d %d %d %d %d %d %d  s_chi+1/s_chi=%.4f\n", n, b,
                c[0], c[1], c[2], c[3], c[4], c[5], c[6], c[7], n > 128 && S[127] > 0 ? S[128] / S[127] : 0.0);
      }
    }
  }
  // low-rank route: M = Q_L (U' S V'^T) Q_R^T stays in that factored form (the
  // QR wrote Q_L^T, Q_R^T into the persistent G.Qq); U = Q_L U', V = Q_R V' are
  // formed only for the kept columns, below.  Everything queued on the second
  // stream (the Q factors and their QR workspaces) is joined before the
  // transient memory is released or G.Qq is read.
  if (aux && !dry && ok()) {
    check(hipEventRecord(aux_ev[2], aux));
    check(hipStreamWaitEvent(s, aux_ev[2], 0));
  }
  ar.release(mk);
  // record the decompositions of this call for a later replay
  for (Group& G : groups) {
    if (G.replayed || svdc_mode != 1 || svdc_slot < 0) continue;
    const long nb = G.nb, n = G.n, rk = G.rk, g = (long)G.idx.size();
    SvdCacheSlot& sl = svdc_slots[svdc_slot];
    const long un = g * n * n, sn = g * n, qn = rk ? 2 * g * rk * nb : 0;
    const long need = ((2 * un + sn + qn + 31) / 32) * 32;
    if (sl.valid && sl.used + need <= sl.cap) {
      if (!dry && ok()) {
        double* dst = svdc_buf.f64() + (long)svdc_slot * svdc_per_slot + sl.used;
        check(hipMemcpyAsync(dst, G.Ub.p, sizeof(double) * un, hipMemcpyDeviceToDevice, s));
        check(hipMemcpyAsync(dst + un, G.Sb.p, sizeof(double) * sn, hipMemcpyDeviceToDevice, s));
        check(hipMemcpyAsync(dst + un + sn, G.Vb.p, sizeof(double) * un, hipMemcpyDeviceToDevice, s));
        if (rk) check(hipMemcpyAsync(dst + 2 * un + sn, G.Qq.p, sizeof(double) * qn, hipMemcpyDeviceToDevice, s));
      }
      sl.off.push_back(sl.used);
      sl.nb.push_back(nb);
      sl.g.push_back(g);
      sl.rk.push_back(rk);
      sl.used += need;
    } else {
      sl.valid = false;   // a later replay of this move recomputes everything
    }
  }
  // projector formation
  for (Group& G : groups) {
    const long nb = G.nb, n = G.n, rk = G.rk, g = (long)G.idx.size();
    for (size_t j = 0; j < G.idx.size(); ++j) {
      const size_t i = G.idx[j];
      const ProjReq& q = reqs[i];
      ProjSaved& P = ps[i];
      const long na = P.na;
      const int chi = q.chi;
      P.rk = (int)rk;
      P.U = view_of(*this, G.Ub, (long)j * n * n, {n, n});
      P.S = view_of(*this, G.Sb, (long)j * n, {n});
      P.V = view_of(*this, G.Vb, (long)j * n * n, {n, n});
      if (rk) {
        P.QLt = view_of(*this, G.Qq, (long)j * rk * nb, {rk, nb});
        P.QRt = view_of(*this, G.Qq, (long)(g + j) * rk * nb, {rk, nb});
      }
      P.kr = alloc(F64, {2});   // two ints (k, r) in its first 8 bytes
      P.X = alloc(F64, {nb, chi});
      P.Y = alloc(F64, {nb, chi});
      if (!dry && ok()) {
        int* kr = (int*)P.kr.p;
        if (!rk) {
          check(trunc_scale(s, (int)nb, (int)nb, chi, P.U.f64(), P.S.f64(), cutoff, P.X.f64(), kr, 1));
          check(trunc_scale(s, (int)nb, (int)nb, chi, P.V.f64(), P.S.f64(), cutoff, P.Y.f64(), kr, 1));
        }
        check(rank_count(s, (int)n, P.S.f64(), 1e-14, kr + 1));
      }
      if (rk) {   // X = Q_L (U'_k S_k^{-1/2}), Y = Q_R (V'_k S_k^{-1/2}): the kept columns only
        size_t m3 = ar.mark();
        Ten Xc = alloc(F64, {rk, chi}), Yc = alloc(F64, {rk, chi});
        if (!dry && ok()) {
          int* kr = (int*)P.kr.p;
          check(trunc_scale(s, (int)rk, (int)rk, chi, P.U.f64(), P.S.f64(), cutoff, Xc.f64(), kr, 1));
          check(trunc_scale(s, (int)rk, (int)rk, chi, P.V.f64(), P.S.f64(), cutoff, Yc.f64(), kr, 1));
        }
        gemm(true, false, (int)nb, chi, (int)rk, 1.0, P.QLt, 0, nb, Xc, 0, chi, 0.0, P.X, 0, chi);
        gemm(true, false, (int)nb, chi, (int)rk, 1.0, P.QRt, 0, nb, Yc, 0, chi, 0.0, P.Y, 0, chi);
        ar.release(m3);
      }
      Ten PT64 = alloc(F64, {na, chi}), PB64 = alloc(F64, {na, chi});
      if (q.rows) {   // P_T = rho_B X, P_B = rho_T Y
        gemm(false, false, (int)na, chi, (int)nb, 1.0, P.rB, 0, nb, P.X, 0, chi, 0.0, PT64, 0, chi);
        gemm(false, false, (int)na, chi, (int)nb, 1.0, P.rT, 0, nb, P.Y, 0, chi, 0.0, PB64, 0, chi);
      } else {        // P_T = rho_B^T X, P_B = rho_T^T Y
        gemm(true, false, (int)na, chi, (int)nb, 1.0, P.rB, 0, na, P.X, 0, chi, 0.0, PT64, 0, chi);
        gemm(true, false, (int)na, chi, (int)nb, 1.0, P.rT, 0, na, P.Y, 0, chi, 0.0, PB64, 0, chi);
      }
      P.sgn = alloc(F64, {chi});
      if (!dry && ok()) check(sign_fix(s, (int)na, chi, PT64.f64(), PB64.f64(), P.sgn.f64(), 1));
      if (q.spectrum_out && !dry && ok()) {   // the nonzero part of M's spectrum (length n)
        q.spectrum_out->resize(n);
        check(hipMemcpyAsync(q.spectrum_out->data(), P.S.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        check(hipStreamSynchronize(s));
      }
      std::vector<long> pshape = a_shapes[i];
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
      for (size_t k = 0; k < pshape.size(); ++k) PT.d[k] = PB.d[k] = pshape[k];
      if (taping && (ng(q.rT) || ng(q.rB))) {
        TapeRec r;
        r.kind = OP_PROJ;
        r.in = {q.rT, q.rB};
        r.out = {PT, PB};
        r.proj = P;
        record(std::move(r));
        needs_grad.insert(PT.id);
        needs_grad.insert(PB.id);
      }
      result[i] = {PT, PB};
    }
  }
  return result;
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
//   triplets with the Lorentzian-broadened F (eps_ij = (adj_eps (s_i^2 + s_j^2))^2):
//   Mbar = U [F o (G_U - G_U^T) S + S F o (G_V - G_V^T) + diag(Sbar)] V^T
//          + (Ubar - U G_U) S^{-1} V^T + U S^{-1} (Vbar - V G_V)^T,
//   G_U = U_r^T Ubar, G_V = V_r^T Vbar; then rho_Bbar += rho_T Mbar^T,
//   rho_Tbar += rho_B Mbar (rows case; the columns case is transposed).
// Ubar and Vbar have only chi nonzero columns, so every product is
// O(b^2 chi): the inner matrix is split into its first chi rows and first chi
// columns.  On the low-rank route (M = Q_L K Q_R^T, K = U' S V'^T of size
// rk) the same formula runs in the core's basis with U = Q_L U', V = Q_R V'
// and the complement term taken in the full space, so every product is
// O(b rk chi) and no b x b factor is ever formed.
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
  // Mbar in the factored form U_c Q1 + Q2 V_c^T (U_c, V_c: n_b x c2, the first
  // c2 singular vectors, at leading dimension ldu, ldv)
  Ten Q1, Q2, Ucm, Vcm;
  long ldu = nb, ldv = nb;
  int c2 = std::min(chi, nb);
  if (!ps.rk) {
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
    Q1 = alloc(F64, {c2, nb});
    Q2 = alloc(F64, {nb, c2});
    gemm(false, true, c2, nb, nb, 1.0, Itop, 0, nb, ps.V, 0, nb, 0.0, Q1, 0, nb);
    if (!dry && ok()) check(add_transposed(s, nb, chi, c2, C2.f64(), Q1.f64()));   // Q1[c][b] += C2[b][c]
    if (!dry && ok()) check(copy_cols(s, nb, chi, c2, C1.f64(), Q2.f64()));         // Q2 = C1[:, :c2]
    if (nb > c2) gemm(false, false, nb, c2, nb - c2, 1.0, ps.U, c2, nb, Ileft, 0, c2, 1.0, Q2, 0, c2);
    Ucm = ps.U;
    Vcm = ps.V;
  } else {
    // M = Q_L K Q_R^T with the core K = U' S V'^T (rk x rk) and Q_L^T Q_L =
    // Q_R^T Q_R = 1: U = Q_L U' and V = Q_R V' span the column and row spaces
    // of M, and the same adjoint runs in the core's basis.  Ubar splits into
    // its part in span(Q_L), Q_L (Q_L^T Ubar), and the rest, which enters
    // through the complement term (Ubar - U U^T Ubar) S^{-1} only.
    const int rk = ps.rk;
    c2 = std::min(chi, rk);
    Ten Xc = alloc(F64, {rk, chi}), Yc = alloc(F64, {rk, chi});
    gemm(false, false, rk, chi, nb, 1.0, ps.QLt, 0, nb, Xb, 0, chi, 0.0, Xc, 0, chi);   // Q_L^T Xbar
    gemm(false, false, rk, chi, nb, 1.0, ps.QRt, 0, nb, Yb, 0, chi, 0.0, Yc, 0, chi);   // Q_R^T Ybar
    Ten Ubc = alloc(F64, {rk, chi}), Vbc = alloc(F64, {rk, chi}), Sb = alloc(F64, {chi});
    Ten Ub = alloc(F64, {nb, chi}), Vb = alloc(F64, {nb, chi});
    if (!dry && ok()) {
      // core: Ubar' = Q_L^T Ubar and Sbar (u_c . xbar_c = u'_c . (Q_L^T xbar)_c)
      check(svd_adj_prep(s, rk, chi, ps.U.f64(), ps.V.f64(), ps.S.f64(), (const int*)ps.kr.p, Xc.f64(), Yc.f64(),
                         Ubc.f64(), Vbc.f64(), Sb.f64()));
      // full space: Ubar = Xbar S^{-1/2}, Vbar = Ybar S^{-1/2}
      check(scale_cols_rsqrt_s(s, nb, chi, Xb.f64(), ps.S.f64(), (const int*)ps.kr.p, Ub.f64()));
      check(scale_cols_rsqrt_s(s, nb, chi, Yb.f64(), ps.S.f64(), (const int*)ps.kr.p, Vb.f64()));
    }
    // G_U = U'^T Ubar' = U^T Ubar, G_V likewise (rk x chi), rows >= r zeroed
    Ten GU = alloc(F64, {rk, chi}), GV = alloc(F64, {rk, chi});
    gemm(true, false, rk, chi, rk, 1.0, ps.U, 0, rk, Ubc, 0, chi, 0.0, GU, 0, chi);
    gemm(true, false, rk, chi, rk, 1.0, ps.V, 0, rk, Vbc, 0, chi, 0.0, GV, 0, chi);
    if (!dry && ok()) check(zero_rows_from(s, rk, chi, GU.f64(), GV.f64(), (const int*)ps.kr.p + 1));
    // inner blocks in the core's basis (the inner matrix vanishes beyond rk)
    Ten Itop = alloc(F64, {c2, rk});
    Ten Ileft = alloc(F64, {std::max(rk - c2, 1), c2});
    if (!dry && ok())
      check(svd_adj_inner(s, rk, c2, chi, ps.S.f64(), Sb.f64(), GU.f64(), GV.f64(), (const int*)ps.kr.p, adj_eps,
                          Itop.f64(), Ileft.f64()));
    // C1 = (Ubar - Q_L (U' G_U)) S^{-1}, C2 = (Vbar - Q_R (V' G_V)) S^{-1}  (nb x chi, in place)
    Ten T1 = alloc(F64, {rk, chi}), T2 = alloc(F64, {rk, chi});
    gemm(false, false, rk, chi, rk, 1.0, ps.U, 0, rk, GU, 0, chi, 0.0, T1, 0, chi);
    gemm(false, false, rk, chi, rk, 1.0, ps.V, 0, rk, GV, 0, chi, 0.0, T2, 0, chi);
    Ten C1 = Ub, C2 = Vb;
    gemm(true, false, nb, chi, rk, -1.0, ps.QLt, 0, nb, T1, 0, chi, 1.0, C1, 0, chi);
    gemm(true, false, nb, chi, rk, -1.0, ps.QRt, 0, nb, T2, 0, chi, 1.0, C2, 0, chi);
    if (!dry && ok()) check(scale_cols_inv_s(s, nb, chi, C1.f64(), C2.f64(), ps.S.f64(), (const int*)ps.kr.p));
    // U_c = Q_L U'[:, :c2], V_c = Q_R V'[:, :c2]  (nb x c2)
    Ucm = alloc(F64, {nb, c2});
    Vcm = alloc(F64, {nb, c2});
    gemm(true, false, nb, c2, rk, 1.0, ps.QLt, 0, nb, ps.U, 0, rk, 0.0, Ucm, 0, c2);
    gemm(true, false, nb, c2, rk, 1.0, ps.QRt, 0, nb, ps.V, 0, rk, 0.0, Vcm, 0, c2);
    ldu = ldv = c2;
    // Q1 = (Itop V'^T) Q_R^T + C2^T  (c2 x nb)
    Ten T3 = alloc(F64, {c2, rk});
    gemm(false, true, c2, rk, rk, 1.0, Itop, 0, rk, ps.V, 0, rk, 0.0, T3, 0, rk);
    Q1 = alloc(F64, {c2, nb});
    gemm(false, false, c2, nb, rk, 1.0, T3, 0, rk, ps.QRt, 0, nb, 0.0, Q1, 0, nb);
    if (!dry && ok()) check(add_transposed(s, nb, chi, c2, C2.f64(), Q1.f64()));
    // Q2 = Q_L (U'[:, c2:] Ileft) + C1[:, :c2]  (nb x c2)
    Q2 = alloc(F64, {nb, c2});
    if (!dry && ok()) check(copy_cols(s, nb, chi, c2, C1.f64(), Q2.f64()));
    if (rk > c2) {
      Ten T4 = alloc(F64, {rk, c2});
      gemm(false, false, rk, c2, rk - c2, 1.0, ps.U, c2, rk, Ileft, 0, c2, 0.0, T4, 0, c2);
      gemm(true, false, nb, c2, rk, 1.0, ps.QLt, 0, nb, T4, 0, c2, 1.0, Q2, 0, c2);
    }
  }
  // Mbar = U_c Q1 + Q2 V_c^T has rank <= 2 c2; the rho bars take it in this
  // factored form (never the b x b matrix): O(na b c2) instead of O(na b^2)
  Ten A1 = alloc(F64, {na, c2}), A2 = alloc(F64, {na, c2});
  if (rows) {   // M = rB^T rT  (rho: na x nb)
    // rBb += rT Mb^T = (rT Q1^T) U_c^T + (rT V_c) Q2^T
    gemm(false, true, na, c2, nb, 1.0, ps.rT, 0, nb, Q1, 0, nb, 0.0, A1, 0, c2);
    gemm(false, false, na, c2, nb, 1.0, ps.rT, 0, nb, Vcm, 0, ldv, 0.0, A2, 0, c2);
    gemm(false, true, na, nb, c2, 1.0, A1, 0, c2, Ucm, 0, ldu, 1.0, rBb, 0, nb);
    gemm(false, true, na, nb, c2, 1.0, A2, 0, c2, Q2, 0, c2, 1.0, rBb, 0, nb);
    // rTb += rB Mb = (rB U_c) Q1 + (rB Q2) V_c^T
    gemm(false, false, na, c2, nb, 1.0, ps.rB, 0, nb, Ucm, 0, ldu, 0.0, A1, 0, c2);
    gemm(false, false, na, c2, nb, 1.0, ps.rB, 0, nb, Q2, 0, c2, 0.0, A2, 0, c2);
    gemm(false, false, na, nb, c2, 1.0, A1, 0, c2, Q1, 0, nb, 1.0, rTb, 0, nb);
    gemm(false, true, na, nb, c2, 1.0, A2, 0, c2, Vcm, 0, ldv, 1.0, rTb, 0, nb);
  } else {      // M = rB rT^T  (rho: nb x na); A1, A2 hold c2 x na products here
    // rBb += Mb rT = U_c (Q1 rT) + Q2 (V_c^T rT)
    gemm(false, false, c2, na, nb, 1.0, Q1, 0, nb, ps.rT, 0, na, 0.0, A1, 0, na);
    gemm(true, false, c2, na, nb, 1.0, Vcm, 0, ldv, ps.rT, 0, na, 0.0, A2, 0, na);
    gemm(false, false, nb, na, c2, 1.0, Ucm, 0, ldu, A1, 0, na, 1.0, rBb, 0, na);
    gemm(false, false, nb, na, c2, 1.0, Q2, 0, c2, A2, 0, na, 1.0, rBb, 0, na);
    // rTb += Mb^T rB = Q1^T (U_c^T rB) + V_c (Q2^T rB)
    gemm(true, false, c2, na, nb, 1.0, Ucm, 0, ldu, ps.rB, 0, na, 0.0, A1, 0, na);
    gemm(true, false, c2, na, nb, 1.0, Q2, 0, c2, ps.rB, 0, na, 0.0, A2, 0, na);
    gemm(true, false, nb, na, c2, 1.0, Q1, 0, nb, A1, 0, na, 1.0, rTb, 0, na);
    gemm(false, false, nb, na, c2, 1.0, Vcm, 0, ldv, A2, 0, na, 1.0, rTb, 0, na);
  }
  Ten gT = grad(r.in[0]);
  Ten gB = grad(r.in[1]);
  add_into(rTb, gT);
  add_into(rBb, gB);
}

}  // namespace sctm
