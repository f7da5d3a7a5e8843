// Host-side launchers of the HIP kernels of the split-CTMRG library (gfx950).
// Every launcher enqueues on the given stream and returns hipError_t.
#pragma once
#include <hip/hip_runtime.h>

#include "timer.hpp"
#include <cstdint>

namespace sctm {

enum class Prec : int { F64 = 0, F32 = 1, BF16X3 = 2, BF16X6 = 3 };

// C[M,N] = alpha * op(A)[M,K] * op(B)[K,N] + beta * C, all row-major.
// transA: A is stored K x M (leading dimension lda); else M x K.
// transB: B is stored N x K; else K x N.  batch problems at strides sA,sB,sC.
hipError_t gemm_f64(hipStream_t s, bool transA, bool transB, int M, int N, int K,
                    double alpha, const double* A, long lda, long sA,
                    const double* B, long ldb, long sB, double beta,
                    double* C, long ldc, long sC, int batch);
// K-sliced batched FP64 product: P[b][sl] = op(A_b) op(B_b) over the sl-th of
// S slices of length ceil(K / S) (every slice non-empty), P[b][sl] row-major
// M x N at stride M N, entry b at stride S M N.  The caller sums the slices.
hipError_t gemm_f64_slices(hipStream_t s, bool transA, bool transB, int M, int N, int K, const double* A, long lda,
                           long sA, const double* B, long ldb, long sB, double* P, int S, int batch);
hipError_t gemm_f32(hipStream_t s, Prec mode, bool transA, bool transB, int M, int N, int K,
                    float alpha, const float* A, long lda, long sA,
                    const float* B, long ldb, long sB, float beta,
                    float* C, long ldc, long sC, int batch);

// out = permute(in): out dims are in dims taken in order perm; elements of size esize.
struct PermDesc {
  int rank;
  long out_dims[12];
  long in_strides_perm[12];  // stride in the input of output axis i
};
hipError_t permute(hipStream_t s, int esize, const void* in, void* out, const PermDesc& d, long n,
                   bool accumulate);

// Elementwise helpers (FP64 or FP32 depending on the suffix).
hipError_t fill_f64(hipStream_t s, double* p, double v, long n);
hipError_t fill_f32(hipStream_t s, float* p, float v, long n);
hipError_t cast_f32_to_f64(hipStream_t s, const float* in, double* out, long n);
hipError_t cast_f64_to_f32(hipStream_t s, const double* in, float* out, long n);
hipError_t axpy_f64(hipStream_t s, double a, const double* x, double* y, long n);
// Split-K products (used when the output has few tiles and K is long; else a
// plain product): scratch = splitk_scratch_elems(M, N, K) elements.
long splitk_scratch_elems(int M, int N, int K);
hipError_t gemm_f64_splitk(hipStream_t s, bool tA, bool tB, int M, int N, int K, double alpha, const double* A,
                           long lda, const double* B, long ldb, double beta, double* C, long ldc, double* scratch);
hipError_t gemm_f32_splitk(hipStream_t s, Prec mode, bool tA, bool tB, int M, int N, int K, float alpha,
                           const float* A, long lda, const float* B, long ldb, float beta, float* C, long ldc,
                           float* scratch);
// Large BF16X3 products (both output dimensions >= 1024, 2^31 multiply-adds
// or more): operands split once into k-contiguous bf16 planes,
// 128 x 128 tiles; scratch = bf16x3_big_scratch_bytes(M, N, K) bytes, 0 when
// the shape takes the plain kernel (gemm_bf16x3_big then fails).
size_t bf16x3_big_scratch_bytes(int M, int N, int K);
hipError_t gemm_bf16x3_big(hipStream_t s, bool tA, bool tB, int M, int N, int K, float alpha, const float* A,
                           long lda, const float* B, long ldb, float beta, float* C, long ldc, void* scratch);
hipError_t splitk_reduce_f64(hipStream_t s, const double* P, int S, int M, int N, double alpha, double beta, double* C,
                             long ldc);
hipError_t splitk_reduce_f32(hipStream_t s, const float* P, int S, int M, int N, float alpha, float beta, float* C,
                             long ldc);
hipError_t axpy_f32(hipStream_t s, float a, const float* x, float* y, long n);
// Two-pass deterministic sum of squares -> *out (device, FP64).
hipError_t sumsq_f64(hipStream_t s, const double* x, long n, double* partial, double* out);
hipError_t sumsq_f32(hipStream_t s, const float* x, long n, double* partial, double* out);
// dot(x, y) in FP64 -> *out (device)
hipError_t dot_f64(hipStream_t s, const double* x, const double* y, long n, double* partial, double* out);
hipError_t dot_f32(hipStream_t s, const float* x, const float* y, long n, double* partial, double* out);
int reduce_partials();   // size of the partial buffer the reductions need

// y = x / sqrt(*nrm2)   (nrm2 = sum of squares, device scalar)
hipError_t scale_by_rsqrt_f64(hipStream_t s, const double* x, double* y, const double* nrm2, long n);
hipError_t scale_by_rsqrt_f32(hipStream_t s, const float* x, float* y, const double* nrm2, long n);
// adjoint of y = x / |x|: xbar += (ybar - y * <y, ybar>) / |x|
hipError_t normalize_adjoint_f64(hipStream_t s, const double* y, const double* ybar, const double* nrm2,
                                 const double* ydot, double* xbar, long n);
hipError_t normalize_adjoint_f32(hipStream_t s, const float* y, const float* ybar, const double* nrm2,
                                 const double* ydot, float* xbar, long n);

// ---------------- SVD (one-sided block Jacobi, FP64) ----------------
// Computes M = U diag(S) V^T for `batch` square n x n matrices (row-major,
// consecutive at stride n*n).  U, V: n x n row-major, S: n, descending.
// Columns of U whose singular value is zero are left zero.
// work must hold svd_work_bytes(n, batch) bytes.
size_t svd_work_bytes(int n, int batch);
// The same decomposition with QR preconditioning (columns sorted by norm,
// A P = Q R, Jacobi SVD of R^T); falls back to svd_f64 for n > 4096.
size_t svd_precond_work_bytes(int n, int batch);
// qs, ev (optional: a second stream and three events): the Q factors of the
// two preconditioning QRs are formed on qs while s goes on with the second QR
// and the Jacobi sweeps; s waits for them before the final products.
hipError_t svd_precond_f64(hipStream_t s, int n, int batch, const double* A, double* U, double* S, double* V,
                           void* work, int max_sweeps, double tol, int* host_flags, int* sweeps_out,
                           hipStream_t qs = nullptr, hipEvent_t* ev = nullptr);
// Householder QR of batch tall matrices X (m x k, m >= k, m <= 8192) given as
// Xt = X^T (k x m row-major, overwritten).  R: k x k upper triangular
// (row-major), Qt = Q^T (k x m); either may be null.
size_t qr_work_bytes(int m, int k, int batch);
hipError_t qr_f64(hipStream_t s, int m, int k, int batch, double* Xt, double* R, double* Qt, void* work);
// the two halves of qr_f64: the factorisation (R, and the reflectors and
// block T factors kept in `work`), then Q from them (possibly on another
// stream, ordered after the factorisation; `work` must stay untouched until
// it has run)
hipError_t qr_f64_factor(hipStream_t s, int m, int k, int batch, double* Xt, double* R, void* work);
hipError_t qr_f64_form_q(hipStream_t s, int m, int k, int batch, double* Qt, void* work);
// host_flags: host buffer of >= batch ints (convergence flags are read back
// once per sweep; the stream is synchronised at that point).
// V0 (optional, batch of n x n): start the iteration from G = M V0, V = V0
// (an orthogonal matrix close to the answer, e.g. the previous sweep's V).
// lower_tri: M is lower triangular; V is then solved for from M V = G after
// the sweeps instead of accumulated (checked for orthogonality; the batch is
// decomposed again with accumulated rotations where the check fails).
hipError_t svd_f64(hipStream_t s, int n, int batch, const double* M, double* U, double* S, double* V,
                   void* work, int max_sweeps, double tol, int* host_flags, int* sweeps_out,
                   const double* V0 = nullptr, bool lower_tri = false);

// ---------------- projector formation ----------------
// k = min(chi, #{S > cutoff * S[0]}) per batch entry -> kout (device int)
// X[b, c] = U[b, c] / sqrt(S[c]) for c < k, else 0 (b < nb rows, c < chi cols; U is nb x n)
hipError_t trunc_scale(hipStream_t s, int nb, int n, int chi, const double* U, const double* S,
                       double cutoff, double* X, int* kout, int batch);
// Sign fix: for each column c of PT (na x chi), flip PT[:,c] and PB[:,c] so that
// the entry of largest magnitude (lowest row on ties) of PT[:,c] is positive.
hipError_t sign_fix(hipStream_t s, int na, int chi, double* PT, double* PB, double* sgn_out, int batch);

// max over nc corners of |S_k - prev_k|_2 -> *out (1e300 if !have); prev = S
hipError_t spectra_delta(hipStream_t s, int nc, int ch, const double* S, double* prev, double* out, int have);

// ---------------- energy ----------------
// e = sum rho[P,Q,P',Q'] h[(P',Q'),(P,Q)] / sum rho[P,Q,P,Q];  rho FP64 [p,p,p,p]
hipError_t bond_energy(hipStream_t s, int p, const double* rho, const double* h, double* e_out);
hipError_t site_energy(hipStream_t s, int nb, const double* eb, double w, double* out);

}  // namespace sctm
