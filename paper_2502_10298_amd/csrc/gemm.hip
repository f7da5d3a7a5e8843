// Batched GEMM on the CDNA4 matrix cores (gfx950).
//
// Every contraction of the split-CTMRG networks is reshaped into a GEMM
// C = alpha op(A) op(B) + beta C on row-major operands.  The kernels tile C in
// 64 x 64 blocks per workgroup of four 64-wide wavefronts (2 x 2 waves, each
// owning a 32 x 32 quadrant = 2 x 2 MFMA 16 x 16 tiles) and stage the A and B
// panels through LDS, k-major, so that the MFMA operand fetches of a wave read
// 16 consecutive LDS words per k row.
//
//   F64     v_mfma_f64_16x16x4_f64     (FP64 parity path)
//   F32     v_mfma_f32_16x16x4_f32
//   BF16X3  v_mfma_f32_16x16x32_bf16 on split operands a = a_hi + a_lo
//           (bf16 each), accumulating a_hi b_hi + a_hi b_lo + a_lo b_hi in FP32
//           (the product a_lo b_lo, of relative size 2^-16, is dropped).
//
// MFMA lane layouts used (16x16xK, 64 lanes):
//   A operand: lane l holds A[l % 16][kblk(l / 16)]
//   B operand: lane l holds B[kblk(l / 16)][l % 16]
//   D (4 per lane): D[4 (l / 16) + r][l % 16], r = 0..3 for f32 and bf16,
//                   D[4 r + l / 16][l % 16] for f64 (measured on gfx950)
// with kblk = one k (x4 f32/f64) or eight consecutive k (x32 bf16); A and B
// use the same k slot order, so only the output layout matters.
#include "kernels.hpp"

#include <algorithm>

namespace sctm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

static constexpr int BM = 64, BN = 64;

template <typename T, typename V4>
__device__ inline V4 mfma_step(T a, T b, V4 c);

template <>
__device__ inline d4 mfma_step<double, d4>(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <>
__device__ inline f4 mfma_step<float, f4>(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// FP64 / FP32: BK = 32 (eight MFMA k-steps of 4).  The next k tile is loaded
// into registers while the MFMAs run on the current one in LDS.
// ---------------------------------------------------------------------------
template <typename T, bool TA>
__device__ inline void load_a(const T* __restrict__ A, long lda, int M, int K, int bm, int k0, int tid, T (&r)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if (!TA) {
      const int row = (tid >> 5) + 8 * i, c = tid & 31, m = bm + row, k = k0 + c;
      r[i] = (m < M && k < K) ? A[(long)m * lda + k] : T(0);
    } else {
      const int row = (tid >> 6) + 4 * i, c = tid & 63, k = k0 + row, m = bm + c;
      r[i] = (m < M && k < K) ? A[(long)k * lda + m] : T(0);
    }
  }
}

template <typename T, bool TB>
__device__ inline void load_b(const T* __restrict__ B, long ldb, int N, int K, int bn, int k0, int tid, T (&r)[8]) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    if (!TB) {
      const int row = (tid >> 6) + 4 * i, c = tid & 63, k = k0 + row, n = bn + c;
      r[i] = (n < N && k < K) ? B[(long)k * ldb + n] : T(0);
    } else {
      const int row = (tid >> 5) + 8 * i, c = tid & 31, n = bn + row, k = k0 + c;
      r[i] = (n < N && k < K) ? B[(long)n * ldb + k] : T(0);
    }
  }
}

template <typename T, typename V4, bool TA, bool TB, bool BETA>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, T alpha,
                                                   const T* __restrict__ A, long lda, long sA,
                                                   const T* __restrict__ B, long ldb, long sB, T beta,
                                                   T* __restrict__ C, long ldc, long sC, int zdiv, long sA2,
                                                   long sB2, long sC2, int Ktot) {
  constexpr int BK = 32;
  __shared__ T As[BK][BM + 4];
  __shared__ T Bs[BK][BN + 4];
  // grid z = batch entry x K slice (zdiv slices of length K, the last one
  // ending at Ktot; zdiv = 1: plain batched product)
  const long bz = blockIdx.z / zdiv, sl = blockIdx.z % zdiv;
  A += bz * sA + sl * sA2;
  B += bz * sB + sl * sB2;
  C += bz * sC + sl * sC2;
  if (zdiv > 1) K = min(K, Ktot - (int)sl * K);
  const int bm = blockIdx.y * BM, bn = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  V4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = V4{0, 0, 0, 0};

  // BETA (beta != 0): the sixteen C entries of the thread are loaded first
  // (clamped addresses, no branches), so that their latency overlaps the
  // operand loads and the MFMAs instead of following the last k tile.
  T cold[2][2][4];
  if (BETA) {
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = sizeof(T) == 8 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
          const int m = min(bm + wm * 32 + ti * 16 + row, M - 1), n = min(bn + wn * 32 + tj * 16 + (lane & 15), N - 1);
          cold[ti][tj][r] = C[(long)m * ldc + n];
        }
  }
  T ra[8], rb[8];
  load_a<T, TA>(A, lda, M, K, bm, 0, tid, ra);
  load_b<T, TB>(B, ldb, N, K, bn, 0, tid, rb);
  for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (!TA) As[tid & 31][(tid >> 5) + 8 * i] = ra[i];
      else As[(tid >> 6) + 4 * i][tid & 63] = ra[i];
      if (!TB) Bs[(tid >> 6) + 4 * i][tid & 63] = rb[i];
      else Bs[tid & 31][(tid >> 5) + 8 * i] = rb[i];
    }
    __syncthreads();
    if (k0 + BK < K) {   // next tile in flight during the MFMAs
      load_a<T, TA>(A, lda, M, K, bm, k0 + BK, tid, ra);
      load_b<T, TB>(B, ldb, N, K, bn, k0 + BK, tid, rb);
    }
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      T a0 = As[kr][wm * 32 + (lane & 15)];
      T a1 = As[kr][wm * 32 + 16 + (lane & 15)];
      T b0 = Bs[kr][wn * 32 + (lane & 15)];
      T b1 = Bs[kr][wn * 32 + 16 + (lane & 15)];
      acc[0][0] = mfma_step<T, V4>(a0, b0, acc[0][0]);
      acc[0][1] = mfma_step<T, V4>(a0, b1, acc[0][1]);
      acc[1][0] = mfma_step<T, V4>(a1, b0, acc[1][0]);
      acc[1][1] = mfma_step<T, V4>(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  // f64 16x16x4: D[4 r + l / 16][l % 16]; f32 16x16x4: D[4 (l / 16) + r][l % 16].
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = sizeof(T) == 8 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        int m = bm + wm * 32 + ti * 16 + row;
        int n = bn + wn * 32 + tj * 16 + (lane & 15);
        if (m < M && n < N) {
          T v = alpha * acc[ti][tj][r];
          long o = (long)m * ldc + n;
          C[o] = BETA ? v + beta * cold[ti][tj][r] : v;
        }
      }
}

// ---------------------------------------------------------------------------
// Split BF16 products: FP32 operands split into NS bf16 terms in the LDS
// staging (x = hi + lo, or hi + mid + lo), BK = 32, and the cross products
// of total order below NS on the BF16 matrix cores with FP32 accumulation,
// smallest first: NS = 2 (BF16x3) lo*hi + hi*lo + hi*hi; NS = 3 (BF16x6)
// adds mid*mid and the hi*mid, mid*hi, hi*lo, lo*hi terms of the three-way
// split, which leaves a residual near the FP32 rounding of the operands.
// ---------------------------------------------------------------------------
template <int NS>
__device__ inline void split_bf16(float x, __bf16 (&out)[NS]) {
  float r = x;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    out[q] = (__bf16)r;            // round to nearest even
    r = r - (float)out[q];
  }
}

template <bool TA, bool TB, int NS>
__global__ __launch_bounds__(256) void gemm_bf16s_kernel(int M, int N, int K, float alpha,
                                                         const float* __restrict__ A, long lda, long sA,
                                                         const float* __restrict__ B, long ldb, long sB,
                                                         float beta, float* __restrict__ C, long ldc, long sC) {
  constexpr int BK = 32;
  // m-major rows of 32 k (bf16) for A, n-major rows of 32 k for B: one lane
  // fetches 8 consecutive k of one row as a 16-byte vector.  Term q of the
  // split of A lives in As[q], of B in Bs[q].
  __shared__ __attribute__((aligned(16))) __bf16 As[NS][BM][BK + 8];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[NS][BN][BK + 8];
  const long bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  const int bm = blockIdx.y * BM, bn = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0, 0, 0, 0};

  // the next k tile is loaded into registers while the MFMAs run on the
  // current one in LDS
  float ra[8], rb[8];
  load_a<float, TA>(A, lda, M, K, bm, 0, tid, ra);
  load_b<float, TB>(B, ldb, N, K, bn, 0, tid, rb);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __bf16 sp[NS];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      // A: m-major rows of k;  B: n-major rows of k (same element mapping as the loads)
      split_bf16<NS>(ra[i], sp);
      if (!TA) {
#pragma unroll
        for (int q = 0; q < NS; ++q) As[q][(tid >> 5) + 8 * i][tid & 31] = sp[q];
      } else {
#pragma unroll
        for (int q = 0; q < NS; ++q) As[q][tid & 63][(tid >> 6) + 4 * i] = sp[q];
      }
      split_bf16<NS>(rb[i], sp);
      if (!TB) {
#pragma unroll
        for (int q = 0; q < NS; ++q) Bs[q][tid & 63][(tid >> 6) + 4 * i] = sp[q];
      } else {
#pragma unroll
        for (int q = 0; q < NS; ++q) Bs[q][(tid >> 5) + 8 * i][tid & 31] = sp[q];
      }
    }
    __syncthreads();
    if (k0 + BK < K) {
      load_a<float, TA>(A, lda, M, K, bm, k0 + BK, tid, ra);
      load_b<float, TB>(B, ldb, N, K, bn, k0 + BK, tid, rb);
    }
    const int kq = 8 * (lane >> 4);
    bf8 a[NS][2], bb[NS][2];
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[q][t] = *reinterpret_cast<const bf8*>(&As[q][wm * 32 + t * 16 + (lane & 15)][kq]);
        bb[q][t] = *reinterpret_cast<const bf8*>(&Bs[q][wn * 32 + t * 16 + (lane & 15)][kq]);
      }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        // terms of total order o = qa + qb < NS, highest order (smallest) first
#pragma unroll
        for (int o = NS - 1; o >= 0; --o)
#pragma unroll
          for (int qa = o; qa >= 0; --qa)
            acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[qa][ti], bb[o - qa][tj], acc[ti][tj], 0, 0, 0);
      }
    __syncthreads();
  }
  float cold[2][2][4];   // C entries loaded before any is combined (beta != 0)
  if (beta != 0.f) {
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = min(bm + wm * 32 + ti * 16 + 4 * (lane >> 4) + r, M - 1);
          const int n = min(bn + wn * 32 + tj * 16 + (lane & 15), N - 1);
          cold[ti][tj][r] = C[(long)m * ldc + n];
        }
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int m = bm + wm * 32 + ti * 16 + 4 * (lane >> 4) + r;
        int n = bn + wn * 32 + tj * 16 + (lane & 15);
        if (m < M && n < N) {
          float v = alpha * acc[ti][tj][r];
          long o = (long)m * ldc + n;
          C[o] = (beta == 0.f) ? v : v + beta * cold[ti][tj][r];
        }
      }
}

// Split BF16 products with K <= 128 on a small grid (the short contractions
// and the K slices of split-K products): the whole k extent of both operand
// tiles is loaded at once (one memory round trip instead of one per 32-wide k tile), split into
// LDS, and the MFMAs run after a single barrier.  Same lane layouts, term
// order and FP32 accumulation order as gemm_bf16s_kernel.
static constexpr int SKM = 128;   // largest K of the short-product kernel

template <bool TA, bool TB, int NS>
__global__ __launch_bounds__(256) void gemm_bf16s_shortk_kernel(int M, int N, int K, float alpha,
                                                                const float* __restrict__ A, long lda, long sA,
                                                                const float* __restrict__ B, long ldb, long sB,
                                                                float beta, float* __restrict__ C, long ldc, long sC) {
  constexpr int BK = 32, NKT = SKM / BK;
  __shared__ __attribute__((aligned(16))) __bf16 As[NS][BM][SKM + 8];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[NS][BN][SKM + 8];
  const long bz = blockIdx.z;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  const int bm = blockIdx.y * BM, bn = blockIdx.x * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int nkt = (K + BK - 1) / BK;   // <= NKT
  float ra[NKT][8], rb[NKT][8];
#pragma unroll
  for (int kt = 0; kt < NKT; ++kt) {
    if (kt < nkt) {
      load_a<float, TA>(A, lda, M, K, bm, kt * BK, tid, ra[kt]);
      load_b<float, TB>(B, ldb, N, K, bn, kt * BK, tid, rb[kt]);
    }
  }
  float cold[2][2][4];
  if (beta != 0.f) {
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = min(bm + wm * 32 + ti * 16 + 4 * (lane >> 4) + r, M - 1);
          const int n = min(bn + wn * 32 + tj * 16 + (lane & 15), N - 1);
          cold[ti][tj][r] = C[(long)m * ldc + n];
        }
  }
#pragma unroll
  for (int kt = 0; kt < NKT; ++kt) {
    if (kt >= nkt) break;
    __bf16 sp[NS];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      split_bf16<NS>(ra[kt][i], sp);
      if (!TA) {
#pragma unroll
        for (int q = 0; q < NS; ++q) As[q][(tid >> 5) + 8 * i][kt * BK + (tid & 31)] = sp[q];
      } else {
#pragma unroll
        for (int q = 0; q < NS; ++q) As[q][tid & 63][kt * BK + (tid >> 6) + 4 * i] = sp[q];
      }
      split_bf16<NS>(rb[kt][i], sp);
      if (!TB) {
#pragma unroll
        for (int q = 0; q < NS; ++q) Bs[q][tid & 63][kt * BK + (tid >> 6) + 4 * i] = sp[q];
      } else {
#pragma unroll
        for (int q = 0; q < NS; ++q) Bs[q][(tid >> 5) + 8 * i][kt * BK + (tid & 31)] = sp[q];
      }
    }
  }
  __syncthreads();
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0, 0, 0, 0};
#pragma unroll
  for (int kt = 0; kt < NKT; ++kt) {
    if (kt >= nkt) break;
    const int kq = kt * BK + 8 * (lane >> 4);
    bf8 a[NS][2], bb[NS][2];
#pragma unroll
    for (int q = 0; q < NS; ++q)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[q][t] = *reinterpret_cast<const bf8*>(&As[q][wm * 32 + t * 16 + (lane & 15)][kq]);
        bb[q][t] = *reinterpret_cast<const bf8*>(&Bs[q][wn * 32 + t * 16 + (lane & 15)][kq]);
      }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
#pragma unroll
        for (int o = NS - 1; o >= 0; --o)
#pragma unroll
          for (int qa = o; qa >= 0; --qa)
            acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[qa][ti], bb[o - qa][tj], acc[ti][tj], 0, 0, 0);
      }
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int m = bm + wm * 32 + ti * 16 + 4 * (lane >> 4) + r;
        int n = bn + wn * 32 + tj * 16 + (lane & 15);
        if (m < M && n < N) {
          float v = alpha * acc[ti][tj][r];
          long o = (long)m * ldc + n;
          C[o] = (beta == 0.f) ? v : v + beta * cold[ti][tj][r];
        }
      }
}

static dim3 gemm_grid(int M, int N, int batch) {
  return dim3((N + BN - 1) / BN, (M + BM - 1) / BM, batch);
}

template <typename T, typename V4, bool TA, bool TB>
static void launch_gemm(int kind, double fl, double by, dim3 g, hipStream_t s, int M, int N, int K, T alpha,
                        const T* A, long lda, long sA, const T* B, long ldb, long sB, T beta, T* C, long ldc, long sC,
                        int zdiv, long sA2, long sB2, long sC2, int Ktot) {
  if (beta != T(0))
    launch_timed(kind, fl, by, gemm_kernel<T, V4, TA, TB, true>, g, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B,
                 ldb, sB, beta, C, ldc, sC, zdiv, sA2, sB2, sC2, Ktot);
  else
    launch_timed(kind, fl, by, gemm_kernel<T, V4, TA, TB, false>, g, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B,
                 ldb, sB, beta, C, ldc, sC, zdiv, sA2, sB2, sC2, Ktot);
}

KernelTimer*& kernel_timer() {
  static thread_local KernelTimer* t = nullptr;
  return t;
}

hipError_t gemm_f64(hipStream_t s, bool tA, bool tB, int M, int N, int K, double alpha,
                    const double* A, long lda, long sA, const double* B, long ldb, long sB,
                    double beta, double* C, long ldc, long sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  dim3 g = gemm_grid(M, N, batch);
  const int kind = KC_GEMM_F64;
  const double fl = 2.0 * M * N * (double)K * batch;
  const double by = 8.0 * batch * ((double)M * K + (double)K * N + (double)M * N * (beta != 0.0 ? 2 : 1));
  if (!tA && !tB)
    launch_gemm<double, d4, false, false>(kind, fl, by, g, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 1, 0L, 0L, 0L, K);
  else if (tA && !tB)
    launch_gemm<double, d4, true, false>(kind, fl, by, g, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 1, 0L, 0L, 0L, K);
  else if (!tA && tB)
    launch_gemm<double, d4, false, true>(kind, fl, by, g, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 1, 0L, 0L, 0L, K);
  else
    launch_gemm<double, d4, true, true>(kind, fl, by, g, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 1, 0L, 0L, 0L, K);
  return hipGetLastError();
}

hipError_t gemm_f64_slices(hipStream_t s, bool tA, bool tB, int M, int N, int K, const double* A, long lda, long sA,
                           const double* B, long ldb, long sB, double* P, int S, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0 || S < 1) return hipSuccess;
  const int Ks = (K + S - 1) / S;
  if ((long)(S - 1) * Ks >= K) return hipErrorInvalidValue;   // every slice non-empty
  dim3 g = gemm_grid(M, N, batch * S);
  const int kind = KC_GEMM_F64;
  const double fl = 2.0 * M * N * (double)K * batch;
  const double by = 8.0 * batch * ((double)M * K + (double)K * N + (double)M * N * S);
  const long sA2 = tA ? (long)Ks * lda : Ks, sB2 = tB ? (long)Ks : (long)Ks * ldb;
  const long sP = (long)S * M * N, sP2 = (long)M * N;
  if (!tA && !tB)
    launch_gemm<double, d4, false, false>(kind, fl, by, g, s, M, N, Ks, 1.0, A, lda, sA, B,
                 ldb, sB, 0.0, P, (long)N, sP, S, sA2, sB2, sP2, K);
  else if (tA && !tB)
    launch_gemm<double, d4, true, false>(kind, fl, by, g, s, M, N, Ks, 1.0, A, lda, sA, B,
                 ldb, sB, 0.0, P, (long)N, sP, S, sA2, sB2, sP2, K);
  else if (!tA && tB)
    launch_gemm<double, d4, false, true>(kind, fl, by, g, s, M, N, Ks, 1.0, A, lda, sA, B,
                 ldb, sB, 0.0, P, (long)N, sP, S, sA2, sB2, sP2, K);
  else
    launch_gemm<double, d4, true, true>(kind, fl, by, g, s, M, N, Ks, 1.0, A, lda, sA, B,
                 ldb, sB, 0.0, P, (long)N, sP, S, sA2, sB2, sP2, K);
  return hipGetLastError();
}

hipError_t gemm_f32(hipStream_t s, Prec mode, bool tA, bool tB, int M, int N, int K, float alpha,
                    const float* A, long lda, long sA, const float* B, long ldb, long sB, float beta,
                    float* C, long ldc, long sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  dim3 g = gemm_grid(M, N, batch);
  const int kind = mode == Prec::BF16X3 ? KC_GEMM_BF16X3 : (mode == Prec::BF16X6 ? KC_GEMM_BF16X6 : KC_GEMM_F32);
  const double fl = 2.0 * M * N * (double)K * batch;
  const double by = 4.0 * batch * ((double)M * K + (double)K * N + (double)M * N * (beta != 0.f ? 2 : 1));
  if (mode == Prec::BF16X3 || mode == Prec::BF16X6) {
    const bool six = mode == Prec::BF16X6;
    // short products on a small grid: one memory round trip per workgroup;
    // on a large grid the pipelined kernel (less LDS, more workgroups per
    // compute unit) is faster
    const bool shortk = K <= SKM && (long)g.x * g.y * g.z <= 512;
#define SPLIT_LAUNCH(TA_, TB_)                                                                                      \
  if (shortk) {                                                                                                      \
    if (six)                                                                                                         \
      launch_timed(kind, fl, by, gemm_bf16s_shortk_kernel<TA_, TB_, 3>, g, dim3(256), 0, s, M, N, K, alpha, A, lda,  \
                   sA, B, ldb, sB, beta, C, ldc, sC);                                                                \
    else                                                                                                             \
      launch_timed(kind, fl, by, gemm_bf16s_shortk_kernel<TA_, TB_, 2>, g, dim3(256), 0, s, M, N, K, alpha, A, lda,  \
                   sA, B, ldb, sB, beta, C, ldc, sC);                                                                \
  } else if (six)                                                                                                    \
    launch_timed(kind, fl, by, gemm_bf16s_kernel<TA_, TB_, 3>, g, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, \
                 sB, beta, C, ldc, sC);                                                                              \
  else                                                                                                               \
    launch_timed(kind, fl, by, gemm_bf16s_kernel<TA_, TB_, 2>, g, dim3(256), 0, s, M, N, K, alpha, A, lda, sA, B, ldb, \
                 sB, beta, C, ldc, sC);
    if (!tA && !tB) {
      SPLIT_LAUNCH(false, false)
    } else if (tA && !tB) {
      SPLIT_LAUNCH(true, false)
    } else if (!tA && tB) {
      SPLIT_LAUNCH(false, true)
    } else {
      SPLIT_LAUNCH(true, true)
    }
#undef SPLIT_LAUNCH
    return hipGetLastError();
  }
  if (!tA && !tB)
    launch_gemm<float, f4, false, false>(kind, fl, by, g, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 1, 0L, 0L, 0L, K);
  else if (tA && !tB)
    launch_gemm<float, f4, true, false>(kind, fl, by, g, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 1, 0L, 0L, 0L, K);
  else if (!tA && tB)
    launch_gemm<float, f4, false, true>(kind, fl, by, g, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 1, 0L, 0L, 0L, K);
  else
    launch_gemm<float, f4, true, true>(kind, fl, by, g, s, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 1, 0L, 0L, 0L, K);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Split-K: a product whose 64 x 64 output tiles are too few to fill the chip
// and whose K is long (>= 512) runs as a strided batch of K slices into a scratch
// buffer; one more pass adds the slices in order and applies alpha and beta.
static int splitk_slices(int M, int N, int K) {
  const long tiles = (long)((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (M <= 0 || N <= 0 || tiles >= 128 || K < 512) return 0;
  int S = (int)std::min<long>(std::min<long>(512 / tiles, K / 128), 64);
  while (S > 1 && (long)S * M * N > (16L << 20)) S /= 2;
  return S >= 2 ? S : 0;
}

long splitk_scratch_elems(int M, int N, int K) {
  const int S = splitk_slices(M, N, K);
  return S ? (long)S * M * N : 0;
}

template <typename T, typename Launch, typename Reduce>
static hipError_t splitk_run(bool tA, bool tB, int M, int N, int K, long lda, long ldb, Launch launch,
                             Reduce reduce) {
  const int S = splitk_slices(M, N, K);
  const int Ks = (K + S - 1) / S;
  const int full = K / Ks;            // slices of length Ks
  const int rest = K - full * Ks;     // one shorter slice (may be 0)
  const long aStep = tA ? (long)Ks * lda : Ks, bStep = tB ? (long)Ks : (long)Ks * ldb;
  const long mn = (long)M * N;
  hipError_t e = launch(Ks, 0L, 0L, 0L, aStep, bStep, mn, full);
  if (e == hipSuccess && rest > 0) e = launch(rest, full * aStep, full * bStep, full * mn, 0L, 0L, 0L, 1);
  if (e == hipSuccess) e = reduce(full + (rest > 0 ? 1 : 0));
  return e;
}

hipError_t gemm_f64_splitk(hipStream_t s, bool tA, bool tB, int M, int N, int K, double alpha, const double* A,
                           long lda, const double* B, long ldb, double beta, double* C, long ldc, double* scratch) {
  if (!splitk_slices(M, N, K))
    return gemm_f64(s, tA, tB, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1);
  return splitk_run<double>(
      tA, tB, M, N, K, lda, ldb,
      [&](int k, long oA, long oB, long oP, long sA, long sB, long sP, int nb) {
        return gemm_f64(s, tA, tB, M, N, k, 1.0, A + oA, lda, sA, B + oB, ldb, sB, 0.0, scratch + oP, N, sP, nb);
      },
      [&](int nsl) { return splitk_reduce_f64(s, scratch, nsl, M, N, alpha, beta, C, ldc); });
}

hipError_t gemm_f32_splitk(hipStream_t s, Prec mode, bool tA, bool tB, int M, int N, int K, float alpha,
                           const float* A, long lda, const float* B, long ldb, float beta, float* C, long ldc,
                           float* scratch) {
  if (!splitk_slices(M, N, K))
    return gemm_f32(s, mode, tA, tB, M, N, K, alpha, A, lda, 0, B, ldb, 0, beta, C, ldc, 0, 1);
  return splitk_run<float>(
      tA, tB, M, N, K, lda, ldb,
      [&](int k, long oA, long oB, long oP, long sA, long sB, long sP, int nb) {
        return gemm_f32(s, mode, tA, tB, M, N, k, 1.f, A + oA, lda, sA, B + oB, ldb, sB, 0.f, scratch + oP, N, sP,
                        nb);
      },
      [&](int nsl) { return splitk_reduce_f32(s, scratch, nsl, M, N, alpha, beta, C, ldc); });
}

// ---------------------------------------------------------------------------
// Large BF16X3 products.  The operands are split once into bf16 hi / lo
// planes stored k-contiguous (A' = op(A) as M x K, B' = op(B)^T as N x K,
// zero-padded to 128 rows and 64 k), and one bf16 GEMM runs over the
// concatenation
//   C = [A_hi | A_hi | A_lo] [B_hi | B_lo | B_hi]^T,
// i.e. the same three products as the in-LDS split.  128 x 128 output tiles
// per workgroup (2 x 2 waves of 64 x 64 = 4 x 4 MFMA 16x16x32 tiles), BK =
// 64, both operand tiles k-contiguous in LDS so that every MFMA operand is
// one 16-byte read, LDS double-buffered (one barrier per k step) with the
// next step's 16-byte global loads in flight during the MFMAs.  When the
// output has too few tiles to fill the chip, the concatenated K runs in
// slices into partial products that one more pass adds in order.
// ---------------------------------------------------------------------------
static constexpr int XBM = 128, XBK = 64, XPAD = 8;
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// H, L [Rp][Kp] = hi / lo split of X (rows R, k extent K); TRANS: X stored
// K x R (element (r, k) at X[k ld + r]), else R x K.  Grid (Kp / 64, Rp / 64):
// a 64 x 64 tile is read along X's contiguous dimension into LDS, then every
// thread splits eight consecutive k of one row and writes them as one
// 16-byte vector per plane.
template <bool TRANS>
__device__ __forceinline__ void bf16_split_tile(const float* __restrict__ X, long ld, int R, int K, int Kp,
                                                __bf16* __restrict__ H, __bf16* __restrict__ L, int r0, int k0,
                                                float (&tile)[64][65]) {
  const int t = threadIdx.x;
  // all sixteen loads in flight before the first LDS write; out-of-range
  // entries read an in-range one (clamped, no branch) and count as zero
  float v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int a = (t >> 6) + 4 * i, c = t & 63;   // a: slow index, c: along X's contiguous dimension
    const int r = TRANS ? r0 + c : r0 + a, k = TRANS ? k0 + a : k0 + c;
    const long rc = min(r, R - 1), kc = min(k, K - 1);
    const float x = TRANS ? X[kc * ld + rc] : X[rc * ld + kc];
    v[i] = (r < R && k < K) ? x : 0.f;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int a = (t >> 6) + 4 * i, c = t & 63;
    if (TRANS)
      tile[c][a] = v[i];
    else
      tile[a][c] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int q = t + 256 * j, rr = q >> 3, kc = (q & 7) * 8;
    bf8 hi, lo;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      __bf16 sp[2];
      split_bf16<2>(tile[rr][kc + e], sp);
      hi[e] = sp[0];
      lo[e] = sp[1];
    }
    const long o = (long)(r0 + rr) * Kp + k0 + kc;
    *reinterpret_cast<bf8*>(H + o) = hi;
    *reinterpret_cast<bf8*>(L + o) = lo;
  }
}

// Both operands of a product in one launch: grid (Kp / 64, RpA / 64 + RpB / 64),
// the first RpA / 64 rows of workgroups split A, the rest B.
template <bool TRANSA, bool TRANSB>
__global__ __launch_bounds__(256) void bf16_split2_kernel(const float* __restrict__ A, long lda, int RA, int RpA,
                                                          const float* __restrict__ B, long ldb, int RB, int K, int Kp,
                                                          __bf16* __restrict__ AH, __bf16* __restrict__ AL,
                                                          __bf16* __restrict__ BH, __bf16* __restrict__ BL) {
  __shared__ float tile[64][65];   // [r][k]
  const int by = blockIdx.y, k0 = blockIdx.x * 64;
  if (by * 64 < RpA)
    bf16_split_tile<TRANSA>(A, lda, RA, K, Kp, AH, AL, by * 64, k0, tile);
  else
    bf16_split_tile<TRANSB>(B, ldb, RB, K, Kp, BH, BL, by * 64 - RpA, k0, tile);
}

// Slice z of the concatenated K' = 3 Kp covers [z ksl, min(3 Kp, (z+1) ksl));
// P == nullptr: C = alpha acc + beta C, else P[z] = acc (M x N).
__global__ __launch_bounds__(256) void gemm_bf16nt_kernel(int M, int N, int Kp, int ksl, float alpha,
                                                          const __bf16* __restrict__ Ah,
                                                          const __bf16* __restrict__ Al,
                                                          const __bf16* __restrict__ Bh,
                                                          const __bf16* __restrict__ Bl, float beta,
                                                          float* __restrict__ C, long ldc, float* __restrict__ P) {
  __shared__ __attribute__((aligned(16))) __bf16 As[2][XBM][XBK + XPAD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][XBM][XBK + XPAD];
  const int bm = blockIdx.y * XBM, bn = blockIdx.x * XBM, z = blockIdx.z;
  const int k_lo = z * ksl, k_hi = min(3 * Kp, k_lo + ksl);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, wm = wave >> 1, wn = wave & 1;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0, 0, 0, 0};
  // loader: 16-byte chunk c = tid + 256 i of a 128 x 64 tile: row c / 8, k 8 (c % 8)
  u4v ra[4], rb[4];
  auto load = [&](int kp) {
    const int g = kp / Kp, k = kp - g * Kp;
    const __bf16* A = (g == 2) ? Al : Ah;
    const __bf16* B = (g == 1) ? Bl : Bh;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = tid + 256 * i, row = c >> 3, kc = (c & 7) * 8;
      ra[i] = *reinterpret_cast<const u4v*>(A + (long)(bm + row) * Kp + k + kc);
      rb[i] = *reinterpret_cast<const u4v*>(B + (long)(bn + row) * Kp + k + kc);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = tid + 256 * i, row = c >> 3, kc = (c & 7) * 8;
      *reinterpret_cast<u4v*>(&As[buf][row][kc]) = ra[i];
      *reinterpret_cast<u4v*>(&Bs[buf][row][kc]) = rb[i];
    }
  };
  load(k_lo);
  store(0);
  __syncthreads();
  int buf = 0;
  for (int kp = k_lo; kp < k_hi; kp += XBK) {
    const bool more = kp + XBK < k_hi;
    if (more) load(kp + XBK);
#pragma unroll
    for (int ks = 0; ks < XBK / 32; ++ks) {
      const int kq = ks * 32 + 8 * (lane >> 4);
      bf8 a[4], b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = *reinterpret_cast<const bf8*>(&As[buf][wm * 64 + t * 16 + (lane & 15)][kq]);
        b[t] = *reinterpret_cast<const bf8*>(&Bs[buf][wn * 64 + t * 16 + (lane & 15)][kq]);
      }
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int ti = 0; ti < 4; ++ti) {
    // with beta != 0 the sixteen C entries of a row tile are loaded (clamped
    // addresses) before any is combined, so their latencies overlap
    float cold[4][4];
    if (!P && beta != 0.f) {
#pragma unroll
      for (int tj = 0; tj < 4; ++tj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = min(bm + wm * 64 + ti * 16 + 4 * (lane >> 4) + r, M - 1);
          const int n = min(bn + wn * 64 + tj * 16 + (lane & 15), N - 1);
          cold[tj][r] = C[(long)m * ldc + n];
        }
    }
#pragma unroll
    for (int tj = 0; tj < 4; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = bm + wm * 64 + ti * 16 + 4 * (lane >> 4) + r;
        const int n = bn + wn * 64 + tj * 16 + (lane & 15);
        if (m < M && n < N) {
          if (P) {
            P[(long)z * M * N + (long)m * N + n] = acc[ti][tj][r];
          } else {
            const float v = alpha * acc[ti][tj][r];
            const long o = (long)m * ldc + n;
            C[o] = (beta == 0.f) ? v : v + beta * cold[tj][r];
          }
        }
      }
  }
}

struct Bf16BigPlan {
  int Mp = 0, Np = 0, Kp = 0, S = 0, ksl = 0;
  size_t offAh = 0, offAl = 0, offBh = 0, offBl = 0, offP = 0, total = 0;
};

// The pre-split path pays for itself (measured on gfx950: 1.36x at 1024 x
// 1024 x 2048, 1.9x at 4096^3, slower than the in-LDS split for thin outputs
// such as 8192 x 128 x 1024) from 2^31 multiply-adds with both output
// dimensions >= 1024; slices give the chip about 512 workgroups (two per
// CU, so that one hides the other's load latency), each with at least
// eight k steps, within 64 MiB of partials.
static bool bf16_big_plan(int M, int N, int K, Bf16BigPlan& p) {
  if (M < 1024 || N < 1024 || K < 256 || (double)M * N * (double)K < 2147483648.0) return false;
  p.Mp = (M + XBM - 1) / XBM * XBM;
  p.Np = (N + XBM - 1) / XBM * XBM;
  p.Kp = (K + XBK - 1) / XBK * XBK;
  const long tiles = (long)(p.Mp / XBM) * (p.Np / XBM);
  const int ksteps = 3 * p.Kp / XBK;
  int S = 1;
  if (tiles < 512) S = (int)std::min<long>((512 + tiles - 1) / tiles, ksteps / 8);
  while (S > 1 && (long)S * M * N * 4 > (64L << 20)) --S;
  if (S < 1) S = 1;
  const int per = (ksteps + S - 1) / S;
  p.ksl = per * XBK;
  p.S = (ksteps + per - 1) / per;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t ap = sizeof(__bf16) * (size_t)p.Mp * p.Kp, bp = sizeof(__bf16) * (size_t)p.Np * p.Kp;
  p.offAh = take(ap);
  p.offAl = take(ap);
  p.offBh = take(bp);
  p.offBl = take(bp);
  p.offP = take(p.S > 1 ? sizeof(float) * (size_t)p.S * M * N : 0);
  p.total = off;
  return true;
}

size_t bf16x3_big_scratch_bytes(int M, int N, int K) {
  Bf16BigPlan p;
  return bf16_big_plan(M, N, K, p) ? p.total : 0;
}

hipError_t gemm_bf16x3_big(hipStream_t s, bool tA, bool tB, int M, int N, int K, float alpha, const float* A,
                           long lda, const float* B, long ldb, float beta, float* C, long ldc, void* scratch) {
  Bf16BigPlan p;
  if (!bf16_big_plan(M, N, K, p) || !scratch) return hipErrorInvalidValue;
  char* w = (char*)scratch;
  __bf16 *Ah = (__bf16*)(w + p.offAh), *Al = (__bf16*)(w + p.offAl);
  __bf16 *Bh = (__bf16*)(w + p.offBh), *Bl = (__bf16*)(w + p.offBl);
  float* P = p.S > 1 ? (float*)(w + p.offP) : nullptr;
  const int kind = KC_GEMM_BF16X3;
  // op(A) rows M: stored K x M when tA;  op(B)^T rows N: stored K x N unless tB
  const double byS = 4.0 * (M + N) * (double)K + 4.0 * (p.Mp + p.Np) * (double)p.Kp;
  const dim3 gs(p.Kp / 64, (p.Mp + p.Np) / 64);
#define SPLIT2(TA_, TB_)                                                                                        \
  launch_timed(kind, 0.0, byS, bf16_split2_kernel<TA_, TB_>, gs, dim3(256), 0, s, A, lda, M, p.Mp, B, ldb, N, K, \
               p.Kp, Ah, Al, Bh, Bl)
  if (tA && !tB)
    SPLIT2(true, true);
  else if (tA && tB)
    SPLIT2(true, false);
  else if (!tA && !tB)
    SPLIT2(false, true);
  else
    SPLIT2(false, false);
#undef SPLIT2
  const double fl = 2.0 * M * N * (double)K;
  const double by = 2.0 * 2.0 * ((double)p.Mp + p.Np) * p.Kp + 4.0 * M * N * (beta != 0.f ? 2 : 1);
  launch_timed(kind, fl, by, gemm_bf16nt_kernel, dim3(p.Np / XBM, p.Mp / XBM, p.S), dim3(256), 0, s, M, N, p.Kp,
               p.ksl, alpha, (const __bf16*)Ah, (const __bf16*)Al, (const __bf16*)Bh, (const __bf16*)Bl, beta, C, ldc,
               P);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && P) e = splitk_reduce_f32(s, P, p.S, M, N, alpha, beta, C, ldc);
  return e;
}

}  // namespace sctm
