// FP64 SVD by blocked one-sided (Hestenes) Jacobi, for the projector matrices
// M = U S V^T of the split-CTMRG projector recipe.
//
// The columns of G = M are orthogonalised by orthogonal rotations G <- G W,
// accumulated in V <- V W; at convergence G = U S.  Columns are grouped in
// blocks of 16; a round-robin tournament pairs the blocks so that every
// round updates disjoint column sets in parallel (one workgroup per block
// pair).  A workgroup forms the 32 x 32 Gram matrix of its two blocks from
// the actual columns, diagonalises it with a cyclic two-sided Jacobi in LDS,
// and applies the resulting rotation to the 32 columns of G and of V.
// Convergence: every pair's largest relative off-diagonal
// |g_i . g_j| / (|g_i| |g_j|) below tol in a whole sweep.  W is a product
// of plane rotations, so the method is backward stable (the result is the
// exact SVD of M + dM with |dM| ~ eps |M|), which is the accuracy of the
// LAPACK SVD used by the oracle.
//
// Storage is column-major for G and V (Gt[j][:] = column j), so that each
// column is one contiguous row of Gt.
#include "kernels.hpp"

#include <algorithm>
#include <cmath>
#include <cstdlib>

namespace sctm {

static constexpr int JW = 16;        // columns per block
static constexpr int JP = 2 * JW;    // columns per block pair

static inline int padded(int n) { return ((n + JP - 1) / JP) * JP; }

struct SvdLayout {
  int np, nb, pairs, rounds;
  long sG, sV, sOff;
  size_t offG, offV, offOff, offNorm, offRank, offDone, offFro, total;
};

static SvdLayout layout(int n, int batch) {
  SvdLayout L;
  L.np = padded(n);
  L.nb = L.np / JW;
  L.pairs = L.nb / 2;
  L.rounds = L.nb - 1;
  L.sG = (long)L.np * n;
  L.sV = (long)L.np * L.np;
  L.sOff = (long)L.pairs * L.rounds;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  L.offG = take(sizeof(double) * L.sG * batch);
  L.offV = take(sizeof(double) * L.sV * batch);
  L.offOff = take(sizeof(double) * L.sOff * batch);
  L.offNorm = take(sizeof(double) * (size_t)L.np * batch);
  L.offRank = take(sizeof(int) * (size_t)L.np * batch);
  L.offDone = take(sizeof(int) * (size_t)batch);
  L.offFro = take(sizeof(double) * (size_t)batch);
  L.total = off;
  return L;
}

size_t svd_work_bytes(int n, int batch) { return layout(n, batch).total; }

// Gt = M^T (cold start) or only its padding rows (warm start: rows < n come
// from Gt = (M V0)^T by GEMM); Vt = I or V0^T, padded with the identity.
__global__ void svd_init_kernel(const double* M, const double* V0, int n, int np, double* Gt, double* Vt, int* done,
                                long sG, long sV) {
  const int b = blockIdx.y;
  M += (long)b * n * n;
  if (V0) V0 += (long)b * n * n;
  Gt += b * sG;
  Vt += b * sV;
  long totG = (long)np * n, totV = (long)np * np;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < totG + totV; e += (long)gridDim.x * blockDim.x) {
    if (e < totG) {
      long j = e / n, i = e % n;
      if (!V0)
        Gt[e] = (j < n) ? M[i * n + j] : 0.0;
      else if (j >= n)
        Gt[e] = 0.0;
    } else {
      long f = e - totG;
      long j = f / np, i = f % np;
      Vt[f] = (V0 && i < n && j < n) ? V0[i * n + j] : ((i == j) ? 1.0 : 0.0);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) done[b] = 0;
}

__device__ inline void circle_pair(int players, int round, int idx, int& a, int& b) {
  if (idx == 0) {
    a = 0;
    b = 1 + round;
  } else {
    a = 1 + (round + idx) % (players - 1);
    b = 1 + (round - idx + players - 1) % (players - 1);
  }
}

// Four 64-wide wavefronts per block pair.  The rows of the 32 columns are
// split over the waves: each wave forms a partial Gram matrix on the FP64
// matrix cores (v_mfma_f64_16x16x4: A lane l holds A[l%16][l/16], B lane l
// holds B[l/16][l%16], D lane l register r holds D[4r + l/16][l%16]), the
// partials are summed in LDS, the 32 x 32 eigenproblem is solved in LDS, and
// each wave rotates its share of the rows of G and V on the matrix cores.
//
// A pair counts as orthogonal when |g_i . g_j| <= tol |g_i| |g_j| (relative
// criterion: every singular triplet, small ones included, is fixed to
// relative accuracy O(tol) when M is well conditioned up to column scaling).
// Columns below 1e-15 |M|_F are rounding noise of the rotations themselves:
// a pair of two such columns is never rotated and does not count.
typedef double d4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void jacobi_round_kernel(double* Gt_all, double* Vt_all, int m, int np, int round,
                                                           double tol, double* off_all, const int* done, long sG,
                                                           long sV, long sOff, int inner_sweeps,
                                                           const double* fro2_all) {
  const int b = blockIdx.y;
  if (done[b]) return;
  double* Gt = Gt_all + b * sG;
  double* Vt = Vt_all + b * sV;
  double* offv = off_all + b * sOff;
  const double negl2 = 1e-30 * fro2_all[b];   // (1e-15 |M|_F)^2
  const int nb = np / JW;
  const int pr = blockIdx.x;
  int p, q;
  circle_pair(nb, round, pr, p, q);

  __shared__ double buf[4][JP][65];     // per-wave staging; reused for the Gram partials
  __shared__ double H[JP][JP + 1];
  __shared__ double W[JP][JP + 1];
  __shared__ int rowidx[JP];
  __shared__ double wmax[4];
  __shared__ int any;
  const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;
  if (tid < JP) rowidx[tid] = (tid < JW) ? p * JW + tid : q * JW + (tid - JW);
  __syncthreads();

  // ---- partial Gram matrices, wave wv takes row chunks wv, wv+4, ... ----
  d4v acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = d4v{0, 0, 0, 0};
  for (int cb = 0; cb < m; cb += 256) {   // uniform trip count for every wave
    const int c0 = cb + wv * 64;
    for (int r = 0; r < JP; ++r) buf[wv][r][l] = (c0 + l < m) ? Gt[(long)rowidx[r] * m + c0 + l] : 0.0;
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      const int kc = kk * 4 + (l >> 4);
      double a0 = buf[wv][l & 15][kc], a1 = buf[wv][16 + (l & 15)][kc];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int ti = 0; ti < 2; ++ti)
    for (int tj = 0; tj < 2; ++tj)
      for (int r = 0; r < 4; ++r) buf[wv][ti * 16 + 4 * r + (l >> 4)][tj * 16 + (l & 15)] = acc[ti][tj][r];
  __syncthreads();
  for (int e = tid; e < JP * JP; e += 256) {
    int i = e / JP, j = e % JP;
    H[i][j] = buf[0][i][j] + buf[1][i][j] + buf[2][i][j] + buf[3][i][j];
  }
  __syncthreads();

  // ---- convergence measure of this pair (NaN-propagating max) ----
  double om = 0.0;
  for (int e = tid; e < JP * JP; e += 256) {
    int i = e / JP, j = e % JP;
    if (j > i) {
      const double hii = fmax(H[i][i], 0.0), hjj = fmax(H[j][j], 0.0);
      double v = (fmax(hii, hjj) <= negl2) ? 0.0 : fabs(H[i][j]) / (sqrt(hii) * sqrt(hjj) + 1e-300);
      if (H[i][j] != H[i][j] || H[i][i] != H[i][i] || H[j][j] != H[j][j]) v = NAN;
      om = (v != v || om != om) ? NAN : fmax(om, v);
    }
  }
  for (int w = 32; w > 0; w >>= 1) {
    double o = __shfl_xor(om, w);
    om = (o != o || om != om) ? NAN : fmax(om, o);
  }
  if (l == 0) wmax[wv] = om;
  __syncthreads();
  {
    double a = wmax[0];
    for (int k = 1; k < 4; ++k) a = (a != a || wmax[k] != wmax[k]) ? NAN : fmax(a, wmax[k]);
    om = a;
  }
  if (tid == 0) offv[(long)round * (nb / 2) + pr] = om;
  if (!(om > tol)) return;   // converged pair (or NaN: leave the data as is)

  // ---- diagonalise H with cyclic two-sided Jacobi; W accumulates.  In each
  // inner round the 32 indices form 16 disjoint pairs; thread (p, q) owns the
  // 2 x 2 block of H at pairs p (rows) and q (columns) and the rows of W at
  // pair p, computes both rotations itself, and forms J_p^T H J_q and W J_q
  // in registers: one barrier after all reads, one after all writes. ----
  for (int e = tid; e < JP * JP; e += 256) W[e / JP][e % JP] = (e / JP == e % JP) ? 1.0 : 0.0;
  const double rot_thr = 0.1 * tol;
  const int pp = tid >> 4, qq = tid & 15;
  for (int sw = 0; sw < inner_sweeps; ++sw) {
    __syncthreads();
    if (tid == 0) any = 0;
    __syncthreads();
    for (int rr = 0; rr < JP - 1; ++rr) {
      int ap, cp, aq, cq;
      circle_pair(JP, rr, pp, ap, cp);
      circle_pair(JP, rr, qq, aq, cq);
      double c1 = 1.0, s1 = 0.0, c2 = 1.0, s2 = 0.0;
      {
        const double haa = H[ap][ap], hcc = H[cp][cp], hac = H[ap][cp];
        if (fmax(haa, hcc) > negl2 && fabs(hac) > rot_thr * sqrt(fmax(haa, 0.0)) * sqrt(fmax(hcc, 0.0))) {
          const double zeta = (hcc - haa) / (2.0 * hac);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c1 = 1.0 / sqrt(1.0 + t * t);
          s1 = c1 * t;
          if (qq == 0) any = 1;
        }
      }
      {
        const double haa = H[aq][aq], hcc = H[cq][cq], hac = H[aq][cq];
        if (fmax(haa, hcc) > negl2 && fabs(hac) > rot_thr * sqrt(fmax(haa, 0.0)) * sqrt(fmax(hcc, 0.0))) {
          const double zeta = (hcc - haa) / (2.0 * hac);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c2 = 1.0 / sqrt(1.0 + t * t);
          s2 = c2 * t;
        }
      }
      const double h00 = H[ap][aq], h01 = H[ap][cq], h10 = H[cp][aq], h11 = H[cp][cq];
      const double w00 = W[ap][aq], w01 = W[ap][cq], w10 = W[cp][aq], w11 = W[cp][cq];
      // rows: J_p^T
      const double r00 = c1 * h00 - s1 * h10, r01 = c1 * h01 - s1 * h11;
      const double r10 = s1 * h00 + c1 * h10, r11 = s1 * h01 + c1 * h11;
      __syncthreads();
      H[ap][aq] = c2 * r00 - s2 * r01;
      H[ap][cq] = s2 * r00 + c2 * r01;
      H[cp][aq] = c2 * r10 - s2 * r11;
      H[cp][cq] = s2 * r10 + c2 * r11;
      W[ap][aq] = c2 * w00 - s2 * w01;
      W[ap][cq] = s2 * w00 + c2 * w01;
      W[cp][aq] = c2 * w10 - s2 * w11;
      W[cp][cq] = s2 * w10 + c2 * w11;
      __syncthreads();
    }
    if (!any) break;
  }
  __syncthreads();

  // ---- rotate the 32 columns of G and of V: new = W^T old, per wave ----
  for (int pass = 0; pass < 2; ++pass) {
    double* X = pass == 0 ? Gt : Vt;
    const int len = pass == 0 ? m : np;
    for (int cb = 0; cb < len; cb += 256) {   // uniform trip count for every wave
      const int c0 = cb + wv * 64;
      for (int r = 0; r < JP; ++r) buf[wv][r][l] = (c0 + l < len) ? X[(long)rowidx[r] * len + c0 + l] : 0.0;
      __syncthreads();
      for (int ti = 0; ti < 2; ++ti)
        for (int tc = 0; tc < 4; ++tc) {
          d4v d = {0, 0, 0, 0};
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            const int j = kk * 4 + (l >> 4);
            double a = W[j][ti * 16 + (l & 15)];      // (W^T)[i][j]
            double bb = buf[wv][j][tc * 16 + (l & 15)];
            d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, d, 0, 0, 0);
          }
          for (int r = 0; r < 4; ++r) {
            const int i = ti * 16 + 4 * r + (l >> 4), c = c0 + tc * 16 + (l & 15);
            if (c < len) X[(long)rowidx[i] * len + c] = d[r];
          }
        }
      __syncthreads();
    }
  }
}

// |M|_F^2 of every batch entry (one block each)
__global__ void svd_fro2_kernel(const double* M, long nn, double* fro2) {
  const double* x = M + (long)blockIdx.x * nn;
  __shared__ double red[256];
  double a = 0.0;
  for (long i = threadIdx.x; i < nn; i += blockDim.x) a += x[i] * x[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) fro2[blockIdx.x] = red[0];
}

__global__ void svd_check_kernel(const double* off_all, long sOff, double tol, int* done) {
  const int b = blockIdx.x;
  const double* o = off_all + b * sOff;
  __shared__ double red[256];
  double m = 0.0;
  for (long i = threadIdx.x; i < sOff; i += blockDim.x) m = fmax(m, o[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    done[b] = (red[0] <= tol) ? 1 : done[b];
  }
}

__global__ void svd_norms_kernel(const double* Gt_all, int n, long sG, double* norms_all, int np) {
  const int j = blockIdx.x, b = blockIdx.y;
  const double* g = Gt_all + b * sG + (long)j * n;
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += g[i] * g[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) norms_all[(long)b * np + j] = sqrt(red[0]);
}

__global__ void svd_rank_kernel(const double* norms_all, int n, int np, int* rank_all) {
  const int b = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double* s = norms_all + (long)b * np;
  double sj = s[j];
  int r = 0;
  for (int i = 0; i < n; ++i) {
    double si = s[i];
    r += (si > sj || (si == sj && i < j)) ? 1 : 0;
  }
  rank_all[(long)b * np + j] = r;
}

__global__ void svd_scatter_kernel(const double* Gt_all, const double* Vt_all, const double* norms_all,
                                   const int* rank_all, int n, int np, long sG, long sV, double* U, double* S,
                                   double* V) {
  const int b = blockIdx.y;
  const double* Gt = Gt_all + b * sG;
  const double* Vt = Vt_all + b * sV;
  const double* nr = norms_all + (long)b * np;
  const int* rk = rank_all + (long)b * np;
  U += (long)b * n * n;
  V += (long)b * n * n;
  S += (long)b * n;
  long tot = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    int j = (int)(e / n), i = (int)(e % n);
    int r = rk[j];
    double sj = nr[j];
    U[(long)i * n + r] = (sj > 0.0) ? Gt[(long)j * n + i] / sj : 0.0;
    V[(long)i * n + r] = Vt[(long)j * np + i];
    if (i == 0) S[r] = sj;
  }
}

hipError_t svd_f64(hipStream_t s, int n, int batch, const double* M, double* U, double* S, double* V, void* work,
                   int max_sweeps, double tol, int* host_flags, int* sweeps_out, const double* V0) {
  if (!(tol > 0.0)) tol = 1.2e-16 * std::sqrt((double)n);   // ~ sqrt(m) eps: the rounding floor of a dot product
  SvdLayout L = layout(n, batch);
  char* w = (char*)work;
  double* Gt = (double*)(w + L.offG);
  double* Vt = (double*)(w + L.offV);
  double* off = (double*)(w + L.offOff);
  double* norms = (double*)(w + L.offNorm);
  int* rank = (int*)(w + L.offRank);
  int* done = (int*)(w + L.offDone);
  double* fro2 = (double*)(w + L.offFro);
  hipLaunchKernelGGL(svd_fro2_kernel, dim3(batch), dim3(256), 0, s, M, (long)n * n, fro2);
  hipError_t err = hipSuccess;
  {
    long tot = (long)L.np * n + (long)L.np * L.np;
    int g = (int)std::min<long>((tot + 255) / 256, 8192);
    hipLaunchKernelGGL(svd_init_kernel, dim3(g, batch), dim3(256), 0, s, M, V0, n, L.np, Gt, Vt, done, L.sG, L.sV);
    if (V0) {   // Gt[j][i] = sum_k V0[k][j] M[i][k]
      err = gemm_f64(s, true, true, n, n, n, 1.0, V0, n, (long)n * n, M, n, (long)n * n, 0.0, Gt, n, L.sG, batch);
      if (err != hipSuccess) return err;
    }
  }
  int sweeps = 0;
  static const int inner = [] {
    const char* e = std::getenv("SPLITCTM_SVD_INNER");
    int v = e ? std::atoi(e) : 2;
    return v < 1 ? 1 : (v > 12 ? 12 : v);
  }();
  err = hipSuccess;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    KernelTimer* tm = kernel_timer();
    // nominal work of one round: Gram matrix and rotation of G and V for every pair
    const double round_work = (double)L.pairs * batch * 2.0 * JP * JP * (2.0 * n + L.np);
    for (int r = 0; r < L.rounds; ++r) {
      if (tm) tm->begin(s, KC_JACOBI, round_work);
      hipLaunchKernelGGL(jacobi_round_kernel, dim3(L.pairs, batch), dim3(256), 0, s, Gt, Vt, n, L.np, r, tol, off,
                         done, L.sG, L.sV, L.sOff, inner, fro2);
      if (tm) tm->end(s);
    }
    hipLaunchKernelGGL(svd_check_kernel, dim3(batch), dim3(256), 0, s, off, L.sOff, tol, done);
    ++sweeps;
    err = hipMemcpyAsync(host_flags, done, sizeof(int) * batch, hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) return err;
    bool all = true;
    for (int b = 0; b < batch; ++b) all = all && host_flags[b];
    if (all) break;
  }
  hipLaunchKernelGGL(svd_norms_kernel, dim3(n, batch), dim3(256), 0, s, Gt, n, L.sG, norms, L.np);
  hipLaunchKernelGGL(svd_rank_kernel, dim3((n + 255) / 256, batch), dim3(256), 0, s, norms, n, L.np, rank);
  {
    long tot = (long)n * n;
    int g = (int)std::min<long>((tot + 255) / 256, 8192);
    hipLaunchKernelGGL(svd_scatter_kernel, dim3(g, batch), dim3(256), 0, s, Gt, Vt, norms, rank, n, L.np, L.sG, L.sV,
                       U, S, V);
  }
  if (sweeps_out) *sweeps_out = sweeps;
  return hipGetLastError();
}

}  // namespace sctm
