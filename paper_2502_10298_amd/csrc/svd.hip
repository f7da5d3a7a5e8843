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

namespace sctm {

static constexpr int JW = 16;        // columns per block
static constexpr int JP = 2 * JW;    // columns per block pair

static inline int padded(int n) { return ((n + JP - 1) / JP) * JP; }

struct SvdLayout {
  int np, nb, pairs, rounds;
  long sG, sV, sOff;
  size_t offG, offV, offOff, offNorm, offRank, offDone, total;
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
  L.total = off;
  return L;
}

size_t svd_work_bytes(int n, int batch) { return layout(n, batch).total; }

__global__ void svd_init_kernel(const double* M, int n, int np, double* Gt, double* Vt, int* done, long sG,
                                long sV) {
  const int b = blockIdx.y;
  M += (long)b * n * n;
  Gt += b * sG;
  Vt += b * sV;
  long totG = (long)np * n, totV = (long)np * np;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < totG + totV; e += (long)gridDim.x * blockDim.x) {
    if (e < totG) {
      long j = e / n, i = e % n;
      Gt[e] = (j < n) ? M[i * n + j] : 0.0;
    } else {
      long f = e - totG;
      long j = f / np, i = f % np;
      Vt[f] = (i == j) ? 1.0 : 0.0;
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

__global__ __launch_bounds__(256) void jacobi_round_kernel(double* Gt_all, double* Vt_all, int m, int np, int round,
                                                           double tol, double* off_all, const int* done, long sG,
                                                           long sV, long sOff) {
  const int b = blockIdx.y;
  if (done[b]) return;
  double* Gt = Gt_all + b * sG;
  double* Vt = Vt_all + b * sV;
  double* offv = off_all + b * sOff;
  const int nb = np / JW;
  const int pr = blockIdx.x;
  int p, q;
  circle_pair(nb, round, pr, p, q);

  __shared__ double H[JP][JP + 1];
  __shared__ double W[JP][JP + 1];
  __shared__ double buf[JP][65];
  __shared__ double red[256];
  __shared__ double csc[16], css[16];
  __shared__ int pa[16], pb[16];
  __shared__ int rowidx[JP];
  __shared__ int any;
  const int tid = threadIdx.x;
  if (tid < JP) rowidx[tid] = (tid < JW) ? p * JW + tid : q * JW + (tid - JW);

  // ---- Gram matrix of the 32 columns ----
  double h[4] = {0.0, 0.0, 0.0, 0.0};
  const int hi = tid >> 3, hj0 = (tid & 7) * 4;
  for (int c0 = 0; c0 < m; c0 += 64) {
    __syncthreads();
    for (int e = tid; e < JP * 64; e += 256) {
      int r = e >> 6, c = e & 63;
      buf[r][c] = (c0 + c < m) ? Gt[(long)rowidx[r] * m + c0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int c = 0; c < 64; ++c) {
      double a = buf[hi][c];
      h[0] += a * buf[hj0 + 0][c];
      h[1] += a * buf[hj0 + 1][c];
      h[2] += a * buf[hj0 + 2][c];
      h[3] += a * buf[hj0 + 3][c];
    }
  }
  for (int t = 0; t < 4; ++t) H[hi][hj0 + t] = h[t];
  __syncthreads();
  // ---- convergence measure of this pair ----
  double om = 0.0;
  for (int t = 0; t < 4; ++t) {
    int j = hj0 + t;
    if (j > hi) {
      double d = H[hi][hi] * H[j][j];
      if (d > 0.0) om = fmax(om, fabs(H[hi][j]) / sqrt(d));
    }
  }
  red[tid] = om;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double omax = red[0];
  if (tid == 0) offv[(long)round * (nb / 2) + pr] = omax;
  if (omax <= tol) return;   // block-uniform

  // ---- diagonalise H with cyclic two-sided Jacobi, W accumulates ----
  for (int e = tid; e < JP * JP; e += 256) W[e / JP][e % JP] = (e / JP == e % JP) ? 1.0 : 0.0;
  for (int sw = 0; sw < 12; ++sw) {
    __syncthreads();
    if (tid == 0) any = 0;
    __syncthreads();
    for (int rr = 0; rr < JP - 1; ++rr) {
      if (tid < 16) {
        int a, c;
        circle_pair(JP, rr, tid, a, c);
        double haa = H[a][a], hcc = H[c][c], hac = H[a][c];
        double cc = 1.0, ss = 0.0;
        if (hac != 0.0 && fabs(hac) > 1e-15 * sqrt(fabs(haa * hcc))) {
          double zeta = (hcc - haa) / (2.0 * hac);
          double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          cc = 1.0 / sqrt(1.0 + t * t);
          ss = cc * t;
          any = 1;
        }
        csc[tid] = cc;
        css[tid] = ss;
        pa[tid] = a;
        pb[tid] = c;
      }
      __syncthreads();
      for (int e = tid; e < 16 * JP; e += 256) {   // H <- J^T H (rows)
        int i = e / JP, k = e % JP, a = pa[i], c = pb[i];
        double cc = csc[i], ss = css[i];
        double x = H[a][k], y = H[c][k];
        H[a][k] = cc * x - ss * y;
        H[c][k] = ss * x + cc * y;
      }
      __syncthreads();
      for (int e = tid; e < 16 * JP; e += 256) {   // H <- H J, W <- W J (columns)
        int i = e / JP, k = e % JP, a = pa[i], c = pb[i];
        double cc = csc[i], ss = css[i];
        double x = H[k][a], y = H[k][c];
        H[k][a] = cc * x - ss * y;
        H[k][c] = ss * x + cc * y;
        x = W[k][a];
        y = W[k][c];
        W[k][a] = cc * x - ss * y;
        W[k][c] = ss * x + cc * y;
      }
      __syncthreads();
    }
    if (!any) break;
  }
  __syncthreads();

  // ---- apply W to the 32 columns of G and of V:  col_i <- sum_j col_j W[j][i] ----
  for (int pass = 0; pass < 2; ++pass) {
    double* X = pass == 0 ? Gt : Vt;
    const int len = pass == 0 ? m : np;
    for (int c0 = 0; c0 < len; c0 += 64) {
      __syncthreads();
      for (int e = tid; e < JP * 64; e += 256) {
        int r = e >> 6, c = e & 63;
        buf[r][c] = (c0 + c < len) ? X[(long)rowidx[r] * len + c0 + c] : 0.0;
      }
      __syncthreads();
      for (int e = tid; e < JP * 64; e += 256) {
        int i = e >> 6, c = e & 63;
        double acc = 0.0;
#pragma unroll 8
        for (int j = 0; j < JP; ++j) acc += W[j][i] * buf[j][c];
        if (c0 + c < len) X[(long)rowidx[i] * len + c0 + c] = acc;
      }
    }
  }
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
                   int max_sweeps, double tol, int* host_flags, int* sweeps_out) {
  SvdLayout L = layout(n, batch);
  char* w = (char*)work;
  double* Gt = (double*)(w + L.offG);
  double* Vt = (double*)(w + L.offV);
  double* off = (double*)(w + L.offOff);
  double* norms = (double*)(w + L.offNorm);
  int* rank = (int*)(w + L.offRank);
  int* done = (int*)(w + L.offDone);
  hipError_t err;
  {
    long tot = (long)L.np * n + (long)L.np * L.np;
    int g = (int)std::min<long>((tot + 255) / 256, 8192);
    hipLaunchKernelGGL(svd_init_kernel, dim3(g, batch), dim3(256), 0, s, M, n, L.np, Gt, Vt, done, L.sG, L.sV);
  }
  int sweeps = 0;
  err = hipSuccess;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    for (int r = 0; r < L.rounds; ++r)
      hipLaunchKernelGGL(jacobi_round_kernel, dim3(L.pairs, batch), dim3(256), 0, s, Gt, Vt, n, L.np, r, tol, off,
                         done, L.sG, L.sV, L.sOff);
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
