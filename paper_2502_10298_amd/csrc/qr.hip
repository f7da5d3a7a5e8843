// Batched FP64 Householder QR of tall matrices X (m x k, m >= k), stored as
// Xt = X^T row-major (row j of Xt = column j of X, contiguous), with the
// explicit thin factor Q (m x k, also stored transposed) and R (k x k).
//
// Blocked right-looking Householder with panels of 16, 8 or 4 columns (as
// many as the rows held per thread allow without register spills):
//   panel:    one workgroup per matrix factors the panel in registers
//             (thread t holds rows p0 + t + NT r), one reflector
//             per column (LAPACK's dlarfg convention: beta = -sign(x0) |x|,
//             tau = (beta - x0) / beta, v = x / (x0 - beta) with v_0 = 1) and
//             builds the triangular factor T of the block reflector
//             H_1 ... H_PW = I - V T V^T (forward, columnwise);
//   trailing: X_trail <- H^T X_trail, i.e. Xt_trail <- Xt_trail - (Xt_trail V) T V^T,
//             one fused kernel on the matrix cores;
//   Q:        Q = H_1 ... H_p [I; 0], accumulated backwards over the panels,
//             Qt <- Qt - (Qt V) T^T V^T on the trailing block, the same kernel.
// Householder QR is backward stable: Q is orthonormal to working accuracy
// and X = Q R + dX with |dX| ~ eps |X|, whatever the rank of X.
#include "kernels.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace sctm {

static constexpr int PW = 16;     // widest panel (T blocks are PW x PW)
static constexpr int TSLOT = 4;   // narrowest panel: one T block per TSLOT columns

struct QrLayout {
  long sX, sT;
  size_t offV, offT, total;
};

static QrLayout qr_layout(int m, int k, int batch) {
  QrLayout L;
  L.sX = (long)k * m;
  const int nslot = (k + TSLOT - 1) / TSLOT;
  L.sT = (long)nslot * PW * PW;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  L.offV = take(sizeof(double) * L.sX * batch);                // reflectors as rows [k][m]
  L.offT = take(sizeof(double) * L.sT * batch);                // T of every panel
  L.total = off;
  return L;
}

size_t qr_work_bytes(int m, int k, int batch) { return qr_layout(m, k, batch).total; }

// Factor the panel of columns p0 .. p0 + w - 1 (rows p0 .. m - 1) of every
// matrix; writes the reflectors (below the diagonal) and R (on and above it)
// back into Xt, the reflectors as full rows into Vr (zeros above, 1 on the
// diagonal) and the panel's T.  NT threads, RM rows per thread
// (m - p0 <= NT RM), PWT columns.
//
// One block-wide reduction per column: with v = [1; x_below scale] every dot
// product the step needs follows from the raw sums s_l = sum_{i > c} x_ij x_il
// and the diagonal row c, d_l = x_cl + scale s_l: for l > j the coefficient of
// the update of column l, for l < j the entry v_l . v_j of T's recurrence,
// and s_j = |x_below|^2.  The sums go through LDS in two stages.
template <int NT, int RM, int PWT>
__global__ __launch_bounds__(NT) void qr_panel_kernel(double* Xt_all, double* Vr_all, double* T_all, int m, int k,
                                                      long sX, long sT, int p0) {
  constexpr int NSEG = NT / PWT;   // stage-2 segments of PWT partial rows each
  const int b = blockIdx.x;
  double* Xt = Xt_all + b * sX;
  double* Vr = Vr_all + b * sX;
  double* Tp = T_all + b * sT + (long)(p0 / TSLOT) * PW * PW;
  const int w = min(PWT, k - p0);
  const int t = threadIdx.x;
  __shared__ double buf[NT][PWT + 1];
  __shared__ double seg[NSEG][PWT + 1];
  __shared__ double S[PWT];
  __shared__ double rowc[2][PWT];
  __shared__ double Ts[PW][PW];
  double x[RM][PWT];
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int i = p0 + t + NT * r;
#pragma unroll
    for (int l = 0; l < PWT; ++l) x[r][l] = (i < m && l < w) ? Xt[(long)(p0 + l) * m + i] : 0.0;
  }
  for (int e = t; e < PW * PW; e += NT) Ts[e / PW][e % PW] = 0.0;
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    const int c = p0 + j;
    double* rc = rowc[j & 1];
    // partial sums over this thread's rows below the diagonal; the owner of
    // row c publishes it
    double part[PWT];
#pragma unroll
    for (int l = 0; l < PWT; ++l) part[l] = 0.0;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const int i = p0 + t + NT * r;
      double xj = 0.0;
#pragma unroll
      for (int l = 0; l < PWT; ++l)
        if (l == j) xj = x[r][l];
      if (i > c && i < m) {
#pragma unroll
        for (int l = 0; l < PWT; ++l) part[l] += xj * x[r][l];
      }
      if (i == c) {
#pragma unroll
        for (int l = 0; l < PWT; ++l) rc[l] = x[r][l];
      }
    }
#pragma unroll
    for (int l = 0; l < PWT; ++l) buf[t][l] = part[l];
    __syncthreads();
    {
      const int l = t % PWT, g = t / PWT;
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < PWT; ++q) a += buf[g * PWT + q][l];
      seg[g][l] = a;
    }
    __syncthreads();
    if (t < PWT) {
      double a = 0.0;
      for (int g = 0; g < NSEG; ++g) a += seg[g][t];
      S[t] = a;
    }
    __syncthreads();
    const double sq = S[j], x0 = rc[j];
    double tau = 0.0, beta = x0, scale = 0.0;
    if (sq > 0.0) {
      beta = -copysign(sqrt(x0 * x0 + sq), x0);
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    // v into column j (R entry on the diagonal), then H_j on columns l > j
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const int i = p0 + t + NT * r;
      double vi = 0.0;
#pragma unroll
      for (int l = 0; l < PWT; ++l)
        if (l == j) {
          if (i > c && i < m) x[r][l] *= scale;
          if (i == c) x[r][l] = beta;
          vi = (i == c) ? 1.0 : ((i > c && i < m) ? x[r][l] : 0.0);
        }
#pragma unroll
      for (int l = 0; l < PWT; ++l)
        if (l > j) x[r][l] -= tau * (rc[l] + scale * S[l]) * vi;
    }
    // T column j:  T[0:j, j] = -tau T[0:j, 0:j] z,  z_q = v_q . v_j = d_q
    if (t < j) {
      double a = 0.0;
      for (int q = t; q < j; ++q) a += Ts[t][q] * (rc[q] + scale * S[q]);
      Ts[t][j] = -tau * a;
    }
    if (t == j) Ts[j][j] = tau;
  }
  __syncthreads();
  // write back: Xt rows p0 .. p0 + w - 1, the reflector rows, T
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int i = p0 + t + NT * r;
    if (i < m)
#pragma unroll
      for (int l = 0; l < PWT; ++l)
        if (l < w) {
          Xt[(long)(p0 + l) * m + i] = x[r][l];
          Vr[(long)(p0 + l) * m + i] = (i < p0 + l) ? 0.0 : ((i == p0 + l) ? 1.0 : x[r][l]);
        }
  }
  // rows of Vr before p0 are zero (the reflectors act on rows >= p0 + l)
  for (int l = 0; l < w; ++l)
    for (int i = t; i < p0; i += NT) Vr[(long)(p0 + l) * m + i] = 0.0;
  for (int e = t; e < PW * PW; e += NT) Tp[e] = Ts[e / PW][e % PW];
}

// Y <- Y - ((Y V) T') V^T for the rows of Y (nt rows of length len, leading
// dimension ld), V^T = the panel's reflectors (pw <= 16 rows of length len,
// leading dimension ld) and T' = T (trailing update of the factorisation) or
// T^T (accumulation of Q).  One workgroup per 16 rows of Y: the four
// wavefronts split the length for Y V (MFMA, partial products summed in LDS
// in a fixed order), form (Y V) T' in LDS, then split the column tiles of
// the rank-pw update (MFMA again).  v_mfma_f64_16x16x4: A lane l holds
// A[l%16][l/16], B lane l holds B[l/16][l%16], D lane l register r holds
// D[4r + l/16][l%16]; in Y V lane l takes the summation index
// k = kb + 16 (l/16) + j at step j, so that each lane streams 16 consecutive
// entries of its row of Y and of V.
template <bool TRANS_T>
__global__ __launch_bounds__(256) void qr_update_kernel(double* Y_all, long sY, int nt, int len, int ld,
                                                        const double* V_all, long sV, const double* T_all, long sT,
                                                        int pw) {
  typedef double d4u __attribute__((ext_vector_type(4)));
  const int b = blockIdx.y;
  double* Y = Y_all + b * sY;
  const double* V = V_all + b * sV;
  const double* T = T_all + b * sT;
  const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;
  const int row0 = blockIdx.x * 16;
  __shared__ double Ts[PW][PW + 1];
  __shared__ double red[4][16][17];
  __shared__ double w2[16][PW + 1];
  for (int e = tid; e < PW * PW; e += 256) Ts[e / PW][e % PW] = T[e];
  // partial W1 = Y V over the wave's quarter of the length (64-entry blocks)
  const int nblk = (len + 63) / 64;
  const int ra = row0 + (l & 15);
  const bool rok = ra < nt, vok = (l & 15) < pw;
  const double* yrow = Y + (long)ra * ld;
  const double* vrow = V + (long)(l & 15) * ld;
  d4u d = {0, 0, 0, 0};
  for (int blk = wv; blk < nblk; blk += 4) {
    const int k0 = blk * 64 + 16 * (l >> 4);
    double av[16], bv[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int kk = k0 + j;
      av[j] = (rok && kk < len) ? yrow[kk] : 0.0;
      bv[j] = (vok && kk < len) ? vrow[kk] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[j], bv[j], d, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wv][4 * r + (l >> 4)][l & 15] = d[r];
  __syncthreads();
  // W2 = W1 T'  (16 x pw), W1 = sum of the four partials
  {
    const int i = tid >> 4, c = tid & 15;
    double a = 0.0;
    for (int j = 0; j < pw; ++j) {
      const double w1 = (red[0][i][j] + red[1][i][j]) + (red[2][i][j] + red[3][i][j]);
      a += w1 * (TRANS_T ? Ts[c][j] : Ts[j][c]);
    }
    w2[i][c] = (c < pw) ? a : 0.0;
  }
  __syncthreads();
  // Y -= W2 V^T, the waves taking 16-column tiles in turn
  const int nk = (pw + 3) / 4;
  for (int i0 = wv * 16; i0 < len; i0 += 64) {
    const int ci = i0 + (l & 15);
    d4u u = {0, 0, 0, 0};
    for (int kk = 0; kk < nk; ++kk) {
      const int j = kk * 4 + (l >> 4);
      const double a = (j < pw) ? w2[l & 15][j] : 0.0;
      const double bb = (j < pw && ci < len) ? V[(long)j * ld + ci] : 0.0;
      u = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bb, u, 0, 0, 0);
    }
    if (ci < len) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = row0 + 4 * r + (l >> 4);
        if (rr < nt) Y[(long)rr * ld + ci] -= u[r];
      }
    }
  }
}

// R (k x k, row-major, zero below the diagonal) from the factored Xt
__global__ void qr_extract_r_kernel(const double* Xt_all, double* R_all, int m, int k, long sX) {
  const int b = blockIdx.y;
  const double* Xt = Xt_all + b * sX;
  double* R = R_all + (long)b * k * k;
  const long n = (long)k * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    R[e] = (j >= i) ? Xt[(long)j * m + i] : 0.0;
  }
}

// Qt = [I_k 0] (k x m)
__global__ void qr_eye_kernel(double* Qt_all, int m, int k, long sX) {
  const int b = blockIdx.y;
  double* Qt = Qt_all + b * sX;
  const long n = (long)k * m;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    Qt[e] = (e / m == e % m) ? 1.0 : 0.0;
}

static int grid_of(long n) { return (int)std::min<long>((n + 255) / 256, 4096); }

hipError_t qr_f64(hipStream_t s, int m, int k, int batch, double* Xt, double* R, double* Qt, void* work) {
  if (m < k || k < 1 || batch < 1) return hipErrorInvalidValue;
  if (m > 4096) return hipErrorInvalidValue;   // rows held in registers: at most 4 per thread
  QrLayout L = qr_layout(m, k, batch);
  char* w = (char*)work;
  double* Vr = (double*)(w + L.offV);
  double* T = (double*)(w + L.offT);
  hipError_t e = hipSuccess;
  // panels: 256 threads with up to 4 rows each and 16 columns, or 8 rows
  // and 8 columns; beyond 2048 rows 1024 threads with 4 columns
  struct Panel {
    int p0, pw, nt_threads, rm;
  };
  std::vector<Panel> pans;
  for (int p0 = 0; p0 < k;) {
    const int rows = m - p0;
    Panel P;
    P.p0 = p0;
    if (rows <= 2048) {
      const int need = (rows + 255) / 256;
      P.nt_threads = 256;
      P.rm = need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 8;
      P.pw = std::min(P.rm == 8 ? 8 : 16, k - p0);
    } else {
      P.nt_threads = 1024;
      P.rm = (rows + 1023) / 1024;
      P.pw = std::min(4, k - p0);
    }
    pans.push_back(P);
    p0 += P.pw;
  }
  for (const Panel& P : pans) {
    if (e != hipSuccess) break;
    const int p0 = P.p0, pw = P.pw, rows = m - p0;
    const dim3 g(batch);
    if (P.nt_threads == 256) {
      if (P.rm == 1)
        hipLaunchKernelGGL((qr_panel_kernel<256, 1, 16>), g, dim3(256), 0, s, Xt, Vr, T, m, k, L.sX, L.sT, p0);
      else if (P.rm == 2)
        hipLaunchKernelGGL((qr_panel_kernel<256, 2, 16>), g, dim3(256), 0, s, Xt, Vr, T, m, k, L.sX, L.sT, p0);
      else if (P.rm == 4)
        hipLaunchKernelGGL((qr_panel_kernel<256, 4, 16>), g, dim3(256), 0, s, Xt, Vr, T, m, k, L.sX, L.sT, p0);
      else
        hipLaunchKernelGGL((qr_panel_kernel<256, 8, 8>), g, dim3(256), 0, s, Xt, Vr, T, m, k, L.sX, L.sT, p0);
    } else {
      if (P.rm <= 3)
        hipLaunchKernelGGL((qr_panel_kernel<1024, 3, 4>), g, dim3(1024), 0, s, Xt, Vr, T, m, k, L.sX, L.sT, p0);
      else
        hipLaunchKernelGGL((qr_panel_kernel<1024, 4, 4>), g, dim3(1024), 0, s, Xt, Vr, T, m, k, L.sX, L.sT, p0);
    }
    e = hipGetLastError();
    const int nt = k - p0 - pw;   // trailing columns of X = rows of Xt
    if (nt <= 0 || e != hipSuccess) continue;
    // Xt_trail (nt x rows, ld m) -= ((Xt_trail V) T) V^T
    hipLaunchKernelGGL(qr_update_kernel<false>, dim3((nt + 15) / 16, batch), dim3(256), 0, s,
                       Xt + (long)(p0 + pw) * m + p0, L.sX, nt, rows, m, (const double*)(Vr + (long)p0 * m + p0),
                       L.sX, (const double*)(T + (long)(p0 / TSLOT) * PW * PW), L.sT, pw);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  if (R) {
    hipLaunchKernelGGL(qr_extract_r_kernel, dim3(grid_of((long)k * k), batch), dim3(256), 0, s, Xt, R, m, k, L.sX);
    e = hipGetLastError();
  }
  if (!Qt || e != hipSuccess) return e;
  hipLaunchKernelGGL(qr_eye_kernel, dim3(grid_of((long)k * m), batch), dim3(256), 0, s, Qt, m, k, L.sX);
  e = hipGetLastError();
  for (int pi = (int)pans.size() - 1; pi >= 0 && e == hipSuccess; --pi) {
    const int p0 = pans[pi].p0, pw = pans[pi].pw;
    const int rows = m - p0, nt = k - p0;
    // Qt_sub (rows p0.., columns p0..) -= ((Qt_sub V) T^T) V^T
    hipLaunchKernelGGL(qr_update_kernel<true>, dim3((nt + 15) / 16, batch), dim3(256), 0, s,
                       Qt + (long)p0 * m + p0, L.sX, nt, rows, m, (const double*)(Vr + (long)p0 * m + p0), L.sX,
                       (const double*)(T + (long)(p0 / TSLOT) * PW * PW), L.sT, pw);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace sctm
