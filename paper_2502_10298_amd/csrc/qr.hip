// Batched FP64 Householder QR of tall matrices X (m x k, m >= k), stored as
// Xt = X^T row-major (row j of Xt = column j of X, contiguous), with the
// explicit thin factor Q (m x k, also stored transposed) and R (k x k).
//
// Blocked right-looking Householder with panels of 16, 8 or 4 columns (as
// many as the rows held per thread allow without register spills):
//   panel:    one workgroup of 1024 threads per matrix factors the panel in
//             registers (thread t holds rows p0 + t + 1024 r), one reflector
//             per column (LAPACK's dlarfg convention: beta = -sign(x0) |x|,
//             tau = (beta - x0) / beta, v = x / (x0 - beta) with v_0 = 1) and
//             builds the triangular factor T of the block reflector
//             H_1 ... H_PW = I - V T V^T (forward, columnwise);
//   trailing: X_trail <- H^T X_trail, i.e. Xt_trail <- Xt_trail - (Xt_trail V) T V^T,
//             three batched GEMMs on the matrix cores;
//   Q:        Q = H_1 ... H_p [I; 0], accumulated backwards over the panels,
//             Qt <- Qt - (Qt V) T^T V^T on the trailing block, again GEMMs.
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
  size_t offV, offT, offW1, offW2, total;
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
  L.offW1 = take(sizeof(double) * (size_t)k * PW * batch);     // (rows x PW) products
  L.offW2 = take(sizeof(double) * (size_t)k * PW * batch);
  L.total = off;
  return L;
}

size_t qr_work_bytes(int m, int k, int batch) { return qr_layout(m, k, batch).total; }

// Block-wide sum of NV values per thread (1024 threads = 16 wavefronts);
// red: LDS scratch of 16 * NV doubles; the sums land in out[0 .. NV-1] (LDS)
// for every thread to read.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* red, double* out) {
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double a = v[q];
    for (int w = 32; w > 0; w >>= 1) a += __shfl_xor(a, w);
    v[q] = a;
  }
  if (l == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) red[wv * NV + q] = v[q];
  __syncthreads();
  if (threadIdx.x < NV) {
    double a = 0.0;
    for (int w = 0; w < 16; ++w) a += red[w * NV + threadIdx.x];
    out[threadIdx.x] = a;
  }
  __syncthreads();
}

// Factor the panel of columns p0 .. p0 + w - 1 (rows p0 .. m - 1) of every
// matrix; writes the reflectors (below the diagonal) and R (on and above it)
// back into Xt, the reflectors as full rows into Vr (zeros above, 1 on the
// diagonal) and the panel's T.  RM = rows per thread (m - p0 <= 1024 RM).
template <int RM, int PWT>
__global__ __launch_bounds__(1024) void qr_panel_kernel(double* Xt_all, double* Vr_all, double* T_all, int m, int k,
                                                        long sX, long sT, int p0) {
  const int b = blockIdx.x;
  double* Xt = Xt_all + b * sX;
  double* Vr = Vr_all + b * sX;
  double* Tp = T_all + b * sT + (long)(p0 / TSLOT) * PW * PW;
  const int w = min(PWT, k - p0);
  const int t = threadIdx.x;
  __shared__ double red[16 * PW];
  __shared__ double dots[PW];
  __shared__ double x0s;
  __shared__ double Ts[PW][PW];
  double x[RM][PWT];
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int i = p0 + t + 1024 * r;
#pragma unroll
    for (int l = 0; l < PWT; ++l) x[r][l] = (i < m && l < w) ? Xt[(long)(p0 + l) * m + i] : 0.0;
  }
  if (t < PW * PW) Ts[t / PW][t % PW] = 0.0;
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    const int c = p0 + j;
    // |x below the diagonal|^2 and the diagonal entry
    double ss[1] = {0.0};
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const int i = p0 + t + 1024 * r;
#pragma unroll
      for (int l = 0; l < PWT; ++l)
        if (l == j) {
          if (i > c && i < m) ss[0] += x[r][l] * x[r][l];
          if (i == c) x0s = x[r][l];
        }
    }
    block_sum<1>(ss, red, dots);
    const double sq = dots[0], x0 = x0s;
    double tau = 0.0, beta = x0, scale = 0.0;
    if (sq > 0.0) {
      beta = -copysign(sqrt(x0 * x0 + sq), x0);
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    // v (v_c = 1 implicit) into column j; R entry on the diagonal
    double vi[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const int i = p0 + t + 1024 * r;
#pragma unroll
      for (int l = 0; l < PWT; ++l)
        if (l == j) {
          if (i > c && i < m) x[r][l] *= scale;
          if (i == c) x[r][l] = beta;
          vi[r] = (i == c) ? 1.0 : ((i > c && i < m) ? x[r][l] : 0.0);
        }
    }
    // d_l = v . x_l for the panel columns (l > j: to update; l < j: v_l . v_j
    // for T), reduced one column at a time (one live partial per thread)
    {
      const int ln = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
      for (int l = 0; l < PWT; ++l) {
        double a = 0.0;
#pragma unroll
        for (int r = 0; r < RM; ++r) {
          const int i = p0 + t + 1024 * r;
          // column l < j holds v_l below its diagonal p0 + l (< c): rows >= c carry v_l values
          a += vi[r] * ((l < j) ? ((i == p0 + l) ? 1.0 : x[r][l]) : x[r][l]);
        }
        for (int o = 32; o > 0; o >>= 1) a += __shfl_xor(a, o);
        if (ln == 0) red[wv * PWT + l] = a;
      }
      __syncthreads();
      if (t < PWT) {
        double a = 0.0;
        for (int q = 0; q < 16; ++q) a += red[q * PWT + t];
        dots[t] = a;
      }
      __syncthreads();
    }
    // apply H_j to the remaining panel columns
#pragma unroll
    for (int l = 0; l < PWT; ++l)
      if (l > j) {
        const double f = tau * dots[l];
#pragma unroll
        for (int r = 0; r < RM; ++r) x[r][l] -= f * vi[r];
      }
    // T column j:  T[0:j, j] = -tau T[0:j, 0:j] z,  z_q = v_q . v_j
    if (t < j) {
      double a = 0.0;
      for (int q = t; q < j; ++q) a += Ts[t][q] * dots[q];
      Ts[t][j] = -tau * a;
    }
    if (t == j) Ts[j][j] = tau;
    __syncthreads();
  }
  // write back: Xt rows p0 .. p0 + w - 1, the reflector rows, T
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    const int i = p0 + t + 1024 * r;
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
    for (int i = t; i < p0; i += 1024) Vr[(long)(p0 + l) * m + i] = 0.0;
  if (t < PW * PW) Tp[t] = Ts[t / PW][t % PW];
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
  double* W1 = (double*)(w + L.offW1);
  double* W2 = (double*)(w + L.offW2);
  hipError_t e = hipSuccess;
  // panels: as wide as the rows per thread allow without register spills
  struct Panel {
    int p0, pw, rm;
  };
  std::vector<Panel> pans;
  for (int p0 = 0; p0 < k;) {
    const int rm = (m - p0 + 1023) / 1024;
    const int pw = std::min(rm <= 1 ? 16 : (rm == 2 ? 8 : 4), k - p0);
    pans.push_back({p0, pw, rm});
    p0 += pw;
  }
  for (const Panel& P : pans) {
    if (e != hipSuccess) break;
    const int p0 = P.p0, pw = P.pw, rows = m - p0;
    dim3 g(batch), blk(1024);
    if (P.rm <= 1)
      hipLaunchKernelGGL((qr_panel_kernel<1, 16>), g, blk, 0, s, Xt, Vr, T, m, k, L.sX, L.sT, p0);
    else if (P.rm == 2)
      hipLaunchKernelGGL((qr_panel_kernel<2, 8>), g, blk, 0, s, Xt, Vr, T, m, k, L.sX, L.sT, p0);
    else if (P.rm == 3)
      hipLaunchKernelGGL((qr_panel_kernel<3, 4>), g, blk, 0, s, Xt, Vr, T, m, k, L.sX, L.sT, p0);
    else
      hipLaunchKernelGGL((qr_panel_kernel<4, 4>), g, blk, 0, s, Xt, Vr, T, m, k, L.sX, L.sT, p0);
    e = hipGetLastError();
    const int nt = k - p0 - pw;   // trailing columns of X = rows of Xt
    if (nt <= 0 || e != hipSuccess) continue;
    double* Xtr = Xt + (long)(p0 + pw) * m + p0;     // Xt_trail: nt x rows, ld m
    const double* V = Vr + (long)p0 * m + p0;        // V^T: pw x rows, ld m
    const double* Tp = T + (long)(p0 / TSLOT) * PW * PW;
    // W1 = Xt_trail V  (nt x pw)
    e = gemm_f64(s, false, true, nt, pw, rows, 1.0, Xtr, m, L.sX, V, m, L.sX, 0.0, W1, pw, (long)k * PW, batch);
    // W2 = W1 T
    if (e == hipSuccess)
      e = gemm_f64(s, false, false, nt, pw, pw, 1.0, W1, pw, (long)k * PW, Tp, PW, L.sT, 0.0, W2, pw, (long)k * PW,
                   batch);
    // Xt_trail -= W2 V^T
    if (e == hipSuccess)
      e = gemm_f64(s, false, false, nt, rows, pw, -1.0, W2, pw, (long)k * PW, V, m, L.sX, 1.0, Xtr, m, L.sX, batch);
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
    double* Qs = Qt + (long)p0 * m + p0;             // Qt rows p0.., columns p0..
    const double* V = Vr + (long)p0 * m + p0;
    const double* Tp = T + (long)(p0 / TSLOT) * PW * PW;
    // W1 = Qt_sub V (nt x pw);  W2 = W1 T^T;  Qt_sub -= W2 V^T
    e = gemm_f64(s, false, true, nt, pw, rows, 1.0, Qs, m, L.sX, V, m, L.sX, 0.0, W1, pw, (long)k * PW, batch);
    if (e == hipSuccess)
      e = gemm_f64(s, false, true, nt, pw, pw, 1.0, W1, pw, (long)k * PW, Tp, PW, L.sT, 0.0, W2, pw, (long)k * PW,
                   batch);
    if (e == hipSuccess)
      e = gemm_f64(s, false, false, nt, rows, pw, -1.0, W2, pw, (long)k * PW, V, m, L.sX, 1.0, Qs, m, L.sX, batch);
  }
  return e;
}

}  // namespace sctm
