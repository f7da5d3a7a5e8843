// Small FP64 kernels of the reverse pass: projector / SVD adjoint pieces and
// the bond-energy adjoint.  All deterministic (no atomics).
#include "adj_kernels.hpp"

namespace sctm {

static inline int gfor(long n) {
  long g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 65535 * 4) g = 65535 * 4;
  return (int)g;
}

__global__ void add_cast_kernel(const void* src, bool sf, void* dst, bool df, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double v = sf ? ((const double*)src)[i] : (double)((const float*)src)[i];
    if (df)
      ((double*)dst)[i] += v;
    else
      ((float*)dst)[i] += (float)v;
  }
}
hipError_t add_cast(hipStream_t s, const void* src, bool sf, void* dst, bool df, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(add_cast_kernel, dim3(gfor(n)), dim3(256), 0, s, src, sf, dst, df, n);
  return hipGetLastError();
}

__global__ void rank_count_kernel(int n, const double* S, double rel, int* out) {
  __shared__ int wc[4];
  int local = 0;
  double thr = rel * S[0];
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (S[i] > thr && S[0] > 0.0) ++local;
  for (int w = 32; w > 0; w >>= 1) local += __shfl_xor(local, w);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = wc[0] + wc[1] + wc[2] + wc[3];
}
hipError_t rank_count(hipStream_t s, int n, const double* S, double rel, int* out) {
  hipLaunchKernelGGL(rank_count_kernel, dim3(1), dim3(256), 0, s, n, S, rel, out);
  return hipGetLastError();
}

__global__ void scale_cols_from_kernel(const void* src, bool sf, double* dst, int na, int chi, const double* sgn) {
  long n = (long)na * chi;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double v = sf ? ((const double*)src)[i] : (double)((const float*)src)[i];
    dst[i] = v * sgn[i % chi];
  }
}
hipError_t scale_cols_from(hipStream_t s, const void* src, bool sf, double* dst, int na, int chi, const double* sgn) {
  hipLaunchKernelGGL(scale_cols_from_kernel, dim3(gfor((long)na * chi)), dim3(256), 0, s, src, sf, dst, na, chi, sgn);
  return hipGetLastError();
}

// one block per column c < chi
__global__ void svd_adj_prep_kernel(int nb, int chi, const double* U, const double* V, const double* S, const int* kr,
                                    const double* Xb, const double* Yb, double* Ub, double* Vb, double* Sb) {
  const int c = blockIdx.x;
  const int k = kr[0];
  __shared__ double red[256];
  double acc = 0.0;
  const bool keep = c < k;
  const double sc = keep ? S[c] : 1.0;
  const double f = keep ? 1.0 / sqrt(sc) : 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    double xb = Xb[(long)b * chi + c], yb = Yb[(long)b * chi + c];
    Ub[(long)b * chi + c] = xb * f;
    Vb[(long)b * chi + c] = yb * f;
    if (keep) acc += U[(long)b * nb + c] * xb + V[(long)b * nb + c] * yb;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) Sb[c] = keep ? -0.5 * red[0] / (sc * sqrt(sc)) : 0.0;
}
hipError_t svd_adj_prep(hipStream_t s, int nb, int chi, const double* U, const double* V, const double* S,
                        const int* kr, const double* Xb, const double* Yb, double* Ub, double* Vb, double* Sb) {
  hipLaunchKernelGGL(svd_adj_prep_kernel, dim3(chi), dim3(256), 0, s, nb, chi, U, V, S, kr, Xb, Yb, Ub, Vb, Sb);
  return hipGetLastError();
}

__global__ void scale_cols_rsqrt_s_kernel(int nb, int chi, const double* X, const double* S, const int* kr,
                                          double* out) {
  const int k = kr[0];
  long n = (long)nb * chi;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % chi);
    out[i] = c < k ? X[i] / sqrt(S[c]) : 0.0;
  }
}
hipError_t scale_cols_rsqrt_s(hipStream_t s, int nb, int chi, const double* X, const double* S, const int* kr,
                              double* out) {
  hipLaunchKernelGGL(scale_cols_rsqrt_s_kernel, dim3(gfor((long)nb * chi)), dim3(256), 0, s, nb, chi, X, S, kr, out);
  return hipGetLastError();
}

__global__ void zero_rows_kernel(int nb, int chi, double* GU, double* GV, const int* r) {
  const int rr = *r;
  long n = (long)nb * chi;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    if (i / chi >= rr) {
      GU[i] = 0.0;
      GV[i] = 0.0;
    }
}
hipError_t zero_rows_from(hipStream_t s, int nb, int chi, double* GU, double* GV, const int* r) {
  hipLaunchKernelGGL(zero_rows_kernel, dim3(gfor((long)nb * chi)), dim3(256), 0, s, nb, chi, GU, GV, r);
  return hipGetLastError();
}

// F_ij = d / (d^2 + (eps (s_i^2 + s_j^2))^2), d = s_j^2 - s_i^2: the
// Lorentzian acts only on pairs whose gap is below eps of their own scale,
// so small but well-separated singular values keep the exact 1 / d
__device__ inline double inner_val(int i, int j, int nb, int chi, int r, const double* S, const double* Sb,
                                   const double* GU, const double* GV, double eps) {
  if (i >= r || j >= r) return 0.0;
  if (i == j) return (i < chi) ? Sb[i] : 0.0;
  double si = S[i], sj = S[j];
  double d = sj * sj - si * si;
  double e = eps * (si * si + sj * sj);
  double F = d / (d * d + e * e);
  double gu = (j < chi ? GU[(long)i * chi + j] : 0.0) - (i < chi ? GU[(long)j * chi + i] : 0.0);
  double gv = (j < chi ? GV[(long)i * chi + j] : 0.0) - (i < chi ? GV[(long)j * chi + i] : 0.0);
  return F * (gu * sj + si * gv);
}

__global__ void svd_adj_inner_kernel(int nb, int c2, int chi, const double* S, const double* Sb, const double* GU,
                                     const double* GV, const int* kr, double eps, double* Itop, double* Ileft) {
  const int r = kr[1];
  long ntop = (long)c2 * nb, nleft = (long)(nb - c2) * c2;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < ntop + nleft; t += (long)gridDim.x * blockDim.x) {
    if (t < ntop) {
      int i = (int)(t / nb), j = (int)(t % nb);
      Itop[t] = inner_val(i, j, nb, chi, r, S, Sb, GU, GV, eps);
    } else {
      long u = t - ntop;
      int i = c2 + (int)(u / c2), j = (int)(u % c2);
      Ileft[u] = inner_val(i, j, nb, chi, r, S, Sb, GU, GV, eps);
    }
  }
}
hipError_t svd_adj_inner(hipStream_t s, int nb, int c2, int chi, const double* S, const double* Sb, const double* GU,
                         const double* GV, const int* kr, double eps, double* Itop, double* Ileft) {
  long n = (long)c2 * nb + (long)(nb - c2) * c2;
  hipLaunchKernelGGL(svd_adj_inner_kernel, dim3(gfor(n)), dim3(256), 0, s, nb, c2, chi, S, Sb, GU, GV, kr, eps, Itop,
                     Ileft);
  return hipGetLastError();
}

__global__ void scale_cols_inv_s_kernel(int nb, int chi, double* C1, double* C2, const double* S, const int* kr) {
  const int k = kr[0];
  long n = (long)nb * chi;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    int c = (int)(i % chi);
    double f = c < k ? 1.0 / S[c] : 0.0;
    C1[i] *= f;
    C2[i] *= f;
  }
}
hipError_t scale_cols_inv_s(hipStream_t s, int nb, int chi, double* C1, double* C2, const double* S, const int* kr) {
  hipLaunchKernelGGL(scale_cols_inv_s_kernel, dim3(gfor((long)nb * chi)), dim3(256), 0, s, nb, chi, C1, C2, S, kr);
  return hipGetLastError();
}

__global__ void add_transposed_kernel(int nb, int chi, int c2, const double* C2, double* Q1) {
  long n = (long)c2 * nb;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    int c = (int)(t / nb), b = (int)(t % nb);
    Q1[t] += C2[(long)b * chi + c];
  }
}
hipError_t add_transposed(hipStream_t s, int nb, int chi, int c2, const double* C2, double* Q1) {
  hipLaunchKernelGGL(add_transposed_kernel, dim3(gfor((long)c2 * nb)), dim3(256), 0, s, nb, chi, c2, C2, Q1);
  return hipGetLastError();
}

__global__ void copy_cols_kernel(int nb, int chi, int c2, const double* C1, double* Q2) {
  long n = (long)nb * c2;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    int b = (int)(t / c2), c = (int)(t % c2);
    Q2[t] = C1[(long)b * chi + c];
  }
}
hipError_t copy_cols(hipStream_t s, int nb, int chi, int c2, const double* C1, double* Q2) {
  hipLaunchKernelGGL(copy_cols_kernel, dim3(gfor((long)nb * c2)), dim3(256), 0, s, nb, chi, c2, C1, Q2);
  return hipGetLastError();
}

__global__ void bond_energy_adjoint_kernel(int p, const double* h, const double* e, const double* eb, double* rb) {
  const int p2 = p * p;
  const long n = (long)p2 * p2;
  const double ev = e[0], den = e[1], g = eb[0];
  for (long t = threadIdx.x; t < n; t += blockDim.x) {
    int PQ = (int)(t / p2), RS = (int)(t % p2);   // rho[P,Q,R,S] flat = PQ * p2 + RS
    double delta = (PQ == RS) ? 1.0 : 0.0;
    rb[t] += g * (h[(long)RS * p2 + PQ] - ev * delta) / den;
  }
}
hipError_t bond_energy_adjoint(hipStream_t s, int p, const double* h, const double* e, const double* ebar,
                               double* rhobar) {
  hipLaunchKernelGGL(bond_energy_adjoint_kernel, dim3(1), dim3(256), 0, s, p, h, e, ebar, rhobar);
  return hipGetLastError();
}

}  // namespace sctm
