// Bandwidth-bound helper kernels: index permutation, casts, fills, axpy,
// deterministic two-pass FP64 reductions (no atomics: fixed grid, fixed
// per-block order, one final block), normalisation and its adjoint,
// projector truncation / sign fix, and the bond-energy ratio.
#include "kernels.hpp"

#include <cstdint>

namespace sctm {

static constexpr int RED_BLOCKS = 1024;
int reduce_partials() { return RED_BLOCKS; }

static inline int grid_for(long n, int per = 256, int cap = 65535 * 4) {
  long g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

// ---------------------------------------------------------------------------
// Index permutation.  Below 2^31 elements all index arithmetic is 32-bit,
// with the per-axis divisions replaced by multiply-high division by invariant
// integers (Granlund and Montgomery, 1994): for d >= 1, l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, and n / d = (t + ((n - t) >> min(l, 1)))
// >> max(l - 1, 0) with t = umulhi(m, n), exact for every 32-bit n.
struct FastDiv {
  unsigned d, m, s1, s2;
};

static FastDiv make_fastdiv(unsigned d) {
  unsigned l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  FastDiv f;
  f.d = d;
  f.m = (unsigned)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
  f.s1 = l < 1 ? l : 1;
  f.s2 = l > 1 ? l - 1 : 0;
  return f;
}

__device__ __forceinline__ unsigned fast_div(unsigned n, const FastDiv& f) {
  const unsigned t = __umulhi(f.m, n);
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

struct PermGeneric {
  int rank;
  FastDiv dv[12];         // output dimensions
  unsigned istr[12];      // input stride of each output axis
};

// any permutation, one output element per thread (writes coalesced)
template <typename T>
__global__ void permute32_kernel(const T* __restrict__ in, T* __restrict__ out, PermGeneric d, unsigned n, bool acc) {
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    unsigned rem = i, off = 0;
    for (int ax = d.rank - 1; ax >= 0; --ax) {
      const unsigned q = fast_div(rem, d.dv[ax]);
      off += (rem - q * d.dv[ax].d) * d.istr[ax];
      rem = q;
    }
    out[i] = acc ? out[i] + in[off] : in[off];
  }
}

struct PermTiled {
  unsigned DX, DY;        // output axis X (last, output stride 1) and axis Y (input stride 1)
  unsigned sx, oy;        // input stride of X, output stride of Y
  int nrest;              // the other axes
  unsigned nr;            // product of their dimensions
  FastDiv rdv[12];
  unsigned rin[12], rout[12];
};

// permutation whose innermost input and output axes differ: 32 x 32 tiles
// of (X, Y) through LDS, read along Y (input-contiguous) and written along X
// (output-contiguous); grid z runs over the other axes.
template <typename T>
__global__ void permute_tiled_kernel(const T* __restrict__ in, T* __restrict__ out, PermTiled d, bool acc) {
  __shared__ T tile[32][33];
  const unsigned x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
  for (unsigned z = blockIdx.z; z < d.nr; z += gridDim.z) {
    unsigned rem = z, bin = 0, bout = 0;
    for (int ax = d.nrest - 1; ax >= 0; --ax) {
      const unsigned q = fast_div(rem, d.rdv[ax]);
      const unsigned c = rem - q * d.rdv[ax].d;
      bin += c * d.rin[ax];
      bout += c * d.rout[ax];
      rem = q;
    }
    for (int j = ty; j < 32; j += 8) {
      const unsigned x = x0 + j, y = y0 + tx;
      if (x < d.DX && y < d.DY) tile[j][tx] = in[bin + x * d.sx + y];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
      const unsigned y = y0 + j, x = x0 + tx;
      if (x < d.DX && y < d.DY) {
        const unsigned o = bout + y * d.oy + x;
        out[o] = acc ? out[o] + tile[tx][j] : tile[tx][j];
      }
    }
    __syncthreads();
  }
}

// 64-bit fallback for tensors of 2^31 elements or more
template <typename T>
__global__ void permute_kernel(const T* __restrict__ in, T* __restrict__ out, PermDesc d, long n,
                               bool acc) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    long rem = i, off = 0;
    for (int ax = d.rank - 1; ax >= 0; --ax) {
      long c = rem % d.out_dims[ax];
      rem /= d.out_dims[ax];
      off += c * d.in_strides_perm[ax];
    }
    out[i] = acc ? out[i] + in[off] : in[off];
  }
}

// 2-D transpose through LDS for the common case: out[b][c][a] = in[b][a][c]
// with the two innermost axes swapped (a x c tiles of 32 x 32).
template <typename T>
__global__ void transpose_kernel(const T* __restrict__ in, T* __restrict__ out, long A, long Cn, bool acc) {
  __shared__ T tile[32][33];
  const long b = blockIdx.z;
  in += b * A * Cn;
  out += b * A * Cn;
  long a0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    long a = a0 + j, c = c0 + tx;
    if (a < A && c < Cn) tile[j][tx] = in[a * Cn + c];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    long c = c0 + j, a = a0 + tx;
    if (a < A && c < Cn) {
      long o = c * A + a;
      out[o] = acc ? out[o] + tile[tx][j] : tile[tx][j];
    }
  }
}

// The permutation with the innermost output axis (innermost in the input
// too) grouped into vectors V of VW elements; false (nothing launched) when
// the run length, another input stride or the alignment does not allow it.
template <typename V, int VW>
static bool permute_vec(hipStream_t s, const void* in, void* out, const PermDesc& d, long n, bool acc) {
  if (d.out_dims[d.rank - 1] % VW != 0 || ((uintptr_t)in | (uintptr_t)out) % sizeof(V) != 0) return false;
  for (int i = 0; i + 1 < d.rank; ++i)
    if (d.out_dims[i] > 1 && d.in_strides_perm[i] % VW != 0) return false;
  PermGeneric gv;
  gv.rank = d.rank;
  for (int i = 0; i < d.rank; ++i) {
    const bool inner = i == d.rank - 1;
    gv.dv[i] = make_fastdiv((unsigned)(inner ? d.out_dims[i] / VW : d.out_dims[i]));
    gv.istr[i] = inner ? 1u : (unsigned)(d.in_strides_perm[i] / VW);
  }
  const long nv = n / VW;
  hipLaunchKernelGGL(permute32_kernel<V>, dim3(grid_for(nv)), dim3(256), 0, s, (const V*)in, (V*)out, gv,
                     (unsigned)nv, acc);
  return true;
}

template <typename T>
static void launch_permute32(hipStream_t s, const void* in, void* out, const PermDesc& d, long n, bool acc) {
  // output strides (row-major over out_dims)
  long ost[12];
  ost[d.rank - 1] = 1;
  for (int i = d.rank - 2; i >= 0; --i) ost[i] = ost[i + 1] * d.out_dims[i + 1];
  int yax = -1;
  for (int i = 0; i < d.rank; ++i)
    if (d.in_strides_perm[i] == 1) yax = i;
  // tiles only pay when both axes fill them
  if (yax >= 0 && yax != d.rank - 1 && d.out_dims[d.rank - 1] >= 32 && d.out_dims[yax] >= 32) {
    PermTiled t;
    t.DX = (unsigned)d.out_dims[d.rank - 1];
    t.DY = (unsigned)d.out_dims[yax];
    t.sx = (unsigned)d.in_strides_perm[d.rank - 1];
    t.oy = (unsigned)ost[yax];
    t.nrest = 0;
    t.nr = 1;
    for (int i = 0; i < d.rank - 1; ++i) {
      if (i == yax) continue;
      t.rdv[t.nrest] = make_fastdiv((unsigned)d.out_dims[i]);
      t.rin[t.nrest] = (unsigned)d.in_strides_perm[i];
      t.rout[t.nrest] = (unsigned)ost[i];
      t.nr *= (unsigned)d.out_dims[i];
      ++t.nrest;
    }
    dim3 g((t.DX + 31) / 32, (t.DY + 31) / 32, t.nr < 65535u ? t.nr : 65535u);
    hipLaunchKernelGGL(permute_tiled_kernel<T>, g, dim3(32, 8), 0, s, (const T*)in, (T*)out, t, acc);
    return;
  }
  // innermost output axis also innermost in the input (contiguous runs of
  // its length in both): the runs move as 16-byte (else 8-byte) vectors,
  // every other input stride being a multiple of the vector width
  if (yax == d.rank - 1 && d.rank > 1) {
    if (sizeof(T) == 4 && permute_vec<float4, 4>(s, in, out, d, n, acc)) return;
    if (sizeof(T) == 4 && permute_vec<float2, 2>(s, in, out, d, n, acc)) return;
    if (sizeof(T) == 8 && permute_vec<double2, 2>(s, in, out, d, n, acc)) return;
  }
  PermGeneric gd;
  gd.rank = d.rank;
  for (int i = 0; i < d.rank; ++i) {
    gd.dv[i] = make_fastdiv((unsigned)d.out_dims[i]);
    gd.istr[i] = (unsigned)d.in_strides_perm[i];
  }
  hipLaunchKernelGGL(permute32_kernel<T>, dim3(grid_for(n)), dim3(256), 0, s, (const T*)in, (T*)out, gd,
                     (unsigned)n, acc);
}

hipError_t permute(hipStream_t s, int esize, const void* in, void* out, const PermDesc& d, long n,
                   bool accumulate) {
  if (n <= 0) return hipSuccess;
  // detect "swap the two innermost groups": out axes = [lead..., x, y] with
  // in order [lead..., y, x] and contiguous groups -> LDS-tiled transpose.
  if (d.rank >= 2) {
    long inner_out = d.out_dims[d.rank - 1];
    long mid_out = d.out_dims[d.rank - 2];
    bool lead_ok = true;
    long lead = 1;
    for (int i = 0; i < d.rank - 2; ++i) lead *= d.out_dims[i];
    // expected input strides for out axis rank-1 (size inner_out) -> mid_out,
    // out axis rank-2 (size mid_out) -> 1, leading axes contiguous blocks
    if (d.in_strides_perm[d.rank - 1] == mid_out && d.in_strides_perm[d.rank - 2] == 1) {
      long st = mid_out * inner_out;
      for (int i = d.rank - 3; i >= 0; --i) {
        if (d.in_strides_perm[i] != st) { lead_ok = false; break; }
        st *= d.out_dims[i];
      }
      if (lead_ok && lead <= 65535) {
        dim3 g((unsigned)((mid_out + 31) / 32), (unsigned)((inner_out + 31) / 32), (unsigned)lead);
        // input viewed as [lead][inner_out][mid_out] -> output [lead][mid_out][inner_out]
        if (esize == 8)
          hipLaunchKernelGGL(transpose_kernel<double>, g, dim3(32, 8), 0, s, (const double*)in,
                             (double*)out, inner_out, mid_out, accumulate);
        else
          hipLaunchKernelGGL(transpose_kernel<float>, g, dim3(32, 8), 0, s, (const float*)in,
                             (float*)out, inner_out, mid_out, accumulate);
        return hipGetLastError();
      }
    }
  }
  if (n < (1L << 31) && d.rank <= 12) {
    if (esize == 8)
      launch_permute32<double>(s, in, out, d, n, accumulate);
    else
      launch_permute32<float>(s, in, out, d, n, accumulate);
    return hipGetLastError();
  }
  int g = grid_for(n);
  if (esize == 8)
    hipLaunchKernelGGL(permute_kernel<double>, dim3(g), dim3(256), 0, s, (const double*)in, (double*)out, d, n, accumulate);
  else
    hipLaunchKernelGGL(permute_kernel<float>, dim3(g), dim3(256), 0, s, (const float*)in, (float*)out, d, n, accumulate);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void fill_kernel(T* p, T v, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
hipError_t fill_f64(hipStream_t s, double* p, double v, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t fill_f32(hipStream_t s, float* p, float v, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

template <typename I, typename O>
__global__ void cast_kernel(const I* in, O* out, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) out[i] = (O)in[i];
}
hipError_t cast_f32_to_f64(hipStream_t s, const float* in, double* out, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((cast_kernel<float, double>), dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t cast_f64_to_f32(hipStream_t s, const double* in, float* out, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((cast_kernel<double, float>), dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

template <typename T>
__global__ void axpy_kernel(T a, const T* x, T* y, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] += a * x[i];
}
hipError_t axpy_f64(hipStream_t s, double a, const double* x, double* y, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, a, x, y, n);
  return hipGetLastError();
}
hipError_t axpy_f32(hipStream_t s, float a, const float* x, float* y, long n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, a, x, y, n);
  return hipGetLastError();
}

// split-K epilogue: C[m][n] = alpha sum_s P[s][m][n] + beta C[m][n], the
// slices added in order (P: S consecutive M x N blocks, C: leading dim ldc)
template <typename T>
__global__ void splitk_reduce_kernel(const T* P, int S, int M, int N, T alpha, T beta, T* C, long ldc) {
  const long mn = (long)M * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < mn; e += (long)gridDim.x * blockDim.x) {
    const long o = (e / N) * ldc + e % N;
    const T c = (beta == T(0)) ? T(0) : C[o];
    // slices added in order; eight loads in flight at a time
    T a = 0;
    for (int k0 = 0; k0 < S; k0 += 8) {
      T v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = P[(long)min(k0 + q, S - 1) * mn + e];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + q < S) a += v[q];
    }
    C[o] = (beta == T(0)) ? alpha * a : alpha * a + beta * c;
  }
}
hipError_t splitk_reduce_f64(hipStream_t s, const double* P, int S, int M, int N, double alpha, double beta, double* C,
                             long ldc) {
  const long n = (long)M * N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(splitk_reduce_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, P, S, M, N, alpha, beta, C, ldc);
  return hipGetLastError();
}
hipError_t splitk_reduce_f32(hipStream_t s, const float* P, int S, int M, int N, float alpha, float beta, float* C,
                             long ldc) {
  const long n = (long)M * N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, P, S, M, N, alpha, beta, C, ldc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reductions: pass 1 writes RED_BLOCKS partials, pass 2 sums them in order.
// ---------------------------------------------------------------------------
__device__ inline double block_sum(double v) {
  __shared__ double sh[256];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

template <typename T>
__global__ void sumsq_pass1(const T* x, long n, double* partial) {
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double v = (double)x[i];
    acc += v * v;
  }
  double r = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}
template <typename T>
__global__ void dot_pass1(const T* x, const T* y, long n, double* partial) {
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc += (double)x[i] * (double)y[i];
  double r = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}
__global__ void sum_pass2(const double* partial, int np, double* out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[i];
  double r = block_sum(acc);
  if (threadIdx.x == 0) *out = r;
}

hipError_t sumsq_f64(hipStream_t s, const double* x, long n, double* partial, double* out) {
  hipLaunchKernelGGL(sumsq_pass1<double>, dim3(RED_BLOCKS), dim3(256), 0, s, x, n, partial);
  hipLaunchKernelGGL(sum_pass2, dim3(1), dim3(256), 0, s, partial, RED_BLOCKS, out);
  return hipGetLastError();
}
hipError_t sumsq_f32(hipStream_t s, const float* x, long n, double* partial, double* out) {
  hipLaunchKernelGGL(sumsq_pass1<float>, dim3(RED_BLOCKS), dim3(256), 0, s, x, n, partial);
  hipLaunchKernelGGL(sum_pass2, dim3(1), dim3(256), 0, s, partial, RED_BLOCKS, out);
  return hipGetLastError();
}
hipError_t dot_f64(hipStream_t s, const double* x, const double* y, long n, double* partial, double* out) {
  hipLaunchKernelGGL(dot_pass1<double>, dim3(RED_BLOCKS), dim3(256), 0, s, x, y, n, partial);
  hipLaunchKernelGGL(sum_pass2, dim3(1), dim3(256), 0, s, partial, RED_BLOCKS, out);
  return hipGetLastError();
}
hipError_t dot_f32(hipStream_t s, const float* x, const float* y, long n, double* partial, double* out) {
  hipLaunchKernelGGL(dot_pass1<float>, dim3(RED_BLOCKS), dim3(256), 0, s, x, y, n, partial);
  hipLaunchKernelGGL(sum_pass2, dim3(1), dim3(256), 0, s, partial, RED_BLOCKS, out);
  return hipGetLastError();
}

template <typename T>
__global__ void scale_rsqrt_kernel(const T* x, T* y, const double* nrm2, long n) {
  double f = 1.0 / sqrt(*nrm2);
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (T)((double)x[i] * f);
}
hipError_t scale_by_rsqrt_f64(hipStream_t s, const double* x, double* y, const double* nrm2, long n) {
  hipLaunchKernelGGL(scale_rsqrt_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, x, y, nrm2, n);
  return hipGetLastError();
}
hipError_t scale_by_rsqrt_f32(hipStream_t s, const float* x, float* y, const double* nrm2, long n) {
  hipLaunchKernelGGL(scale_rsqrt_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, x, y, nrm2, n);
  return hipGetLastError();
}

template <typename T>
__global__ void norm_adj_kernel(const T* y, const T* ybar, const double* nrm2, const double* ydot, T* xbar, long n) {
  double inv = 1.0 / sqrt(*nrm2), d = *ydot;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    xbar[i] += (T)(((double)ybar[i] - (double)y[i] * d) * inv);
}
hipError_t normalize_adjoint_f64(hipStream_t s, const double* y, const double* ybar, const double* nrm2,
                                 const double* ydot, double* xbar, long n) {
  hipLaunchKernelGGL(norm_adj_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, y, ybar, nrm2, ydot, xbar, n);
  return hipGetLastError();
}
hipError_t normalize_adjoint_f32(hipStream_t s, const float* y, const float* ybar, const double* nrm2,
                                 const double* ydot, float* xbar, long n) {
  hipLaunchKernelGGL(norm_adj_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, y, ybar, nrm2, ydot, xbar, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// projector truncation: X[b, c] = U[b, c] / sqrt(S[c]) for c < k, else 0
// ---------------------------------------------------------------------------
__global__ void trunc_count_kernel(int n, int chi, const double* S, double cutoff, int* kout) {
  // one block per batch entry; count of singular values above cutoff * s_1
  const double* s = S + (long)blockIdx.x * n;
  __shared__ int wc[16];
  double thr = cutoff * s[0];
  int local = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (s[i] > thr && s[0] > 0.0) ++local;
  for (int w = 32; w > 0; w >>= 1) local += __shfl_xor(local, w);
  if ((threadIdx.x & 63) == 0) wc[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) c += wc[w];
    kout[blockIdx.x] = c < chi ? c : chi;
  }
}

__global__ void trunc_scale_kernel(int nb, int n, int chi, const double* U, const double* S, const int* kin,
                                   double* X) {
  const int b = blockIdx.y;
  U += (long)b * nb * n;
  S += (long)b * n;
  X += (long)b * nb * chi;
  const int k = kin[b];
  long tot = (long)nb * chi;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < tot; i += (long)gridDim.x * blockDim.x) {
    int r = (int)(i / chi), c = (int)(i % chi);
    X[i] = (c < k) ? U[(long)r * n + c] / sqrt(S[c]) : 0.0;
  }
}

hipError_t trunc_scale(hipStream_t s, int nb, int n, int chi, const double* U, const double* S, double cutoff,
                       double* X, int* kout, int batch) {
  hipLaunchKernelGGL(trunc_count_kernel, dim3(batch), dim3(256), 0, s, n, chi, S, cutoff, kout);
  long tot = (long)nb * chi;
  hipLaunchKernelGGL(trunc_scale_kernel, dim3(grid_for(tot), batch), dim3(256), 0, s, nb, n, chi, U, S, kout, X);
  return hipGetLastError();
}

// one block per (column, batch): argmax |PT[:, c]| (lowest row on ties)
__global__ void sign_fix_kernel(int na, int chi, double* PT, double* PB, double* sgn) {
  const int c = blockIdx.x, b = blockIdx.y;
  PT += (long)b * na * chi;
  PB += (long)b * na * chi;
  __shared__ double bv[256];
  __shared__ int bi[256];
  double best = -1.0;
  int bidx = 0x7fffffff;
  for (int r = threadIdx.x; r < na; r += blockDim.x) {
    double v = fabs(PT[(long)r * chi + c]);
    if (v > best || (v == best && r < bidx)) { best = v; bidx = r; }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      double o = bv[threadIdx.x + w];
      int oi = bi[threadIdx.x + w];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  double f = 1.0;
  if (bi[0] < na && PT[(long)bi[0] * chi + c] < 0.0) f = -1.0;
  __syncthreads();
  if (f < 0.0)
    for (int r = threadIdx.x; r < na; r += blockDim.x) {
      PT[(long)r * chi + c] = -PT[(long)r * chi + c];
      PB[(long)r * chi + c] = -PB[(long)r * chi + c];
    }
  if (threadIdx.x == 0 && sgn) sgn[(long)b * chi + c] = f;
}

hipError_t sign_fix(hipStream_t s, int na, int chi, double* PT, double* PB, double* sgn_out, int batch) {
  hipLaunchKernelGGL(sign_fix_kernel, dim3(chi, batch), dim3(256), 0, s, na, chi, PT, PB, sgn_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void bond_energy_kernel(int p, const double* rho, const double* h, double* e) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int p2 = p * p;
  double num = 0.0, den = 0.0;
  for (int P = 0; P < p; ++P)
    for (int Q = 0; Q < p; ++Q) {
      den += rho[(((long)P * p + Q) * p + P) * p + Q];
      for (int R = 0; R < p; ++R)
        for (int S = 0; S < p; ++S)
          num += rho[(((long)P * p + Q) * p + R) * p + S] * h[(long)(R * p + S) * p2 + (P * p + Q)];
    }
  e[0] = num / den;
  e[1] = den;
}
hipError_t bond_energy(hipStream_t s, int p, const double* rho, const double* h, double* e_out) {
  hipLaunchKernelGGL(bond_energy_kernel, dim3(1), dim3(64), 0, s, p, rho, h, e_out);
  return hipGetLastError();
}

// energy per site: the mean over the unit cell's 2 Lx Ly bond energies (each
// site owns its right and its lower bond), summed in bond order on one lane
__global__ void site_energy_kernel(int nb, const double* eb, double w, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = 0.0;
  for (int i = 0; i < nb; ++i) t += eb[i];
  out[0] = w * t;
}
hipError_t site_energy(hipStream_t s, int nb, const double* eb, double w, double* out) {
  hipLaunchKernelGGL(site_energy_kernel, dim3(1), dim3(64), 0, s, nb, eb, w, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// corner-spectrum convergence measure: max_k |S_k - prev_k|_2, then prev = S
// ---------------------------------------------------------------------------
__global__ void spectra_delta_kernel(int nc, int ch, const double* S, double* prev, double* out, int have) {
  // NaN-propagating max (fmax would drop a NaN and report convergence)
  __shared__ double red[256];
  double m = 0.0;
  for (int k = threadIdx.x; k < nc; k += blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < ch; ++i) {
      double sv = S[(long)k * ch + i];
      double d = sv - prev[(long)k * ch + i];
      acc += d * d;
      if (!(sv == sv) || isinf(sv)) acc = NAN;
    }
    double v = sqrt(acc);
    m = (v != v || m != m) ? NAN : fmax(m, v);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      double a = red[threadIdx.x], b = red[threadIdx.x + w];
      red[threadIdx.x] = (a != a || b != b) ? NAN : fmax(a, b);
    }
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  for (long i = threadIdx.x; i < (long)nc * ch; i += blockDim.x) prev[i] = S[i];
  if (threadIdx.x == 0) *out = (r != r) ? r : (have ? r : 1.0e300);
}
hipError_t spectra_delta(hipStream_t s, int nc, int ch, const double* S, double* prev, double* out, int have) {
  hipLaunchKernelGGL(spectra_delta_kernel, dim3(1), dim3(256), 0, s, nc, ch, S, prev, out, have);
  return hipGetLastError();
}

}  // namespace sctm
