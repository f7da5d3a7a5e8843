// Batched FP64 Householder QR of tall matrices X (m x k, m >= k), stored as
// Xt = X^T row-major (row j of Xt = column j of X, contiguous), with the
// explicit thin factor Q (m x k, also stored transposed) and R (k x k).
//
// Two-level blocked right-looking Householder:
//   outer blocks of NBW = 64 columns; inside a block, panels of 16, 8 or 4
//   columns (as many as the rows held per thread allow without register
//   spills):
//   panel:    one workgroup per matrix factors the panel in registers
//             (thread t holds rows p0 + t + NT r), one reflector
//             per column (LAPACK's dlarfg convention: beta = -sign(x0) |x|,
//             tau = (beta - x0) / beta, v = x / (x0 - beta) with v_0 = 1) and
//             builds the triangular factor T of the panel's block reflector
//             H_1 ... H_pw = I - V T V^T (forward, columnwise);
//   in-block: the rest of the outer block <- H^T (rest), one fused kernel;
//   block:    the block's T (64 x 64) from S = V^T V and the taus
//             (T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] S[0:i, i]), and
//             the columns beyond the block <- H^T (columns) on the matrix
//             cores: W = Xt_trail V in K slices, W T from the summed slices,
//             then Xt_trail <- Xt_trail - (W T) V^T;
//   Q:        Q = H_1 ... H_k [I; 0], accumulated backwards over the outer
//             blocks with T^T, by the same two kernels.
// Householder QR is backward stable: Q is orthonormal to working accuracy
// and X = Q R + dX with |dX| ~ eps |X|, whatever the rank of X.
#include "kernels.hpp"

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <utility>
#include <vector>

namespace sctm {

static constexpr int PW = 16;     // widest panel (T blocks are PW x PW)
static constexpr int TSLOT = 4;   // narrowest panel: one T block per TSLOT columns
static constexpr int NBW = 64;    // columns per outer block
static constexpr int QR_SMAX = 8;  // K slices of the W = Y V^T products at most

// f(integral_constant<int, J>) for J = Js... in order
template <typename F, int... Js>
__device__ __forceinline__ void static_for(F& f, std::integer_sequence<int, Js...>) {
  (f(std::integral_constant<int, Js>{}), ...);
}

struct QrLayout {
  long sX, sT, sTB, sW, sP, sTau;
  int nch;
  size_t offV, offT, offTB, offW, offW2, offP, offTau, total;
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
  const int nblk = (k + NBW - 1) / NBW;
  L.sTB = (long)nblk * NBW * NBW;
  L.sW = (long)k * NBW;
  L.nch = (m + 127) / 128;
  L.sP = (long)L.nch * NBW * NBW;
  L.sTau = k;
  L.offV = take(sizeof(double) * L.sX * batch);                // reflectors as rows [k][m]
  L.offT = take(sizeof(double) * L.sT * batch);                // T of every panel
  L.offTB = take(sizeof(double) * L.sTB * batch);              // T of every outer block
  L.offW = take(sizeof(double) * L.sW * QR_SMAX * batch);      // K slices of W = Y V^T of a block update
  L.offW2 = take(sizeof(double) * L.sW * batch);               // W T
  L.offP = take(sizeof(double) * L.sP * batch);                // chunk partials of S or of an in-block W
  L.offTau = take(sizeof(double) * L.sTau * batch);            // tau of every reflector
  L.total = off;
  return L;
}

size_t qr_work_bytes(int m, int k, int batch) { return qr_layout(m, k, batch).total; }

// Factor the panel of columns p0 .. p0 + w - 1 (rows p0 .. m - 1) of every
// matrix; writes the reflectors (below the diagonal) and R (on and above it)
// back into Xt, the reflectors as full rows into Vr (zeros above, 1 on the
// diagonal) and the panel's T.  NT threads, RM rows per thread
// (m - p0 <= NT RM), w <= PWT columns.
//
// One block-wide reduction per column: with v = [1; x_below scale] every dot
// product the step needs follows from the raw sums s_l = sum_{i > c} x_ij x_il
// and the diagonal row c, d_l = x_cl + scale s_l: for l > j the coefficient of
// the update of column l, for l < j the entry v_l . v_j of T's recurrence,
// and s_j = |x_below|^2.  Inside a wavefront the PWT partial sums are
// reduce-scattered by DPP lane exchanges (VALU moves, no LDS), the four 16-lane
// rows are added by the cross-half lane swaps, the wavefront totals meet in
// LDS (one barrier per column) and every wavefront adds them in the same
// order and takes the PWT sums as wavefront-uniform values.
//
// DPP controls (16-lane rows): quad_perm [1,0,3,2] = lane ^ 1, [2,3,0,1] =
// lane ^ 2, row_half_mirror = 7 - lane within eight, row_ror:8 = lane ^ 8,
// row_ror:4 = lane +- 4 within the row.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// lower-half value + upper-half value of the lane pairs (l, l + 32) (HALF =
// 32) or (l, l + 16) within each 32 (HALF = 16); the same sum in both lanes
template <int HALF>
__device__ __forceinline__ double swap_add(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)u, hi = (unsigned)(u >> 32);
  unsigned lo0, lo1, hi0, hi1;
  if constexpr (HALF == 32) {
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    lo0 = a[0], lo1 = a[1], hi0 = b[0], hi1 = b[1];
  } else {
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    lo0 = a[0], lo1 = a[1], hi0 = b[0], hi1 = b[1];
  }
  return __builtin_bit_cast(double, ((unsigned long long)hi0 << 32) | lo0) +
         __builtin_bit_cast(double, ((unsigned long long)hi1 << 32) | lo1);
}

// One reduce-scatter step over N values: a lane with `up` keeps the upper N/2,
// the others the lower N/2, and adds the partner's copy of the half it keeps
// (the partner, selected by CTRL, has the opposite `up` and the same set).
template <int N, int CTRL, int M>
__device__ __forceinline__ void rs_step(double (&v)[M], bool up) {
#pragma unroll
  for (int q = 0; q < N / 2; ++q) {
    const double lo = v[q], hi = v[q + N / 2];
    const double keep = up ? hi : lo, send = up ? lo : hi;
    v[q] = keep + dpp_f64<CTRL>(send);
  }
}

// Wavefront total of v[sel(lane)] for PWT = 16 (sel = 8 b2 + 4 b1 + 2 b0 + b3
// with b the bits of lane % 16) or PWT = 4 (sel = lane % 4); v is consumed.
template <int PWT>
__device__ __forceinline__ int rs_sel(int lane) {
  if constexpr (PWT == 16)
    return 8 * ((lane >> 2) & 1) + 4 * ((lane >> 1) & 1) + 2 * (lane & 1) + ((lane >> 3) & 1);
  else
    return lane & 3;
}
template <int PWT>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[PWT], int lane) {
  if constexpr (PWT == 16) {
    rs_step<16, 0x141>(v, (lane >> 2) & 1);   // partner 7 - lane (bit 2 differs)
    rs_step<8, 0x4E>(v, (lane >> 1) & 1);     // lane ^ 2
    rs_step<4, 0xB1>(v, lane & 1);            // lane ^ 1
    rs_step<2, 0x128>(v, (lane >> 3) & 1);    // lane ^ 8
  } else {
    static_assert(PWT == 4, "panel widths 16 and 4");
    rs_step<4, 0x4E>(v, (lane >> 1) & 1);
    rs_step<2, 0xB1>(v, lane & 1);
    v[0] = v[0] + dpp_f64<0x124>(v[0]);       // the four quads of the row
    v[0] = v[0] + dpp_f64<0x128>(v[0]);
  }
  return swap_add<16>(swap_add<32>(v[0]));
}

template <int NT, int RM, int PWT>
__global__ __launch_bounds__(NT) void qr_panel_kernel(double* Xt_all, double* Vr_all, double* T_all,
                                                      double* tau_all, int m, int k, long sX, long sT, int p0,
                                                      int w) {
  constexpr int NW = NT / 64;   // wavefronts
  const int b = blockIdx.x;
  double* Xt = Xt_all + b * sX;
  double* Vr = Vr_all + b * sX;
  double* Tp = T_all + b * sT + (long)(p0 / TSLOT) * PW * PW;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // wavefront totals and the diagonal row, double-buffered over the columns
  // (one barrier per column: column j + 2 reuses the buffers of column j only
  // after every wavefront has passed the barrier of column j + 1)
  __shared__ double wsum[2][NW][PWT];
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
  // columns of the panel, expanded at compile time so that every column index
  // (and with it every register index) is a constant
  auto column = [&](auto jc) {
    constexpr int j = decltype(jc)::value;
    if (j >= w) return;   // uniform
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
      const double xj = x[r][j];
      if (i > c && i < m) {
#pragma unroll
        for (int l = 0; l < PWT; ++l) part[l] += xj * x[r][l];
      }
      if (i == c) {
#pragma unroll
        for (int l = 0; l < PWT; ++l) rc[l] = x[r][l];
      }
    }
    {
      const double tot = wave_reduce_scatter<PWT>(part, lane);
      if (lane < PWT) wsum[j & 1][wv][rs_sel<PWT>(lane)] = tot;
    }
    __syncthreads();
    // lane l < PWT adds the wavefront totals of s_l in wavefront order; S[l]
    // is then read from that lane (the same value in every wavefront)
    double S[PWT];
    {
      double a = 0.0;
      if (lane < PWT) {
#pragma unroll
        for (int q = 0; q < NW; ++q) a += wsum[j & 1][q][lane];
      }
      const unsigned long long u = __builtin_bit_cast(unsigned long long, a);
#pragma unroll
      for (int l = 0; l < PWT; ++l) {
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
        S[l] = __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
      }
    }
    const double sq = S[j], x0 = rc[j];
    double tau = 0.0, beta = x0, scale = 0.0;
    if (sq > 0.0) {
      beta = -copysign(sqrt(x0 * x0 + sq), x0);
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    // coefficients of the update of columns l > j (and the T recurrence)
    double d[PWT];
#pragma unroll
    for (int l = 0; l < PWT; ++l) d[l] = (l != j) ? rc[l] + scale * S[l] : 0.0;
    // v into column j (R entry on the diagonal), then H_j on columns l > j
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const int i = p0 + t + NT * r;
      const bool below = i > c && i < m;
      const double xs = x[r][j] * scale;
      const double vi = (i == c) ? 1.0 : (below ? xs : 0.0);
      x[r][j] = (i == c) ? beta : (below ? xs : x[r][j]);
      const double tv = tau * vi;
#pragma unroll
      for (int l = j + 1; l < PWT; ++l) x[r][l] -= tv * d[l];
    }
    // T column j:  T[0:j, j] = -tau T[0:j, 0:j] z,  z_q = v_q . v_j = d_q
    if (t < j) {
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < j; ++q)
        if (q >= t) a += Ts[t][q] * d[q];
      Ts[t][j] = -tau * a;
    }
    if (t == j) Ts[j][j] = tau;   // tau_all is written after the last column (no global store in the loop)
  };
  static_for(column, std::make_integer_sequence<int, PWT>{});
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
  if (t < w) tau_all[(long)b * k + p0 + t] = Ts[t][t];
}

// Partial products over chunks of the column length:
//   P[ch] = A[:, chunk] B[:, chunk]^T   (A: na <= 64 rows, B: nb rows, both of
//   length len and leading dimension ld; chunk ch = entries SCH ch .. SCH ch + SCH - 1),
// written as 64 x 64 row-major tiles.  SAME: B = A (nb = na, the Gram matrix
// S = V V^T of an outer block's reflectors; only the tiles on and above the
// diagonal are formed); else nb <= 16 (W = Y V^T of an in-block update).
// Operands are staged through LDS with coalesced loads; wave w forms the
// 16-row strip w on the FP64 matrix cores (v_mfma_f64_16x16x4: A lane l holds
// A[l%16][l/16], B lane l holds B[l/16][l%16], D lane l register r holds
// D[4r + l/16][l%16]).
static constexpr int SCH = 128;

template <bool SAME>
__global__ __launch_bounds__(256) void qr_rowprod_partial_kernel(const double* A_all, long sA, int na,
                                                                 const double* B_all, long sB, int nb, int len,
                                                                 int ld, double* P_all, int nch) {
  typedef double d4u __attribute__((ext_vector_type(4)));
  constexpr int NBR = SAME ? NBW : 16;
  const int b = blockIdx.y, ch = blockIdx.x;
  const double* A = A_all + b * sA;
  const double* B = B_all + b * sB;
  double* P = P_all + ((long)b * nch + ch) * NBW * NBW;
  const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;
  const int c0 = ch * SCH;
  __shared__ double As[NBW][SCH + 1];
  __shared__ double Bs[SAME ? 1 : NBR][SCH + 1];
  // every staging load is issued before the first LDS store, so that their
  // latencies overlap
  constexpr int LA = NBW * SCH / 256, LB = SAME ? 1 : NBR * SCH / 256;
  double va[LA], vb[LB];
#pragma unroll
  for (int q = 0; q < LA; ++q) {
    const int e = tid + 256 * q, r = e / SCH, c = e % SCH;
    va[q] = (r < na && c0 + c < len) ? A[(long)r * ld + c0 + c] : 0.0;
  }
  if (!SAME) {
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + 256 * q, r = e / SCH, c = e % SCH;
      vb[q] = (r < nb && c0 + c < len) ? B[(long)r * ld + c0 + c] : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < LA; ++q) {
    const int e = tid + 256 * q;
    As[e / SCH][e % SCH] = va[q];
  }
  if (!SAME) {
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int e = tid + 256 * q;
      Bs[e / SCH][e % SCH] = vb[q];
    }
  }
  __syncthreads();
  if (wv * 16 >= na) return;   // no rows for this wave (uniform)
  const int ntile = SAME ? NBW / 16 : 1;
  for (int tj = SAME ? wv : 0; tj < ntile; ++tj) {
    if (tj * 16 >= nb) break;
    d4u d = {0, 0, 0, 0};
#pragma unroll 8
    for (int kk = 0; kk < SCH / 4; ++kk) {
      const int kc = 4 * kk + (l >> 4);
      const double av = As[wv * 16 + (l & 15)][kc];
      const double bv = SAME ? As[tj * 16 + (l & 15)][kc] : Bs[l & 15][kc];
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, d, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) P[(wv * 16 + 4 * r + (l >> 4)) * NBW + tj * 16 + (l & 15)] = d[r];
  }
}

// T of an outer block (nv <= NBW reflectors) from S = V V^T (the sum of the
// chunk partials, fixed order) and the taus, by pairwise merging of adjacent
// diagonal blocks: H_a H_c = I - [V_a V_c] [[T_aa, T_ac], [0, T_cc]] [V_a V_c]^T
// with T_ac = -T_aa S_ac T_cc, from 1 x 1 blocks (T_ii = tau_i) up to nv.
// T is written NBW x NBW (zero below the diagonal and beyond nv).
// Sum over the chunk partials (in chunk order, eight chunks' loads in
// flight) of E entries per thread of the 64 x 64 tiles, entry e = tid + NTH i.
template <int NTH, int E, typename Pred>
__device__ __forceinline__ void sum_partials(const double* P, int nch, int tid, Pred need, double (&acc)[E]) {
#pragma unroll
  for (int i = 0; i < E; ++i) acc[i] = 0.0;
  for (int ch0 = 0; ch0 < nch; ch0 += 8) {
    double v[8][E];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const int e = tid + NTH * i;
        v[q][i] = (ch0 + q < nch && need(e)) ? P[(long)(ch0 + q) * NBW * NBW + e] : 0.0;
      }
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int i = 0; i < E; ++i) acc[i] += v[q][i];
  }
}

__global__ __launch_bounds__(1024) void qr_tblock_kernel(const double* P_all, int nch, int nv, const double* tau_all,
                                                         long sTau, double* TB_all, long sTB) {
  const int b = blockIdx.x;
  const double* P = P_all + (long)b * nch * NBW * NBW;
  const double* tau = tau_all + b * sTau;
  double* TB = TB_all + b * sTB;
  __shared__ double Ss[NBW][NBW + 1];
  __shared__ double Tm[NBW][NBW + 1];
  __shared__ double X[NBW][NBW + 1];
  const int tid = threadIdx.x;
  {
    double acc[4];
    sum_partials<1024, 4>(P, nch, tid,
                          [&](int e) {
                            const int r = e / NBW, c = e % NBW;
                            return r / 16 <= c / 16 && r < nv && c < nv;
                          },
                          acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int e = tid + 1024 * i, r = e / NBW, c = e % NBW;
      Ss[r][c] = acc[i];
      Tm[r][c] = (r == c && r < nv) ? tau[r] : 0.0;
    }
  }
  __syncthreads();
  for (int h = 1; h < NBW; h *= 2) {
    const int nent = (NBW / (2 * h)) * h * h;
    for (int e = tid; e < nent; e += 1024) {
      const int s0 = 2 * h * (e / (h * h)), ii = (e / h) % h, jj = e % h;
      double a = 0.0;
      for (int q = 0; q <= jj; ++q) a += Ss[s0 + ii][s0 + h + q] * Tm[s0 + h + q][s0 + h + jj];
      X[s0 + ii][s0 + h + jj] = a;
    }
    __syncthreads();
    for (int e = tid; e < nent; e += 1024) {
      const int s0 = 2 * h * (e / (h * h)), ii = (e / h) % h, jj = e % h;
      double a = 0.0;
      for (int q = ii; q < h; ++q) a += Tm[s0 + ii][s0 + q] * X[s0 + q][s0 + h + jj];
      Tm[s0 + ii][s0 + h + jj] = -a;
    }
    __syncthreads();
  }
  for (int e = tid; e < NBW * NBW; e += 1024) TB[e] = Tm[e / NBW][e % NBW];
}

// In-block update: Y <- Y - (W T) V for the nt <= 64 rows of Y (length len,
// leading dimension ld), V the panel's pw <= 16 reflector rows, T its
// triangular factor (PW x PW) and W = Y V^T the sum of the chunk partials.
// Grid: (chunk of IB_T entries of the length) x batch x (group of IB_R rows
// of Y), so that a small batch still spreads over the chip; a workgroup sums
// the partials of its IB_R rows of W (in chunk order), forms their W T and
// applies them to its entries (thread = one entry).
static constexpr int IB_T = 128, IB_R = 8;
__global__ __launch_bounds__(IB_T) void qr_inblock_apply_kernel(double* Y_all, long sY, int nt, int len, int ld,
                                                                const double* V_all, long sV, int pw,
                                                                const double* P_all, int nch, const double* T_all,
                                                                long sT) {
  static_assert(IB_R * PW == IB_T, "one W entry per thread");
  const int b = blockIdx.y, r0 = blockIdx.z * IB_R;
  double* Y = Y_all + b * sY;
  const double* V = V_all + b * sV;
  const double* P = P_all + (long)b * nch * NBW * NBW;
  const double* T = T_all + b * sT;
  const int tid = threadIdx.x;
  __shared__ double Wm[IB_R][PW + 1];
  __shared__ double W2[IB_R][PW + 1];
  __shared__ double Ts[PW][PW + 1];
  {
    const int r = r0 + tid / PW, c = tid % PW;
    const bool in = r < nt && c < pw;
    double acc = 0.0;
    for (int ch0 = 0; ch0 < nch; ch0 += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[q] = (ch0 + q < nch && in) ? P[(long)(ch0 + q) * NBW * NBW + r * NBW + c] : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += v[q];
    }
    Wm[tid / PW][c] = acc;
  }
  for (int e = tid; e < PW * PW; e += IB_T) Ts[e / PW][e % PW] = T[e];
  __syncthreads();
  {
    const int r = tid / PW, c = tid % PW;
    double a = 0.0;
    for (int j = 0; j < pw; ++j) a += Wm[r][j] * Ts[j][c];
    W2[r][c] = (c < pw) ? a : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * IB_T + tid;
  if (i >= len) return;
  double v[PW];
#pragma unroll
  for (int c = 0; c < PW; ++c) v[c] = (c < pw) ? V[(long)c * ld + i] : 0.0;
  const int nr = min(IB_R, nt - r0);
  for (int r = 0; r < nr; ++r) {
    double a = 0.0;
#pragma unroll
    for (int c = 0; c < PW; ++c) a += W2[r][c] * v[c];
    Y[(long)(r0 + r) * ld + i] -= a;
  }
}

// W2 = (sum of the S K-slices of W = Y V^T) T' for 16 rows of W per
// workgroup (slices summed in order), T' = T (factorisation) or T^T (Q).
// The slices come from gemm_f64_slices: nt x nv each, slice stride nt nv,
// batch entry stride S nt nv.  W2 is written nt x nv, leading dimension NBW.
template <bool TRANS_T>
__global__ __launch_bounds__(256) void qr_w2_kernel(const double* P_all, int S, int nt, int nv,
                                                    const double* TB_all, long sTB, double* W2_all, long sW2) {
  const int b = blockIdx.y;
  const long snn = (long)nt * nv;
  const double* P = P_all + (long)b * S * snn;
  const double* TB = TB_all + b * sTB;
  double* W2 = W2_all + b * sW2;
  const int tid = threadIdx.x, row0 = blockIdx.x * 16;
  __shared__ double Ts[NBW][NBW + 1];
  __shared__ double Ws[16][NBW + 1];
  // all loads (T, then every slice of this thread's entries) are issued
  // before the first LDS store
  double tv[NBW * NBW / 256], pv[4][QR_SMAX];
#pragma unroll
  for (int q = 0; q < NBW * NBW / 256; ++q) tv[q] = TB[tid + 256 * q];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + 256 * i, r = e / NBW, c = e % NBW;
    const bool ok = row0 + r < nt && c < nv;
#pragma unroll
    for (int sl = 0; sl < QR_SMAX; ++sl) pv[i][sl] = (ok && sl < S) ? P[sl * snn + (long)(row0 + r) * nv + c] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < NBW * NBW / 256; ++q) {
    const int e = tid + 256 * q;
    Ts[e / NBW][e % NBW] = tv[q];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + 256 * i, r = e / NBW, c = e % NBW;
    double a = 0.0;
#pragma unroll
    for (int sl = 0; sl < QR_SMAX; ++sl)
      if (sl < S) a += pv[i][sl];
    Ws[r][c] = a;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int e = tid + 256 * i, r = e / NBW, c = e % NBW;
    if (row0 + r >= nt || c >= nv) continue;
    double a = 0.0;
    for (int j = 0; j < nv; ++j) a += Ws[r][j] * (TRANS_T ? Ts[c][j] : Ts[j][c]);
    W2[(long)(row0 + r) * NBW + c] = a;
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

// K slices of W = Y V^T: about four workgroups per compute unit (the
// product streams Y once, so it needs many loads in flight), slices of at
// least 256 entries
static int w_slices(int nt, int len, int batch) {
  const int tiles = (nt + 63) / 64;
  int S = (1024 + tiles * batch - 1) / (tiles * batch);
  S = std::min(S, std::min(QR_SMAX, len / 256));
  return std::max(S, 1);
}

hipError_t qr_f64_factor(hipStream_t s, int m, int k, int batch, double* Xt, double* R, void* work) {
  if (m < k || k < 1 || batch < 1) return hipErrorInvalidValue;
  if (m > 8192) return hipErrorInvalidValue;   // rows held in registers: at most 8 per thread
  QrLayout L = qr_layout(m, k, batch);
  char* w = (char*)work;
  double* Vr = (double*)(w + L.offV);
  double* T = (double*)(w + L.offT);
  double* TB = (double*)(w + L.offTB);
  double* Wb = (double*)(w + L.offW);
  double* W2b = (double*)(w + L.offW2);
  double* Pb = (double*)(w + L.offP);
  double* tau = (double*)(w + L.offTau);
  hipError_t e = hipSuccess;
  // panels of 16 columns with 256 threads (up to 4 rows each) or 512 threads
  // (4 rows each, up to 2048 rows); beyond 2048 rows 1024 threads with 4
  // columns (up to 8 rows each); no panel crosses an outer block boundary
  struct Panel {
    int p0, pw, nt_threads, rm;
  };
  std::vector<Panel> pans;
  for (int p0 = 0; p0 < k;) {
    const int rows = m - p0;
    const int bend = std::min(k, (p0 / NBW + 1) * NBW);
    Panel P;
    P.p0 = p0;
    if (rows <= 1024) {
      const int need = (rows + 255) / 256;
      P.nt_threads = 256;
      P.rm = need <= 1 ? 1 : need <= 2 ? 2 : 4;
      P.pw = std::min(16, bend - p0);
    } else if (rows <= 2048) {
      P.nt_threads = 512;
      P.rm = 4;
      P.pw = std::min(16, bend - p0);
    } else {
      P.nt_threads = 1024;
      P.rm = (rows + 1023) / 1024;
      P.pw = std::min(4, bend - p0);
    }
    pans.push_back(P);
    p0 += P.pw;
  }
  const int nblk = (k + NBW - 1) / NBW;
  size_t pi = 0;
  for (int bi = 0; bi < nblk && e == hipSuccess; ++bi) {
    const int j0 = bi * NBW, j1 = std::min(k, j0 + NBW), nv = j1 - j0;
    for (; pi < pans.size() && pans[pi].p0 < j1 && e == hipSuccess; ++pi) {
      const Panel& P = pans[pi];
      const int p0 = P.p0, pw = P.pw, rows = m - p0;
      const dim3 g(batch);
      if (P.nt_threads == 256) {
        if (P.rm == 1)
          hipLaunchKernelGGL((qr_panel_kernel<256, 1, 16>), g, dim3(256), 0, s, Xt, Vr, T, tau, m, k, L.sX, L.sT, p0, pw);
        else if (P.rm == 2)
          hipLaunchKernelGGL((qr_panel_kernel<256, 2, 16>), g, dim3(256), 0, s, Xt, Vr, T, tau, m, k, L.sX, L.sT, p0, pw);
        else
          hipLaunchKernelGGL((qr_panel_kernel<256, 4, 16>), g, dim3(256), 0, s, Xt, Vr, T, tau, m, k, L.sX, L.sT, p0, pw);
      } else if (P.nt_threads == 512) {
        hipLaunchKernelGGL((qr_panel_kernel<512, 4, 16>), g, dim3(512), 0, s, Xt, Vr, T, tau, m, k, L.sX, L.sT, p0, pw);
      } else {
        if (P.rm <= 3)
          hipLaunchKernelGGL((qr_panel_kernel<1024, 3, 4>), g, dim3(1024), 0, s, Xt, Vr, T, tau, m, k, L.sX, L.sT, p0, pw);
        else if (P.rm <= 4)
          hipLaunchKernelGGL((qr_panel_kernel<1024, 4, 4>), g, dim3(1024), 0, s, Xt, Vr, T, tau, m, k, L.sX, L.sT, p0, pw);
        else if (P.rm <= 6)
          hipLaunchKernelGGL((qr_panel_kernel<1024, 6, 4>), g, dim3(1024), 0, s, Xt, Vr, T, tau, m, k, L.sX, L.sT, p0, pw);
        else
          hipLaunchKernelGGL((qr_panel_kernel<1024, 8, 4>), g, dim3(1024), 0, s, Xt, Vr, T, tau, m, k, L.sX, L.sT, p0, pw);
      }
      e = hipGetLastError();
      const int nt = j1 - p0 - pw;   // rest of the outer block (rows of Xt)
      if (nt <= 0 || e != hipSuccess) continue;
      // Xt_rest (nt x rows, ld m) -= ((Xt_rest V^T) T) V: chunk partials of W, then the update
      double* Y = Xt + (long)(p0 + pw) * m + p0;
      const double* Vp = Vr + (long)p0 * m + p0;
      const int nch = (rows + SCH - 1) / SCH;
      hipLaunchKernelGGL(qr_rowprod_partial_kernel<false>, dim3(nch, batch), dim3(256), 0, s, (const double*)Y,
                         L.sX, nt, Vp, L.sX, pw, rows, m, Pb, nch);
      e = hipGetLastError();
      if (e != hipSuccess) break;
      hipLaunchKernelGGL(qr_inblock_apply_kernel, dim3((rows + IB_T - 1) / IB_T, batch, (nt + IB_R - 1) / IB_R),
                         dim3(IB_T), 0, s, Y, L.sX, nt, rows,
                         m, Vp, L.sX, pw, (const double*)Pb, nch,
                         (const double*)(T + (long)(p0 / TSLOT) * PW * PW), L.sT);
      e = hipGetLastError();
    }
    if (e != hipSuccess) break;
    // block reflector: T from S = V V^T, then the trailing columns
    const int nt = k - j1, rows = m - j0;
    const double* Vb = Vr + (long)j0 * m + j0;
    const int nch = (rows + SCH - 1) / SCH;
    hipLaunchKernelGGL(qr_rowprod_partial_kernel<true>, dim3(nch, batch), dim3(256), 0, s, Vb, L.sX, nv, Vb, L.sX, nv,
                       rows, m, Pb, nch);
    e = hipGetLastError();
    if (e != hipSuccess) break;
    double* TBb = TB + (long)bi * NBW * NBW;
    hipLaunchKernelGGL(qr_tblock_kernel, dim3(batch), dim3(1024), 0, s, (const double*)Pb, nch, nv,
                       (const double*)(tau + j0), L.sTau, TBb, L.sTB);
    e = hipGetLastError();
    if (nt <= 0 || e != hipSuccess) continue;
    // Xt_trail (nt x rows) -= ((Xt_trail V^T) T) V
    double* Y = Xt + (long)j1 * m + j0;
    const int S = w_slices(nt, rows, batch);
    e = gemm_f64_slices(s, false, true, nt, nv, rows, Y, m, L.sX, Vb, m, L.sX, Wb, S, batch);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(qr_w2_kernel<false>, dim3((nt + 15) / 16, batch), dim3(256), 0, s, (const double*)Wb, S, nt,
                         nv, (const double*)TBb, L.sTB, W2b, L.sW);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = gemm_f64(s, false, false, nt, rows, nv, -1.0, W2b, NBW, L.sW, Vb, m, L.sX, 1.0, Y, m, L.sX, batch);
  }
  if (e != hipSuccess) return e;
  if (R) {
    hipLaunchKernelGGL(qr_extract_r_kernel, dim3(grid_of((long)k * k), batch), dim3(256), 0, s, Xt, R, m, k, L.sX);
    e = hipGetLastError();
  }
  return e;
}

// Q = H_1 ... H_k [I; 0] from the reflectors and block T factors that
// qr_f64_factor left in `work` (which it reads and whose W buffers it uses;
// nothing else).  It may run on another stream than the factorisation, after
// it, while that stream goes on with work that leaves `work` alone.
hipError_t qr_f64_form_q(hipStream_t s, int m, int k, int batch, double* Qt, void* work) {
  if (m < k || k < 1 || batch < 1 || m > 8192) return hipErrorInvalidValue;
  QrLayout L = qr_layout(m, k, batch);
  char* w = (char*)work;
  const double* Vr = (const double*)(w + L.offV);
  const double* TB = (const double*)(w + L.offTB);
  double* Wb = (double*)(w + L.offW);
  double* W2b = (double*)(w + L.offW2);
  const int nblk = (k + NBW - 1) / NBW;
  hipLaunchKernelGGL(qr_eye_kernel, dim3(grid_of((long)k * m), batch), dim3(256), 0, s, Qt, m, k, L.sX);
  hipError_t e = hipGetLastError();
  for (int bi = nblk - 1; bi >= 0 && e == hipSuccess; --bi) {
    const int j0 = bi * NBW, nv = std::min(k, j0 + NBW) - j0;
    const int rows = m - j0, nt = k - j0;
    const double* Vb = Vr + (long)j0 * m + j0;
    const double* TBb = TB + (long)bi * NBW * NBW;
    double* Y = Qt + (long)j0 * m + j0;
    // Qt_sub (rows j0.., columns j0..) -= ((Qt_sub V^T) T^T) V
    const int S = w_slices(nt, rows, batch);
    e = gemm_f64_slices(s, false, true, nt, nv, rows, Y, m, L.sX, Vb, m, L.sX, Wb, S, batch);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(qr_w2_kernel<true>, dim3((nt + 15) / 16, batch), dim3(256), 0, s, (const double*)Wb, S, nt,
                         nv, TBb, L.sTB, W2b, L.sW);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = gemm_f64(s, false, false, nt, rows, nv, -1.0, W2b, NBW, L.sW, Vb, m, L.sX, 1.0, Y, m, L.sX, batch);
  }
  return e;
}

hipError_t qr_f64(hipStream_t s, int m, int k, int batch, double* Xt, double* R, double* Qt, void* work) {
  hipError_t e = qr_f64_factor(s, m, k, batch, Xt, R, work);
  if (e == hipSuccess && Qt) e = qr_f64_form_q(s, m, k, batch, Qt, work);
  return e;
}

}  // namespace sctm
