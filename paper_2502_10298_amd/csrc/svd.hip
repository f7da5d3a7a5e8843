// FP64 SVD by blocked one-sided (Hestenes) Jacobi, for the projector matrices
// M = U S V^T of the split-CTMRG projector recipe.
//
// The columns of G = M are orthogonalised by orthogonal rotations G <- G W,
// accumulated in V <- V W (or, for a lower-triangular M, V is solved for from
// M V = G once after the sweeps); at convergence G = U S.  Columns are grouped in
// blocks of 16; a round-robin tournament pairs the blocks so that every
// round updates disjoint column sets in parallel.  For each block pair the
// 32 x 32 Gram matrix of its columns is formed from the actual columns,
// diagonalised with a cyclic two-sided Jacobi in LDS, and the resulting
// rotation is applied to the 32 columns of G and of V.
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
#include <cstdio>
#include <vector>

namespace sctm {

static constexpr int JW = 16;        // columns per block
static constexpr int JP = 2 * JW;    // columns per block pair

static inline int padded(int n) { return ((n + JP - 1) / JP) * JP; }

struct SvdLayout {
  int np, nb, pairs, rounds, nchG, nchV;
  long sG, sV, sOff;
  size_t offG, offV, offG2, offV2, offOff, offNorm, offRank, offDone, offFro, offPart, offW, offRot, offCnt, offBad,
      total;
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
  L.nchG = (n + 255) / 256;
  L.nchV = (L.np + 255) / 256;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  L.offG = take(sizeof(double) * L.sG * batch);
  L.offV = take(sizeof(double) * L.sV * batch);
  L.offG2 = take(sizeof(double) * L.sG * batch);
  L.offV2 = take(sizeof(double) * L.sV * batch);
  L.offOff = take(sizeof(double) * L.sOff * batch);
  L.offNorm = take(sizeof(double) * (size_t)L.np * batch);
  L.offRank = take(sizeof(int) * (size_t)L.np * batch);
  L.offDone = take(sizeof(int) * (size_t)batch);
  L.offFro = take(sizeof(double) * (size_t)batch);
  L.offPart = take(sizeof(double) * (size_t)L.pairs * L.nchG * 1024 * batch);
  L.offW = take(sizeof(double) * (size_t)L.pairs * 1024 * batch);
  L.offRot = take(sizeof(int) * (size_t)L.pairs * batch);
  L.offCnt = take(sizeof(unsigned long long));
  L.offBad = take(sizeof(int) * (size_t)batch);
  L.total = off;
  return L;
}

size_t svd_work_bytes(int n, int batch) { return layout(n, batch).total; }

// Gt = M^T (cold start) or only its padding rows (warm start: rows < n come
// from Gt = (M V0)^T by GEMM); Vt = I or V0^T, padded with the identity.
__global__ void svd_init_kernel(const double* M, const double* V0, int n, int np, double* Gt, double* Vt, int* done,
                                long sG, long sV, unsigned long long* cnt) {
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
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    done[b] = 0;
    if (b == 0) *cnt = 0;
  }
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

// One round of the tournament is two launches:
//   pair:   grid (pair): the 32 x 32 Gram matrix of the pair's columns on the
//           FP64 matrix cores, the convergence test and, unless the pair is
//           converged, its diagonalisation by cyclic two-sided Jacobi in LDS,
//           giving the 32 x 32 rotation W (one workgroup per pair, so the
//           Gram matrix is summed in a fixed order and never leaves the chip);
//   rotate: grid (pair, chunk of G or of V): new columns = old columns W,
//           again on the matrix cores.
//
// A pair counts as orthogonal when
//   |g_i . g_j| <= tol max(|g_i|, f) max(|g_j|, f),   f = 1e-13 |M|_F:
// relative for columns above the floor f (every singular triplet above it is
// fixed to relative accuracy O(tol)), absolute at the floor for columns below
// it.  Columns that small carry the rounding noise of the rotations of the
// large ones; asking them to be orthogonal in relative terms never converges
// for a numerically rank-deficient M.
typedef double d4v __attribute__((ext_vector_type(4)));

// Jacobi rotation that zeroes the (a, c) entry of a symmetric 2 x 2 block:
// new row a = c row_a - s row_c, new row c = s row_a + c row_c (same on
// columns).  Below the threshold the identity is returned.  With D = h_cc -
// h_aa, E = 2 h_ac and r = sqrt(D^2 + E^2), the smaller angle has tangent
// t = sign(D E) |E| / (|D| + r); writing d = |D| + r, the pair
//   c = d / sqrt(d^2 + E^2),  s = sign(D E) |E| / sqrt(d^2 + E^2)
// has that tangent, and c^2 + s^2 = 1 holds to the accuracy of the one
// reciprocal square root, whatever the accuracy of r (any t gives an exact
// rotation; r only steers how well the entry is zeroed).  r comes from the
// hardware reciprocal square root with one Newton step, 1 / sqrt(d^2 + E^2)
// with two.  Branch-free.
__device__ inline void jacobi_rot(double haa, double hcc, double hac, double thr, double negl2, double& c, double& s) {
  const bool active = hac * hac > thr * thr * fmax(haa, negl2) * fmax(hcc, negl2);
  const double D = hcc - haa, E = 2.0 * hac;
  const double q = D * D + E * E;
  double y = __builtin_amdgcn_rsq(q);
  y = y * (1.5 - 0.5 * q * y * y);
  const double d = fabs(D) + q * y;   // |D| + r
  const double x = d * d + E * E;
  double z = __builtin_amdgcn_rsq(x);
  z = z * (1.5 - 0.5 * x * z * z);
  z = z * (1.5 - 0.5 * x * z * z);
  const double sg = ((D >= 0.0) == (E >= 0.0)) ? fabs(E) : -fabs(E);
  c = active ? d * z : 1.0;
  s = active ? sg * z : 0.0;
}

// One workgroup of eight wavefronts per block pair: the 32 x 32 Gram matrix
// of the pair's columns, its convergence test and, unless the pair is
// converged, its diagonalisation by cyclic two-sided Jacobi, giving the
// rotation W.  Fused so that the Gram matrix never leaves the chip.
//
// Gram: wave w takes entries [512 k + 64 w, +64) of the column length in
// slice k (the same number of slices in every wave); the 64 x 32 block is
// loaded in one go (the next slice's loads are issued before the current one
// is multiplied), staged through the wavefront's own LDS region (no
// workgroup barrier, so the wavefronts drift apart and overlap their loads
// and multiplies) two 16-entry subs at a time into the operand layout of
// v_mfma_f64_16x16x4 (A lane l holds A[l%16][l/16], B lane
// l holds B[l/16][l%16], D lane l register r holds D[4r + l/16][l%16]), and
// accumulated per wave; the eight wave partials are summed in a fixed order.
//
// Eigensolve: in each inner round the 32 indices form 16 disjoint pairs;
// thread (p, q) < 256 owns the 2 x 2 blocks of H and of W (the accumulated
// rotations) at row pair p and column pair q, applies both rotations and
// forms J_p^T H J_q and W J_q in registers; H is double-buffered, so one
// barrier per inner round.  Threads 256..511 take part in the barriers only.
static constexpr int JPT = 512;                 // threads of the pair kernel
static constexpr int JSL = 64 * (JPT / 64);     // column-length entries per slice

// Orders the LDS accesses of one wavefront around a point (its lanes exchange
// data through the wavefront's own LDS region): a wavefront executes its LDS
// instructions in order, so it suffices that the compiler neither moves
// memory accesses across this point nor leaves the writes outstanding.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

// Raw loads of a wavefront's 64-entry slice of the pair's 32 columns
// (entries past the end read the last one); they are zeroed when staged, so
// that nothing waits for a prefetch before it is used.
__device__ inline void gram_load(const double* Gp, const double* Gq, int m, int c0, int l, double (&v)[4][8]) {
#pragma unroll
  for (int sub = 0; sub < 4; ++sub)
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int cc = min(c0 + sub * 16 + (l & 15), m - 1);
      v[sub][i] = (i < 4) ? Gp[(long)(i * 4) * m + cc] : Gq[(long)((i - 4) * 4) * m + cc];
    }
}

__global__ __launch_bounds__(JPT) void jacobi_pair_kernel(const double* Gt_all, int m, int np, int round, long sG,
                                                          double tol, double* off_all, long sOff, double* W_all,
                                                          int* rot_all, const int* done, int inner_sweeps,
                                                          const double* fro2_all, unsigned long long* entries) {
  const int b = blockIdx.y, pr = blockIdx.x;
  const int nb = np / JW, pairs = nb / 2;
  const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;
  int* rot = rot_all + (long)b * pairs + pr;
  if (done[b]) {
    if (tid == 0) *rot = 0;
    return;
  }
  int p, q;
  circle_pair(nb, round, pr, p, q);
  // staging [wave][2 subs][32][17]; then the wave partials [8][768]; then
  // W [32][33] at the start and H (two copies of [32][33]) after the partials
  __shared__ double sm[8 * 2 * JP * 17];
  __shared__ double wmax[8];
  // ---- Gram matrix ----
  const double* Gt = Gt_all + b * sG;
  const double* Gp = Gt + (long)(p * JW + (l >> 4)) * m;   // column i < JW of the pair: row p*JW + i
  const double* Gq = Gt + (long)(q * JW + (l >> 4)) * m;   // column JW + i: row q*JW + i
  d4v acc00 = d4v{0, 0, 0, 0}, acc01 = d4v{0, 0, 0, 0}, acc11 = d4v{0, 0, 0, 0};
  const int nsl = (m + JSL - 1) / JSL;
  double v[4][8], vn[4][8];
  gram_load(Gp, Gq, m, wv * 64, l, v);
  double* stg = sm + wv * 2 * JP * 17;
  for (int k = 0; k < nsl; ++k) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const bool in = k * JSL + wv * 64 + (2 * half + s2) * 16 + (l & 15) < m;
          stg[(s2 * JP + i * 4 + (l >> 4)) * 17 + (l & 15)] = in ? v[2 * half + s2][i] : 0.0;
        }
      wave_lds_sync();   // the staging region is the wavefront's own
      if (half == 0 && k + 1 < nsl) gram_load(Gp, Gq, m, (k + 1) * JSL + wv * 64, l, vn);
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        const double* buf = stg + s2 * JP * 17;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int kc = kk * 4 + (l >> 4);
          const double a0 = buf[(l & 15) * 17 + kc], a1 = buf[(16 + (l & 15)) * 17 + kc];
          acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a0, acc00, 0, 0, 0);
          acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, a1, acc01, 0, 0, 0);
          acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, a1, acc11, 0, 0, 0);
        }
      }
      wave_lds_sync();
    }
    if (k + 1 < nsl) {
#pragma unroll
      for (int sub = 0; sub < 4; ++sub)
#pragma unroll
        for (int i = 0; i < 8; ++i) v[sub][i] = vn[sub][i];
    }
  }
  // wave partials of the tiles (0,0), (0,1), (1,1); the tile (1,0) is the
  // transpose of (0,1) and is not formed.  They overwrite other wavefronts'
  // staging regions: every wavefront must be done with its own first.
  __syncthreads();
  double* wp = sm + wv * 768;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    wp[(0 * 4 + r) * 64 + l] = acc00[r];
    wp[(1 * 4 + r) * 64 + l] = acc01[r];
    wp[(2 * 4 + r) * 64 + l] = acc11[r];
  }
  __syncthreads();
  double (*H2)[JP][JP + 1] = reinterpret_cast<double (*)[JP][JP + 1]>(sm + 8 * 768);
  double (*W)[JP + 1] = reinterpret_cast<double (*)[JP + 1]>(sm);
  double (*H)[JP + 1] = H2[0];
  for (int e = tid; e < 768; e += JPT) {
    double a = 0.0;
#pragma unroll
    for (int w = 0; w < 8; ++w) a += sm[w * 768 + e];
    const int lane = e & 63, r = (e >> 6) & 3, tt = e >> 8;
    const int ti = tt == 2 ? 1 : 0, tj = tt == 0 ? 0 : 1;
    H[ti * 16 + 4 * r + (lane >> 4)][tj * 16 + (lane & 15)] = a;
  }
  __syncthreads();
  if (tid < 256) {
    const int i = tid >> 4, j = tid & 15;
    H[16 + j][i] = H[i][16 + j];
  }
  for (int e = tid; e < JP * JP; e += JPT) W[e / JP][e % JP] = (e / JP == e % JP) ? 1.0 : 0.0;
  __syncthreads();

  // ---- convergence measure of this pair (NaN-propagating max); the
  // hardware reciprocal square root is ample for a threshold test ----
  double* offv = off_all + b * sOff;
  const double negl2 = 1e-26 * fro2_all[b];   // f^2 = (1e-13 |M|_F)^2
  double om = 0.0;
  for (int e = tid; e < JP * JP; e += JPT) {
    const int i = e / JP, j = e % JP;
    if (j > i) {
      const double hii = fmax(H[i][i], negl2), hjj = fmax(H[j][j], negl2);
      double x = fabs(H[i][j]) * __builtin_amdgcn_rsq(hii * hjj);
      if (H[i][j] != H[i][j] || H[i][i] != H[i][i] || H[j][j] != H[j][j]) x = NAN;
      om = (x != x || om != om) ? NAN : fmax(om, x);
    }
  }
  for (int w = 32; w > 0; w >>= 1) {
    const double o = __shfl_xor(om, w);
    om = (o != o || om != om) ? NAN : fmax(om, o);
  }
  if (l == 0) wmax[wv] = om;
  __syncthreads();
  {
    double a = wmax[0];
    for (int k = 1; k < JPT / 64; ++k) a = (a != a || wmax[k] != wmax[k]) ? NAN : fmax(a, wmax[k]);
    om = a;
  }
  if (tid == 0) {
    offv[(long)round * pairs + pr] = om;
    *rot = (om > tol) ? 1 : 0;
    // column-length entries of G and V the rotation will touch (statistics)
    if (om > tol) atomicAdd(entries, (unsigned long long)(m + np));
  }
  if (!(om > tol)) return;   // converged pair (or NaN: leave the data as is)

  // Thread (pp, qq) computes the rotation of index pair qq and takes that of
  // pair pp from the lane of its wavefront that computed it (computing both
  // in every thread doubles the quarter-rate reciprocal square roots and is
  // slower).  The pairs of the circle tournament advance by one position per
  // round; the 2 x 2 blocks of the 256 owners cover H, and W entries are read
  // and written by their owner only within a round.
  const bool owner = tid < 256;
  const double thr = 0.1 * tol;
  const int pp = (tid >> 4) & 15, qq = tid & 15;
  const int src = (l & 48) | pp;   // lane (pp mod 4, pp) of this wavefront
  int cur = 0;
  for (int sw = 0; sw < inner_sweeps; ++sw) {
    int ap, cp, aq, cq;
    circle_pair(JP, 0, pp, ap, cp);
    circle_pair(JP, 0, qq, aq, cq);
    int moved = 0;
    for (int rr = 0; rr < JP - 1; ++rr) {
      if (owner) {
        double (*Hc)[JP + 1] = H2[cur];
        double (*Hn)[JP + 1] = H2[cur ^ 1];
        // every LDS read of the round first: the reads of the 2 x 2 blocks
        // overlap the rotation's dependent chain
        const double haa = Hc[aq][aq], hcc = Hc[cq][cq], hac = Hc[aq][cq];
        const double h00 = Hc[ap][aq], h01 = Hc[ap][cq], h10 = Hc[cp][aq], h11 = Hc[cp][cq];
        const double w00 = W[ap][aq], w01 = W[ap][cq], w10 = W[cp][aq], w11 = W[cp][cq];
        double c2, s2;
        jacobi_rot(haa, hcc, hac, thr, negl2, c2, s2);
        const double c1 = __shfl(c2, src), s1 = __shfl(s2, src);
        moved |= (s2 != 0.0) ? 1 : 0;
        const double r00 = c1 * h00 - s1 * h10, r01 = c1 * h01 - s1 * h11;
        const double r10 = s1 * h00 + c1 * h10, r11 = s1 * h01 + c1 * h11;
        Hn[ap][aq] = c2 * r00 - s2 * r01;
        Hn[ap][cq] = s2 * r00 + c2 * r01;
        Hn[cp][aq] = c2 * r10 - s2 * r11;
        Hn[cp][cq] = s2 * r10 + c2 * r11;
        W[ap][aq] = c2 * w00 - s2 * w01;
        W[ap][cq] = s2 * w00 + c2 * w01;
        W[cp][aq] = c2 * w10 - s2 * w11;
        W[cp][cq] = s2 * w10 + c2 * w11;
      }
      cur ^= 1;
      // next round of the circle: index 0 keeps player 0, the others move on
      const int ap1 = (ap == JP - 1) ? 1 : ap + 1, cp1 = (cp == JP - 1) ? 1 : cp + 1;
      const int aq1 = (aq == JP - 1) ? 1 : aq + 1, cq1 = (cq == JP - 1) ? 1 : cq + 1;
      ap = (pp == 0) ? ap : ap1;
      cp = (pp == 0) ? cp + 1 : cp1;
      aq = (qq == 0) ? aq : aq1;
      cq = (qq == 0) ? cq + 1 : cq1;
      __syncthreads();
    }
    if (!__syncthreads_or(moved)) break;
  }
  double* Wout = W_all + ((long)b * pairs + pr) * JP * JP;
  for (int e = tid; e < JP * JP; e += JPT) Wout[e] = W[e / JP][e % JP];
}

// new columns = old columns W for the rows of Gt (chunks 0 .. nchG-1 of JCHR
// entries, length m) and of Vt (chunks nchG .., length np); each of the eight
// wavefronts owns 64 entries of the column length and reads all 32 columns
// there before writing them back.
static constexpr int JCHR = 512;

__global__ __launch_bounds__(512) void jacobi_rotate_kernel(double* Gt_all, double* Vt_all, int m, int np, int round,
                                                            long sG, long sV, const double* W_all, const int* rot_all,
                                                            int nchG, const int* done) {
  const int b = blockIdx.z;
  const int nb = np / JW, pairs = nb / 2;
  const int pr = blockIdx.x;
  if (done[b] || !rot_all[(long)b * pairs + pr]) return;
  int p, q;
  circle_pair(nb, round, pr, p, q);
  __shared__ double Ws[JP][JP + 1];
  const int tid = threadIdx.x, l = tid & 63, wv = tid >> 6;
  const bool isG = (int)blockIdx.y < nchG;
  double* X = isG ? Gt_all + b * sG : Vt_all + b * sV;
  const int len = isG ? m : np;
  const int c0 = (isG ? blockIdx.y : blockIdx.y - nchG) * JCHR + wv * 64;
  // the wave's 64 entries of all 32 columns are loaded before any is written,
  // and before W (their latency covers W's); column i of the pair is row
  // p*JW + i (i < JW) or q*JW + i - JW of X.  Entries past the end read the
  // last one (in bounds, never stored), so the loads carry no branches.
  double* Xp = X + (long)(p * JW + (l >> 4)) * len;
  double* Xq = X + (long)(q * JW + (l >> 4)) * len;
  double old[4][8];
#pragma unroll
  for (int tc = 0; tc < 4; ++tc) {
    const int c = min(c0 + tc * 16 + (l & 15), len - 1);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
      old[tc][kk] = (kk < 4) ? Xp[(long)(kk * 4) * len + c] : Xq[(long)((kk - 4) * 4) * len + c];
    // loads stay in column-tile order: the multiply of tile 0 waits for its
    // eight loads only
    __builtin_amdgcn_sched_barrier(0);
  }
  const double* Wg = W_all + ((long)b * pairs + pr) * JP * JP;
  for (int e = tid; e < JP * JP; e += 512) Ws[e / JP][e % JP] = Wg[e];
  __syncthreads();
  if (c0 >= len) return;   // whole wave past the end (no barrier follows)
  // column tile by column tile (two independent accumulator chains each), so
  // that the stores of one tile stream out while the next is multiplied
  double a[8][2];
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    a[kk][0] = Ws[kk * 4 + (l >> 4)][l & 15];        // (W^T)[i][j]
    a[kk][1] = Ws[kk * 4 + (l >> 4)][16 + (l & 15)];
  }
#pragma unroll
  for (int tc = 0; tc < 4; ++tc) {
    d4v d0 = d4v{0, 0, 0, 0}, d1 = d4v{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk][0], old[tc][kk], d0, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kk][1], old[tc][kk], d1, 0, 0, 0);
    }
    const int c = c0 + tc * 16 + (l & 15);
    if (c < len) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        Xp[(long)(4 * r) * len + c] = d0[r];
        Xq[(long)(4 * r) * len + c] = d1[r];
      }
    }
  }
}

// |M|_F^2 of every batch entry: FRO_BLOCKS blocks per entry write partial
// sums, a second pass adds them in a fixed order.
static constexpr int FRO_BLOCKS = 64;

__global__ void svd_fro2_partial_kernel(const double* M, long nn, double* part) {
  const int b = blockIdx.y;
  const double* x = M + (long)b * nn;
  __shared__ double red[256];
  double a = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < nn; i += 256L * FRO_BLOCKS) a += x[i] * x[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[b * FRO_BLOCKS + blockIdx.x] = red[0];
}

__global__ void svd_fro2_final_kernel(const double* part, double* fro2) {
  const int b = blockIdx.x;
  __shared__ double red[FRO_BLOCKS];
  red[threadIdx.x] = part[b * FRO_BLOCKS + threadIdx.x];
  __syncthreads();
  for (int w = FRO_BLOCKS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) fro2[b] = red[0];
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

// Rows of X (length len, np rows per batch entry) moved to the positions of
// the descending column-norm order (rows >= n keep their place).
__global__ void svd_permute_rows_kernel(const double* Xin_all, double* Xout_all, const int* rank_all, int n, int np,
                                        int len, long sX) {
  const int j = blockIdx.x, b = blockIdx.y;
  const int dst = (j < n) ? rank_all[(long)b * np + j] : j;
  const double* src = Xin_all + b * sX + (long)j * len;
  double* out = Xout_all + b * sX + (long)dst * len;
  for (int i = threadIdx.x; i < len; i += blockDim.x) out[i] = src[i];
}

// position of column j in the descending-norm order (ties: lower index
// first); the norms of the batch entry are staged in LDS (n <= 4096)
__global__ void svd_rank_kernel(const double* norms_all, int n, int np, int* rank_all) {
  const int b = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const double* s = norms_all + (long)b * np;
  __shared__ double sn[4096];
  for (int i = threadIdx.x; i < n; i += blockDim.x) sn[i] = s[i];
  __syncthreads();
  if (j >= n) return;
  const double sj = sn[j];
  int r = 0;
#pragma unroll 8
  for (int i = 0; i < n; ++i) {
    const double si = sn[i];
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

// V from the final columns when M is lower triangular: with G = M V (V the
// product of all rotations) each row v of V^T solves v M^T = g for the row g
// of G^T, i.e. v_c = (g_c - sum_{k<c} v_k M[c][k]) / M[c][c], forward in c.
// Blocked: TRSM_NB columns at a time, the in-block substitution here (one
// thread per row of V^T, right-looking so that the updates of the later
// columns are independent of each other), the rest of the row by a rank-NB
// GEMM update.  A triangular solve is backward stable componentwise, so the
// result is the exact V of a matrix within n eps |M| of M, entry by entry.
static constexpr int TRSM_NB = 64;

// One wavefront per 64 rows of V^T: the diagonal block of M (stored
// transposed, so that a column of M is contiguous for 16-byte reads) and the
// 64 x 64 tile of V^T are staged through LDS with coalesced row loads; each
// thread then substitutes its own row in registers, reading M as wavefront-
// uniform (broadcast) LDS values, and the tile goes back the same way.
template <bool FULL>
__global__ __launch_bounds__(64) void trsm_rows_block_kernel(const double* __restrict__ M_all, int n, int i0,
                                                             double* Vt_all, int ldv, long sV) {
  __shared__ __attribute__((aligned(16))) double Mt[TRSM_NB][TRSM_NB + 2];   // Mt[c][r] = M[i0 + r][i0 + c]
  __shared__ double Xs[TRSM_NB][TRSM_NB + 1];                              // Xs[row][c]
  const int b = blockIdx.y, t = threadIdx.x, j0 = blockIdx.x * 64;
  const double* M = M_all + (long)b * n * n + (long)i0 * n + i0;   // the diagonal block
  double* Vt = Vt_all + b * sV + i0;
  const int nbk = FULL ? TRSM_NB : n - i0;
  for (int r = 0; r < TRSM_NB; ++r) {
    Mt[t][r] = (r < nbk && t < nbk) ? M[(long)r * n + t] : (r == t ? 1.0 : 0.0);
    Xs[r][t] = (j0 + r < n && t < nbk) ? Vt[(long)(j0 + r) * ldv + t] : 0.0;
  }
  __syncthreads();
  double x[TRSM_NB];
#pragma unroll
  for (int c = 0; c < TRSM_NB; ++c) x[c] = Xs[t][c];
#pragma unroll
  for (int c = 0; c < TRSM_NB; ++c) {
    x[c] = x[c] / Mt[c][c];
#pragma unroll
    for (int r = c + 1; r < TRSM_NB; ++r) x[r] -= x[c] * Mt[c][r];
  }
#pragma unroll
  for (int c = 0; c < TRSM_NB; ++c) Xs[t][c] = x[c];
  __syncthreads();
  for (int r = 0; r < TRSM_NB; ++r)
    if (j0 + r < n && t < nbk) Vt[(long)(j0 + r) * ldv + t] = Xs[r][t];
}

// flag[b] = 1 when more than max(16, n / 4) diagonal entries of the triangle
// M_b are at most 1e-13 of the largest (or any is NaN): many pivots at the
// rounding level of a numerically rank-deficient matrix.  The count is a
// predictor only (triangles with more such pivots often pass the check of
// the solved V, and some with none fail it); the bound balances a second
// decomposition against the rotations of V on the projector matrices of the
// 2x2 D = 8 and the chi = 170 scaling workloads.
__global__ __launch_bounds__(256) void svd_tiny_pivots_kernel(const double* M_all, int n, int* flag) {
  const int b = blockIdx.x, t = threadIdx.x;
  const double* M = M_all + (long)b * n * n;
  __shared__ double red[256];
  __shared__ int cnt;
  double mx = 0.0;
  int nan = 0;
  for (int i = t; i < n; i += 256) {
    const double d = fabs(M[(long)i * n + i]);
    nan |= (d != d) ? 1 : 0;
    mx = fmax(mx, d);
  }
  red[t] = mx;
  if (t == 0) cnt = 0;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] = fmax(red[t], red[t + w]);
    __syncthreads();
  }
  const double floor = 1e-13 * red[0];
  int mine = 0;
  for (int i = t; i < n; i += 256) mine += (fabs(M[(long)i * n + i]) <= floor) ? 1 : 0;
  if (mine) atomicAdd(&cnt, mine);
  if (nan) atomicAdd(&cnt, 1 << 20);
  __syncthreads();
  if (t == 0) flag[b] = (cnt > max(16, n / 4)) ? 1 : 0;
}

// Orthogonality check of Y = V^T V in two passes: part[b][k] = 1 unless
// |Y - I| <= tau on the rows k, k + 64, ... (NaN counts as bad), then
// bad[b] = OR of the 64 partials
static constexpr int ORTH_PARTS = 64;

__global__ __launch_bounds__(256) void orth_check_partial_kernel(const double* Y_all, int n, long sY, double tau,
                                                                 int* part) {
  const int b = blockIdx.y;
  const double* Y = Y_all + b * sY;
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  int mine = 0;
  for (int r = blockIdx.x; r < n; r += ORTH_PARTS)
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      const double d = Y[(long)r * n + c] - (r == c ? 1.0 : 0.0);
      mine |= (fabs(d) <= tau) ? 0 : 1;
    }
  if (mine) any = 1;   // benign race: every writer stores 1
  __syncthreads();
  if (threadIdx.x == 0) part[b * ORTH_PARTS + blockIdx.x] = any;
}

__global__ void orth_check_final_kernel(const int* part, int* bad) {
  const int b = blockIdx.x;
  int any = 0;
  for (int k = 0; k < ORTH_PARTS; ++k) any |= part[b * ORTH_PARTS + k];
  if (threadIdx.x == 0) bad[b] = any;
}

// Y <- 1.5 I - 0.5 Y for batch n x n matrices at stride sY
__global__ void ns_shift_kernel(double* Y_all, int n, long sY) {
  double* Y = Y_all + blockIdx.y * sY;
  const long tot = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x)
    Y[e] = ((e / n) == (e % n) ? 1.5 : 0.0) - 0.5 * Y[e];
}

hipError_t svd_f64(hipStream_t s, int n, int batch, const double* M, double* U, double* S, double* V, void* work,
                   int max_sweeps, double tol, int* host_flags, int* sweeps_out, const double* V0, bool lower_tri) {
  if (n < 1 || n > 4096) return hipErrorInvalidValue;   // the column ranks stage n norms in LDS
  if (!(tol > 0.0)) tol = 1.2e-16 * std::sqrt((double)n);   // ~ sqrt(m) eps: the rounding floor of a dot product
  SvdLayout L = layout(n, batch);
  char* w = (char*)work;
  double* Gt = (double*)(w + L.offG);
  double* Vt = (double*)(w + L.offV);
  double* Gt2 = (double*)(w + L.offG2);
  double* Vt2 = (double*)(w + L.offV2);
  double* off = (double*)(w + L.offOff);
  double* norms = (double*)(w + L.offNorm);
  int* rank = (int*)(w + L.offRank);
  int* done = (int*)(w + L.offDone);
  double* fro2 = (double*)(w + L.offFro);
  double* part = (double*)(w + L.offPart);
  double* Wr = (double*)(w + L.offW);
  int* rot = (int*)(w + L.offRot);
  unsigned long long* cnt = (unsigned long long*)(w + L.offCnt);
  int* bad = (int*)(w + L.offBad);
  // V is accumulated from the rotations, or (lower-triangular M, cold start)
  // solved for after the sweeps, which halves the rotations' memory traffic.
  // A triangle with many pivots at the rounding level (a numerically
  // rank-deficient M) would fail the orthogonality check of the solved V and
  // cost a second decomposition: such a batch accumulates V from the start.
  bool solveV = lower_tri && V0 == nullptr;
  if (solveV) {
    hipLaunchKernelGGL(svd_tiny_pivots_kernel, dim3(batch), dim3(256), 0, s, M, n, bad);
    hipError_t e = hipMemcpyAsync(host_flags, bad, sizeof(int) * batch, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int b = 0; b < batch; ++b) solveV = solveV && host_flags[b] == 0;
  }
  // the Gram partial buffer is free until the first round: it holds the norm partials
  hipLaunchKernelGGL(svd_fro2_partial_kernel, dim3(FRO_BLOCKS, batch), dim3(256), 0, s, M, (long)n * n, part);
  hipLaunchKernelGGL(svd_fro2_final_kernel, dim3(batch), dim3(FRO_BLOCKS), 0, s, (const double*)part, fro2);
  hipError_t err = hipSuccess;
  {
    long tot = (long)L.np * n + (long)L.np * L.np;
    int g = (int)std::min<long>((tot + 255) / 256, 8192);
    hipLaunchKernelGGL(svd_init_kernel, dim3(g, batch), dim3(256), 0, s, M, V0, n, L.np, Gt, Vt, done, L.sG, L.sV, cnt);
    if (V0) {   // Gt[j][i] = sum_k V0[k][j] M[i][k]
      err = gemm_f64(s, true, true, n, n, n, 1.0, V0, n, (long)n * n, M, n, (long)n * n, 0.0, Gt, n, L.sG, batch);
      if (err != hipSuccess) return err;
    }
  }
  int sweeps = 0;
  static const int inner = [] {
    const char* e = std::getenv("SPLITCTM_SVD_INNER");
    int v = e ? std::atoi(e) : 1;
    return v < 1 ? 1 : (v > 12 ? 12 : v);
  }();
  err = hipSuccess;
  int running = batch;
  const int nrG = (n + JCHR - 1) / JCHR, nrV = (L.np + JCHR - 1) / JCHR;   // rotation chunks
  for (int sw = 0; sw < max_sweeps; ++sw) {
    // columns in descending norm order before every sweep (the large ones
    // meet first in the tournament, which cuts the sweep count of graded
    // spectra); V's columns follow the same permutation
    hipLaunchKernelGGL(svd_norms_kernel, dim3(n, batch), dim3(256), 0, s, (const double*)Gt, n, L.sG, norms, L.np);
    hipLaunchKernelGGL(svd_rank_kernel, dim3((n + 255) / 256, batch), dim3(256), 0, s, (const double*)norms, n, L.np,
                       rank);
    hipLaunchKernelGGL(svd_permute_rows_kernel, dim3(L.np, batch), dim3(256), 0, s, (const double*)Gt, Gt2,
                       (const int*)rank, n, L.np, n, L.sG);
    std::swap(Gt, Gt2);
    if (!solveV) {
      hipLaunchKernelGGL(svd_permute_rows_kernel, dim3(L.np, batch), dim3(256), 0, s, (const double*)Vt, Vt2,
                         (const int*)rank, n, L.np, L.np, L.sV);
      std::swap(Vt, Vt2);
    }
    // algorithmic work of one round for the batch entries still running (the
    // rotation's share is added from the device counter after the sweep)
    const double gram_fl = (double)L.pairs * running * 2.0 * JP * JP * n;
    const double gram_by = (double)L.pairs * running * 8.0 * (JP * (double)n + JP * JP);
    for (int r = 0; r < L.rounds; ++r) {
      launch_timed(KC_JACOBI_GRAM, gram_fl, gram_by, jacobi_pair_kernel, dim3(L.pairs, batch), dim3(JPT), 0, s,
                   (const double*)Gt, n, L.np, r, L.sG, tol, off, L.sOff, Wr, rot, (const int*)done, inner,
                   (const double*)fro2, cnt);
      launch_timed(KC_JACOBI_ROTATE, 0.0, 0.0, jacobi_rotate_kernel, dim3(L.pairs, nrG + (solveV ? 0 : nrV), batch),
                   dim3(512), 0, s,
                   Gt, Vt, n, L.np, r, L.sG, L.sV, (const double*)Wr, (const int*)rot, nrG, (const int*)done);
    }
    hipLaunchKernelGGL(svd_check_kernel, dim3(batch), dim3(256), 0, s, off, L.sOff, tol, done);
    ++sweeps;
    err = hipMemcpyAsync(host_flags, done, sizeof(int) * batch, hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) return err;
    running = 0;
    for (int b = 0; b < batch; ++b) running += host_flags[b] ? 0 : 1;
    static const int conv_trace = [] {
      const char* e = std::getenv("SPLITCTM_SVD_TRACE");
      return e ? std::atoi(e) : 0;
    }();
    if (conv_trace >= 2) {   // largest off-diagonal measure of the sweep, per batch entry
      std::vector<double> ho((size_t)L.sOff * batch);
      err = hipMemcpy(ho.data(), off, sizeof(double) * ho.size(), hipMemcpyDeviceToHost);
      if (err != hipSuccess) return err;
      fprintf(stderr, "[svd] n=%d sweep %d off:", n, sw + 1);
      for (int b = 0; b < batch; ++b) {
        double mx = 0.0;
        for (long i = 0; i < L.sOff; ++i) mx = std::max(mx, ho[(size_t)b * L.sOff + i]);
        fprintf(stderr, " %.1e", mx);
      }
      fprintf(stderr, "\n");
    }
    if (running == 0) break;
  }
  if (KernelTimer* tm = kernel_timer()) {   // exact work of the rotations that ran
    unsigned long long e = 0;
    err = hipMemcpyAsync(&e, cnt, sizeof(e), hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    if (err != hipSuccess) return err;
    // the pair kernel counts m + np entries per rotation; the V part only
    // when V is accumulated
    if (solveV) e = e / (unsigned long long)(n + L.np) * (unsigned long long)n;
    tm->add(KC_JACOBI_ROTATE, 2.0 * JP * JP * (double)e, 2.0 * JP * 8.0 * (double)e);
  }
  if (solveV) {
    // V^T rows = G^T rows, then the forward substitution in place
    err = hipMemcpy2DAsync(Vt, sizeof(double) * L.np, Gt, sizeof(double) * n, sizeof(double) * n, (size_t)L.np * batch,
                           hipMemcpyDeviceToDevice, s);
    if (err != hipSuccess) return err;
    for (int i0 = 0; i0 < n; i0 += TRSM_NB) {
      const int nbk = std::min(TRSM_NB, n - i0), rest = n - i0 - nbk;
      if (nbk == TRSM_NB)
        hipLaunchKernelGGL(trsm_rows_block_kernel<true>, dim3((n + 63) / 64, batch), dim3(64), 0, s, M, n, i0, Vt,
                           L.np, L.sV);
      else   // the ragged last block: the identity pads the diagonal block
        hipLaunchKernelGGL(trsm_rows_block_kernel<false>, dim3((n + 63) / 64, batch), dim3(64), 0, s, M, n, i0, Vt,
                           L.np, L.sV);
      if (rest > 0) {   // v[c] -= sum_{k in block} v[k] M[c][k] for the later columns c
        err = gemm_f64(s, false, true, n, rest, nbk, -1.0, Vt + i0, L.np, L.sV, M + (long)(i0 + nbk) * n + i0, n,
                       (long)n * n, 1.0, Vt + i0 + nbk, L.np, L.sV, batch);
        if (err != hipSuccess) return err;
      }
    }
  }
  hipLaunchKernelGGL(svd_norms_kernel, dim3(n, batch), dim3(256), 0, s, Gt, n, L.sG, norms, L.np);
  hipLaunchKernelGGL(svd_rank_kernel, dim3((n + 255) / 256, batch), dim3(256), 0, s, norms, n, L.np, rank);
  {
    long tot = (long)n * n;
    int g = (int)std::min<long>((tot + 255) / 256, 8192);
    hipLaunchKernelGGL(svd_scatter_kernel, dim3(g, batch), dim3(256), 0, s, Gt, Vt, norms, rank, n, L.np, L.sG, L.sV,
                       U, S, V);
  }
  // An accumulated V is the product of every rotation of every sweep: each is
  // orthogonal to rounding, but their product drifts (~1e-13 after ten sweeps
  // at n ~ 1000); a solved V is orthogonal to ~kappa eps (checked below);
  // U = G / |G| is orthogonal to the stopping tolerance.  The reverse pass of
  // a truncated SVD with a strongly graded spectrum (s_k / s_1 down to 1e-8)
  // turns an orthogonality defect d into a gradient error of about
  // d s_1 / s_k, so both factors are brought to working orthogonality by one
  // Newton-Schulz step X <- X (3 I - X^T X) / 2 (d becomes ~ d^2; zero columns
  // of U stay zero).  U S V^T then differs from M by the stopping tolerance,
  // an exact SVD of a matrix that close to M.  The buffers of the sweeps,
  // free now, hold X^T X and the product.
  {
    double* Y = Vt2;   // n x n at stride sV >= n^2
    double* Xn = Gt2;  // n x n at stride sG >= n^2
    const long nn = (long)n * n;
    for (double* X : {V, U}) {
      err = gemm_f64(s, true, false, n, n, n, 1.0, X, n, nn, X, n, nn, 0.0, Y, n, L.sV, batch);
      if (err != hipSuccess) return err;
      if (X == V && solveV) {
        // the solved V is orthogonal to about kappa eps, kappa the condition
        // number of M with its rows scaled to unit length (small for the
        // preconditioned triangle of a full-rank matrix); a numerically
        // rank-deficient M leaves rows of rounding noise and V far from
        // orthogonal, and the whole batch is then decomposed again with V
        // accumulated from the rotations
        int* opart = (int*)(w + L.offPart);   // free after the sweeps
        hipLaunchKernelGGL(orth_check_partial_kernel, dim3(ORTH_PARTS, batch), dim3(256), 0, s, (const double*)Y, n,
                           L.sV, 2e-12, opart);
        hipLaunchKernelGGL(orth_check_final_kernel, dim3(batch), dim3(64), 0, s, (const int*)opart, bad);
        err = hipMemcpyAsync(host_flags, bad, sizeof(int) * batch, hipMemcpyDeviceToHost, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        if (err != hipSuccess) return err;
        int nbad = 0;
        for (int b = 0; b < batch; ++b) nbad += host_flags[b] ? 1 : 0;
        if (nbad) {
          static const bool trace = std::getenv("SPLITCTM_SVD_TRACE") != nullptr;
          if (trace) fprintf(stderr, "[svd] n=%d: V by substitution not orthogonal in %d of %d, rotations kept\n", n,
                             nbad, batch);
          return svd_f64(s, n, batch, M, U, S, V, work, max_sweeps, tol, host_flags, sweeps_out, nullptr, false);
        }
      }
      hipLaunchKernelGGL(ns_shift_kernel, dim3((int)std::min<long>((nn + 255) / 256, 4096), batch), dim3(256), 0, s,
                         Y, n, L.sV);
      err = gemm_f64(s, false, false, n, n, n, 1.0, X, n, nn, Y, n, L.sV, 0.0, Xn, n, L.sG, batch);
      if (err != hipSuccess) return err;
      err = hipMemcpy2DAsync(X, sizeof(double) * nn, Xn, sizeof(double) * L.sG, sizeof(double) * nn, batch,
                             hipMemcpyDeviceToDevice, s);
      if (err != hipSuccess) return err;
    }
  }
  if (sweeps_out) *sweeps_out = sweeps;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Preconditioned SVD (Drmac and Veselic's QR preconditioning of one-sided
// Jacobi): with the columns of A sorted by decreasing norm (permutation P),
// A P = Q R by Householder QR, then the QR of the lower-triangular R^T =
// Q1 R1, and the Jacobi SVD of R1^T = U_J S V_J^T gives
//   A = (Q U_J) S (P Q1 V_J)^T.
// R^T has nearly orthogonal columns for graded A, and the second QR (one
// step of the QR iteration on R R^T) makes them closer still: the Jacobi
// needs about half the sweeps of the plain matrix, and two fewer with the
// second QR than without it at the projector sizes; each QR costs less than
// one sweep.

// column norms of row-major n x n matrices (thread = column, coalesced rows)
__global__ __launch_bounds__(256) void pre_colnorm_kernel(const double* A_all, int n, double* nrm_all) {
  const int b = blockIdx.y;
  const int cl = threadIdx.x & 63, rg = threadIdx.x >> 6;   // 64 columns x 4 row groups
  const int c = blockIdx.x * 64 + cl;
  const double* A = A_all + (long)b * n * n;
  __shared__ double red[4][64];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (c < n) {
    int r = rg;
    for (; r + 12 < n; r += 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double v = A[(long)(r + 4 * u) * n + c];
        acc[u] += v * v;
      }
    }
    for (; r < n; r += 4) {
      const double v = A[(long)r * n + c];
      acc[0] += v * v;
    }
  }
  red[rg][cl] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (rg == 0 && c < n) nrm_all[(long)b * n + c] = (red[0][cl] + red[1][cl]) + (red[2][cl] + red[3][cl]);
}

// position of column c in the decreasing-norm order (ties: lower index first)
__global__ void pre_rank_kernel(const double* nrm_all, int n, int* rank_all) {
  const int b = blockIdx.y;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const double* s = nrm_all + (long)b * n;
  __shared__ double sn[4096];
  for (int i = threadIdx.x; i < n; i += blockDim.x) sn[i] = s[i];
  __syncthreads();
  if (c >= n) return;
  const double sc = sn[c];
  int r = 0;
#pragma unroll 8
  for (int i = 0; i < n; ++i) r += (sn[i] > sc || (sn[i] == sc && i < c)) ? 1 : 0;
  rank_all[(long)b * n + c] = r;
}

// Xt[rank[c]][r] = A[r][c]  (rows of Xt = the sorted columns of A), 32 x 32
// tiles through LDS so that reads and writes are both coalesced
__global__ void pre_gather_kernel(const double* A_all, const int* rank_all, int n, double* Xt_all) {
  const int b = blockIdx.z;
  const double* A = A_all + (long)b * n * n;
  double* Xt = Xt_all + (long)b * n * n;
  const int* rk = rank_all + (long)b * n;
  __shared__ double tile[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 8 rows per pass
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    tile[k][tx] = (r < n && c < n) ? A[(long)r * n + c] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (c < n && r < n) Xt[(long)rk[c] * n + r] = tile[tx][k];
  }
}

// V[c][:] = UJ[rank[c]][:]
__global__ void pre_unpermute_rows_kernel(const double* UJ_all, const int* rank_all, int n, double* V_all) {
  const int c = blockIdx.x, b = blockIdx.y;
  const double* src = UJ_all + (long)b * n * n + (long)rank_all[(long)b * n + c] * n;
  double* dst = V_all + (long)b * n * n + (long)c * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
}

// B = A^T for row-major n x n matrices (32 x 32 LDS tiles)
__global__ void pre_transpose_kernel(const double* A_all, int n, double* B_all) {
  const int b = blockIdx.z;
  const double* A = A_all + (long)b * n * n;
  double* B = B_all + (long)b * n * n;
  __shared__ double tile[32][33];
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    tile[k][tx] = (r < n && c < n) ? A[(long)r * n + c] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (c < n && r < n) B[(long)c * n + r] = tile[tx][k];
  }
}

struct PreLayout {
  size_t offX, offR, offQ, offQ1, offUJ, offVJ, offN, offRk, offQW, offQW2, offJW, total;
};

static PreLayout pre_layout(int n, int batch) {
  PreLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t nn = sizeof(double) * (size_t)n * n * batch;
  L.offX = take(nn);
  L.offR = take(nn);
  L.offQ = take(nn);
  L.offQ1 = take(nn);
  L.offUJ = take(nn);
  L.offVJ = take(nn);
  L.offN = take(sizeof(double) * (size_t)n * batch);
  L.offRk = take(sizeof(int) * (size_t)n * batch);
  L.offQW = take(qr_work_bytes(n, n, batch));    // first QR (its Q may still be formed during the second)
  L.offQW2 = take(qr_work_bytes(n, n, batch));   // second QR
  L.offJW = take(svd_work_bytes(n, batch));
  L.total = off;
  return L;
}

size_t svd_precond_work_bytes(int n, int batch) {
  return pre_layout(n, batch).total;
}

hipError_t svd_precond_f64(hipStream_t s, int n, int batch, const double* A, double* U, double* S, double* V,
                           void* work, int max_sweeps, double tol, int* host_flags, int* sweeps_out,
                           hipStream_t qs, hipEvent_t* ev) {
  if (n < 1 || n > 4096) return hipErrorInvalidValue;   // the limit of svd_f64
  PreLayout L = pre_layout(n, batch);
  char* w = (char*)work;
  double* Xt = (double*)(w + L.offX);
  double* R = (double*)(w + L.offR);
  double* Qt = (double*)(w + L.offQ);
  double* Q1t = (double*)(w + L.offQ1);
  double* UJ = (double*)(w + L.offUJ);
  double* VJ = (double*)(w + L.offVJ);
  double* nrm = (double*)(w + L.offN);
  int* rk = (int*)(w + L.offRk);
  const long nn = (long)n * n;
  const dim3 tiles((n + 31) / 32, (n + 31) / 32, batch);
  hipLaunchKernelGGL(pre_colnorm_kernel, dim3((n + 63) / 64, batch), dim3(256), 0, s, A, n, nrm);
  hipLaunchKernelGGL(pre_rank_kernel, dim3((n + 255) / 256, batch), dim3(256), 0, s, (const double*)nrm, n, rk);
  hipLaunchKernelGGL(pre_gather_kernel, tiles, dim3(256), 0, s, A, (const int*)rk, n, Xt);
  // A P = Q R (Xt holds (A P)^T).  Only R feeds the second QR and the Jacobi;
  // Q and Q1 are needed at the end, so with a second stream they are formed
  // there while this stream runs the second QR and the sweeps (the two QRs
  // have workspaces of their own).
  const bool split = qs != nullptr && ev != nullptr;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = qr_f64_factor(s, n, n, batch, Xt, R, w + L.offQW);
  if (e == hipSuccess && split) {
    e = hipEventRecord(ev[0], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(qs, ev[0], 0);
    if (e == hipSuccess) e = qr_f64_form_q(qs, n, n, batch, Qt, w + L.offQW);
  } else if (e == hipSuccess) {
    e = qr_f64_form_q(s, n, n, batch, Qt, w + L.offQW);
  }
  // R^T = Q1 R1: the QR of the lower-triangular R^T, whose transpose is R
  // itself (R is overwritten by the reflectors; R1 lands in Xt)
  if (e == hipSuccess) e = qr_f64_factor(s, n, n, batch, R, Xt, w + L.offQW2);
  if (e == hipSuccess && split) {
    e = hipEventRecord(ev[1], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(qs, ev[1], 0);
    if (e == hipSuccess) e = qr_f64_form_q(qs, n, n, batch, Q1t, w + L.offQW2);
    if (e == hipSuccess) e = hipEventRecord(ev[2], qs);
  } else if (e == hipSuccess) {
    e = qr_f64_form_q(s, n, n, batch, Q1t, w + L.offQW2);
  }
  // the Jacobi input is R1^T (row-major, in R)
  if (e == hipSuccess) {
    hipLaunchKernelGGL(pre_transpose_kernel, tiles, dim3(256), 0, s, (const double*)Xt, n, R);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = svd_f64(s, n, batch, R, UJ, S, VJ, w + L.offJW, max_sweeps, tol, host_flags, sweeps_out, nullptr, true);
  // Q and Q1 (formed on qs) before they are read
  if (e == hipSuccess && split) e = hipStreamWaitEvent(s, ev[2], 0);
  // R1^T = U_J S V_J^T  =>  A P = Q R1^T Q1^T... = (Q U_J) S (Q1 V_J)^T:
  // U = Q U_J, V = P Q1 V_J
  if (e == hipSuccess) e = gemm_f64(s, true, false, n, n, n, 1.0, Qt, n, nn, UJ, n, nn, 0.0, U, n, nn, batch);
  if (e == hipSuccess) e = gemm_f64(s, true, false, n, n, n, 1.0, Q1t, n, nn, VJ, n, nn, 0.0, Xt, n, nn, batch);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(pre_unpermute_rows_kernel, dim3(n, batch), dim3(256), 0, s, (const double*)Xt,
                       (const int*)rk, n, V);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace sctm
