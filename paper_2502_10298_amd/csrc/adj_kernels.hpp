// Small FP64 kernels of the reverse pass (projector / SVD adjoint, energy).
#pragma once
#include <hip/hip_runtime.h>

namespace sctm {

// dst += (cast) src
hipError_t add_cast(hipStream_t s, const void* src, bool src_f64, void* dst, bool dst_f64, long n);
// out[0] = #{S > rel * S[0]}
hipError_t rank_count(hipStream_t s, int n, const double* S, double rel, int* out);
// dst[i][c] = src[i][c] * sgn[c]   (src FP64 or FP32, dst FP64, na x chi)
hipError_t scale_cols_from(hipStream_t s, const void* src, bool src_f64, double* dst, int na, int chi,
                           const double* sgn);
// Ubar = Xbar S^{-1/2}, Vbar = Ybar S^{-1/2}, Sbar = -1/2 S^{-3/2} diag(U^T Xbar + V^T Ybar) (first k columns)
hipError_t svd_adj_prep(hipStream_t s, int nb, int chi, const double* U, const double* V, const double* S,
                        const int* kr, const double* Xb, const double* Yb, double* Ub, double* Vb, double* Sb);
// out[i][c] = X[i][c] / sqrt(S[c]) for c < k (= kr[0]), zero otherwise (nb x chi)
hipError_t scale_cols_rsqrt_s(hipStream_t s, int nb, int chi, const double* X, const double* S, const int* kr,
                              double* out);
// zero rows i >= *r of GU and GV (nb x chi)
hipError_t zero_rows_from(hipStream_t s, int nb, int chi, double* GU, double* GV, const int* r);
// inner matrix of the thin SVD adjoint, first c2 rows (Itop, c2 x nb) and the
// first c2 columns of the remaining rows (Ileft, (nb-c2) x c2)
hipError_t svd_adj_inner(hipStream_t s, int nb, int c2, int chi, const double* S, const double* Sb,
                         const double* GU, const double* GV, const int* kr, double eps, double* Itop,
                         double* Ileft);
// C1[:, c] /= s_c, C2[:, c] /= s_c for c < k, zero otherwise (nb x chi)
hipError_t scale_cols_inv_s(hipStream_t s, int nb, int chi, double* C1, double* C2, const double* S, const int* kr);
// Q1[c][b] += C2[b][c], c < c2   (C2: nb x chi, Q1: c2 x nb)
hipError_t add_transposed(hipStream_t s, int nb, int chi, int c2, const double* C2, double* Q1);
// Q2[b][c] = C1[b][c], c < c2    (C1: nb x chi, Q2: nb x c2)
hipError_t copy_cols(hipStream_t s, int nb, int chi, int c2, const double* C1, double* Q2);
// rhobar[P,Q,R,S] += ebar * (h[(R,S),(P,Q)] - e delta) / den
hipError_t bond_energy_adjoint(hipStream_t s, int p, const double* h, const double* e, const double* ebar,
                               double* rhobar);

}  // namespace sctm
