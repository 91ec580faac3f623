// Dense kernels of the randomized eigensolver and the posterior sampler:
// tall-skinny block products on the matrix cores (FP64, or BF16 inputs with
// FP32 accumulation) and small s x s factorizations, batched over matrices.
#pragma once

#include "common.h"

namespace hinv {

// C (s1 x s2, column-major, ldc) = X^T Y with X: n x s1 (ldx), Y: n x s2 (ldy).
// bf16: inputs rounded to BF16, products accumulated in FP32 per K-chunk and
// the chunks summed in FP64 in a fixed order.
void gram(Ctx* ctx, DenseWork& w, int n, int s1, int s2, const double* X, int ldx, const double* Y,
          int ldy, double* C, int ldc, bool bf16 = false);

// C (n x t, ldc) = alpha X (n x s, ldx) B (s x t, ldb) + beta C.
void gemm_tall(Ctx* ctx, int n, int s, int t, double alpha, const double* X, int ldx,
               const double* B, int ldb, double beta, double* C, int ldc);

// The small s x s routines below treat nb independent matrices at once, one
// workgroup each: matrix b starts at base + b * stride (strides in elements).

// Upper Cholesky factors in place: A_b (s x s, lda) = R^T R, R upper, lower
// part zeroed, after adding shift[b] (device array, or null for none) to the
// diagonal.  Returns false if any matrix met a non-positive pivot
// (synchronizes the stream).
bool cholesky_upper(Ctx* ctx, DenseWork& w, int nb, int s, double* A, int lda, size_t sa,
                    const double* shift = nullptr);

// Rinv_b (s x s) = R_b^-1 for upper-triangular R_b (Rinv_b must not overlap R_b).
void tri_inverse_upper(Ctx* ctx, DenseWork& w, int nb, int s, const double* R, int ldr, size_t sr, double* Rinv,
                       int ldi, size_t si);

// Symmetric eigendecompositions T_b = S_b diag(lam_b) S_b^T by parallel
// cyclic Jacobi; T_b is symmetrized and overwritten; eigenpairs sorted by
// decreasing eigenvalue.
void sym_eig(Ctx* ctx, DenseWork& w, int nb, int s, double* T, int ldt, size_t st, double* S, int lds, size_t ss,
             double* lam, size_t sl);

// out[b] = factor * trace(A_b) (device, no synchronization).
void scaled_trace(Ctx* ctx, int nb, int s, const double* A, int lda, size_t sa, double factor, double* out);

// C (m x n) = alpha op(A) op(B) + beta C, op(X) = X^T when its flag is set
// (kk inner dimension; small matrices, one thread per entry of C).
void small_gemm(Ctx* ctx, bool ta, bool tb, int m, int n, int kk, double alpha, const double* A, int lda,
                const double* B, int ldb, double beta, double* C, int ldc);

// C[i, j] /= d[i] + d[j] for the s x s matrix C (device d).
void sylvester_diag(Ctx* ctx, int s, const double* d, double* C, int ldc);

// out[i] = base[i] + sum_j w[j] V[i, j]^2 (base may be null: 0; w: device, k).
void weighted_squares(Ctx* ctx, int n, int k, const double* V, int ldv, const double* w, const double* base,
                      double* out);

// Row scaling B[i, :] *= d[i] (B: s x t column-major).
void scale_rows(Ctx* ctx, int s, int t, const double* d, double* B, int ldb);

}  // namespace hinv
