// Dense kernels of the randomized eigensolver and the posterior sampler:
// tall-skinny block products on the matrix cores (FP64, or BF16 inputs with
// FP32 accumulation) and small s x s factorizations in one workgroup.
#pragma once

#include "common.h"

namespace hinv {

// Scratch for split-K partial products.
struct DenseWork {
    DBuf<double> part;
    DBuf<int> flag;
};

// C (s1 x s2, column-major, ldc) = X^T Y with X: n x s1 (ldx), Y: n x s2 (ldy).
// bf16: inputs rounded to BF16, products accumulated in FP32 per K-chunk and
// the chunks summed in FP64 in a fixed order.
void gram(Ctx* ctx, DenseWork& w, int n, int s1, int s2, const double* X, int ldx, const double* Y,
          int ldy, double* C, int ldc, bool bf16 = false);

// C (n x t, ldc) = alpha X (n x s, ldx) B (s x t, ldb) + beta C.
void gemm_tall(Ctx* ctx, int n, int s, int t, double alpha, const double* X, int ldx,
               const double* B, int ldb, double beta, double* C, int ldc);

// Upper Cholesky factor in place: A (s x s, lda) = R^T R, R upper, lower part
// zeroed.  Adds `shift` to the diagonal first.  Returns false on a
// non-positive pivot.
bool cholesky_upper(Ctx* ctx, DenseWork& w, int s, double* A, int lda, double shift);

// Rinv (s x s) = R^-1 for upper-triangular R.
void tri_inverse_upper(Ctx* ctx, int s, const double* R, int ldr, double* Rinv, int ldi);

// Symmetric eigendecomposition T = S diag(lam) S^T by parallel cyclic Jacobi;
// T is symmetrized and overwritten; eigenpairs sorted by decreasing eigenvalue.
void sym_eig(Ctx* ctx, DenseWork& w, int s, double* T, int ldt, double* S, int lds, double* lam);

// Frobenius-norm trace helper: returns trace(A) (host value; synchronizes).
double trace(Ctx* ctx, DenseWork& w, int s, const double* A, int lda);

// Row scaling B[i, :] *= d[i] (B: s x t column-major).
void scale_rows(Ctx* ctx, int s, int t, const double* d, double* B, int ldb);

}  // namespace hinv
