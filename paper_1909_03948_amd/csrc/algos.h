// Host drivers of the paper's algorithms; all vector and matrix work runs in
// device kernels, the host only makes the scalar decisions.
#pragma once

#include "problem.h"

namespace hinv {

// Inexact Newton-CG (Alg. 1).  Returns HINV_OK, HINV_ENOCONV or HINV_ESTATE.
int map_newton(Problem& P, const double* m0, double* m_map, const hinv_newton_opts& o,
               hinv_newton_info* info);

// Double-pass randomized generalized eigensolver (Alg. 2) with PreCholQR (Alg. 4).
int lowrank_eig(Problem& P, int mode, int tprod, int s, const double* omega, int ldo, int k,
                double* lambda_host, double* V, int ldv, SolveStats* st);

// The two dense stages of the double pass for a group of ni instances of one
// mesh size (n nodes): member j's n x s blocks start at base + j n s (Y, Zb,
// Q, AQ), its s x s matrices at base + j s^2 (G, Ri, T, S) and its s
// eigenvalues at lam + j s.  The s x s factorizations of all members run in
// one launch each; the tall products run per member.
struct DenseWork;
// b_identity: B = I (Zbar = Z) instead of the prior operator R.
// rank: when given (one instance only), a block Y of numerical rank r < s does
// not fail: qr(Y) keeps the r leading directions of Y^T Y (U: s x s and g: s
// doubles of workspace), Q gets r columns and *rank = r; otherwise *rank = s.
int precholqr(Problem* const* P, int ni, DenseWork& dw, int s, double* Y, double* Zb, double* Q, double* G,
              double* Ri, bool b_identity = false, int* rank = nullptr, double* U = nullptr, double* g = nullptr);
void rayleigh_ritz(Problem* const* P, int ni, DenseWork& dw, int s, int k, int tprod, const double* Q,
                   const double* AQ, double* T, double* S, double* lam, double* const* V, int ldv,
                   double* const* lambda_host);

// Single-pass randomized generalized eigensolver (Alg. 3) with PreCholQR (Alg. 4).
int lowrank_eig_single(Problem& P, int mode, int s, const double* omega, int ldo, int k,
                       double* lambda_host, double* V, int ldv, SolveStats* st);

// Pointwise variance (Sec. 4.4): the prior's from a randomized
// eigendecomposition of R^-1 (Eq. eq:prior_mvar), the posterior's by the
// low-rank correction (Eq. eq:post_mvar).
int prior_variance(Problem& P, int s, const double* omega, int ldo, double* diag, double* mu_host,
                   SolveStats* st);
void posterior_variance(Problem& P, const double* prior_diag, int k, const double* lambda_host, const double* V,
                        int ldv, double* diag);

// Samples per internal chunk of posterior_sample_seeded (its white noise:
// 6 N^2 kSampleChunk doubles, 12.9 GB at N = 1024).
constexpr int kSampleChunk = 256;

// Posterior samples with their white noise drawn on the device in chunks
// (samples first .. first + ns - 1 of the counter-based stream), R V formed
// once per call.
void posterior_sample_seeded(Problem& P, const double* m_map, int k, const double* lambda_host, const double* V,
                             int ldv, uint64_t seed, uint64_t stream, long long first, int ns, double* out, int ldo,
                             SolveStats* st);

// Posterior samples through the low-rank update (Sec. 4.3.2).
void posterior_sample(Problem& P, const double* m_map, int k, const double* lambda_host,
                      const double* V, int ldv, int ns, const double* eta, int ldeta, double* out,
                      int ldo, SolveStats* st);

}  // namespace hinv
