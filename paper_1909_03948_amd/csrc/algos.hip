// Drivers of the paper's algorithms on top of the device operations.
#include <algorithm>
#include <vector>
#include <cmath>

#include "algos.h"
#include "dense.h"

namespace hinv {

namespace {

__global__ void k_post_scale(int k, const double* __restrict__ lam, double* __restrict__ s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) s[i] = 1.0 - 1.0 / sqrt(1.0 + lam[i]);
}

__global__ void k_add_vec(int n, const double* __restrict__ v, double* __restrict__ x, int ld) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) x[(size_t)blockIdx.y * ld + k] += v[k];
}

double nrm(Ctx* c, int n, const double* x) { return std::sqrt(dev_dot(c, n, x, x)); }

// Scalars of the Newton-CG loop kept on the device (slots of cgs): 0 = r^T z,
// 1 = d^T H d, 2 = alpha, 3 = 1 when d^T H d <= 0, 4 = |r|^2, 5 = new r^T z.
// Only slots 3 and 4 travel to the host, once per CG iteration.
__global__ void k_cg_alpha(double* __restrict__ cgs) {
    if (threadIdx.x == 0) {
        const double dHd = cgs[1];
        const bool ok = dHd > 0.0;
        cgs[2] = ok ? cgs[0] / dHd : 0.0;
        cgs[3] = ok ? 0.0 : 1.0;
    }
}

// mhat += alpha d, r -= alpha H d (alpha = 0 after non-positive curvature)
__global__ void k_cg_step(int n, const double* __restrict__ cgs, const double* __restrict__ d,
                          const double* __restrict__ Hd, double* __restrict__ mh, double* __restrict__ r) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double alpha = cgs[2];
    mh[k] = alpha * d[k] + 1.0 * mh[k];
    r[k] = -alpha * Hd[k] + 1.0 * r[k];
}

// d = z + beta d with beta = (new r^T z) / (r^T z)
__global__ void k_cg_dir(int n, const double* __restrict__ cgs, const double* __restrict__ z,
                         double* __restrict__ d) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    d[k] = 1.0 * z[k] + (cgs[5] / cgs[0]) * d[k];
}

__global__ void k_cg_roll(double* __restrict__ cgs) {
    if (threadIdx.x == 0) cgs[0] = cgs[5];
}

// Tightens the problem's solve tolerance for the lifetime of the guard.
struct TolGuard {
    Problem& P;
    double saved;
    TolGuard(Problem& p, double t) : P(p), saved(p.rtol) { P.rtol = std::min(P.rtol, t); }
    ~TolGuard() { P.rtol = saved; }
};

// Forward and adjoint solves of the outer loop (two per Newton step) run to
// this tolerance: near the minimizer the Armijo decrease and the gradient norm
// fall below the noise that 1e-10 solves leave in J and g.
constexpr double kOuterRtol = 1e-12;

}  // namespace

// ------------------------------------------------------------ Newton-CG ---
// Algorithm 1 with the readings: eta_i = min(0.5, sqrt(|g_i|/|g_0|)); CG
// preconditioned by R^{-1}, started at zero, stopped at |H mhat + g| <= eta |g|
// or at non-positive curvature (first iteration: take the preconditioned
// steepest-descent direction); Armijo backtracking with step halving.
int map_newton(Problem& P, const double* m0, double* m_map, const hinv_newton_opts& o,
               hinv_newton_info* info) {
    Ctx* c = P.ctx;
    const int n = P.n, ns = P.ns;
    std::memset(info, 0, sizeof(*info));
    P.ws_newton.ensure((size_t)n * 7 + (size_t)ns * 3);
    P.ws_scal.ensure(8);
    double* cgs = P.ws_scal.get();
    if (!c->host_red)
        HINV_HIP(hipHostMalloc((void**)&c->host_red, sizeof(double) * Ctx::kHostRed, hipHostMallocDefault));
    double* m = m_map;
    // state vectors (ns entries): u, p, ut; parameter vectors (n): the rest
    double* u = P.ws_newton.get();
    double* p = u + ns;
    double* ut = p + ns;
    double* g = ut + ns;
    double* mh = g + n;
    double* r = mh + n;
    double* z = r + n;
    double* d = z + n;
    double* Hd = d + n;
    double* mt = Hd + n;
    SolveStats st;
    if (m0)
        dev_copy(c, n, 1, m0, n, m, n);
    else
        dev_fill(c, n, P.m_prior, m);
    {
        TolGuard tg(P, kOuterRtol);
        P.forward(m, u, &st);
    }
    double mis, reg;
    P.cost(m, u, &mis, &reg);
    double J = mis + reg;
    info->cost[0] = J;
    double g0 = -1.0;
    int status = HINV_ENOCONV;
    int it = 0;
    bool have_grad_at_m = false;
    while (it < o.max_iter) {
        {
            TolGuard tg(P, kOuterRtol);
            P.gradient(m, u, p, g, &st);
        }
        have_grad_at_m = true;
        const double gn = nrm(c, n, g);
        info->gnorm[it] = gn;
        if (g0 < 0) g0 = gn;
        if (gn <= std::max(o.rel_tol * g0, o.abs_tol)) {
            info->converged = 1;
            status = HINV_OK;
            break;
        }
        const double eta = std::min(0.5, std::sqrt(gn / g0));
        // Gauss-Newton Hessian (positive semidefinite misfit part) for the first
        // steps, where the full Hessian can be indefinite; the full Hessian after
        const int hmode = it < o.gn_iters ? HINV_HESS_GN_FULL : HINV_HESS_FULL;
        P.linearize(m, u, p);
        // --- CG on H mhat = -g ---
        dev_fill(c, n, 0.0, mh);
        dev_copy(c, n, 1, g, n, r, n);
        dev_axpby(c, n, 0.0, g, -1.0, r);  // r = -g
        P.prior_solve(1, r, n, z, n, &st);
        dev_copy(c, n, 1, z, n, d, n);
        dev_dot_to(c, n, r, z, cgs);  // r^T z
        int ncg = 0;
        const int nb = ceil_div(n, kBlock);
        for (int k = 0; k < o.max_cg; ++k) {
            P.hessian(hmode, 1, d, n, Hd, n, &st);
            ++info->hessian_applies;
            ++ncg;
            dev_dot_to(c, n, d, Hd, cgs + 1);
            k_cg_alpha<<<1, 64, 0, c->stream>>>(cgs);
            k_cg_step<<<nb, kBlock, 0, c->stream>>>(n, cgs, d, Hd, mh, r);
            dev_dot_to(c, n, r, r, cgs + 4);
            HINV_LAUNCH_CHECK();
            HINV_HIP(hipMemcpyAsync(c->host_red, cgs + 3, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HINV_HIP(hipStreamSynchronize(c->stream));
            if (c->host_red[0] != 0.0) {
                // non-positive curvature: the step above used alpha = 0
                if (k == 0) dev_copy(c, n, 1, d, n, mh, n);
                break;
            }
            if (std::sqrt(c->host_red[1]) <= eta * gn) break;
            P.prior_solve(1, r, n, z, n, &st);
            dev_dot_to(c, n, r, z, cgs + 5);
            k_cg_dir<<<nb, kBlock, 0, c->stream>>>(n, cgs, z, d);  // d = z + beta d
            k_cg_roll<<<1, 64, 0, c->stream>>>(cgs);
            HINV_LAUNCH_CHECK();
        }
        info->cg_iters[it] = ncg;
        // --- Armijo backtracking ---
        const double gm = dev_dot(c, n, g, mh);
        double alpha = 1.0;
        bool accepted = false;
        for (int j = 0; j < o.max_backtrack; ++j) {
            dev_copy(c, n, 1, m, n, mt, n);
            dev_axpby(c, n, alpha, mh, 1.0, mt);
            // a trial point whose forward solve misses its tolerance is rejected
            SolveStats trial;
            {
                TolGuard tg(P, kOuterRtol);
                P.forward(mt, ut, &trial);
            }
            const bool solved = trial.converged;
            trial.converged = true;  // counted, but a failed trial does not fail the run
            st.add(trial);
            double mt_mis, mt_reg;
            P.cost(mt, ut, &mt_mis, &mt_reg);
            const double Jt = mt_mis + mt_reg;
            if (solved && Jt < J + alpha * o.c_armijo * gm) {
                dev_copy(c, n, 1, mt, n, m, n);
                dev_copy(c, ns, 1, ut, ns, u, ns);
                J = Jt;
                accepted = true;
                break;
            }
            alpha *= 0.5;
        }
        info->alpha[it] = alpha;
        info->cost[it + 1] = J;
        have_grad_at_m = false;
        ++it;
        if (!accepted) {
            status = HINV_ESTATE;
            break;
        }
    }
    info->iterations = it;
    // leave the problem linearized at the returned point
    if (!have_grad_at_m) {
        TolGuard tg(P, kOuterRtol);
        P.gradient(m, u, p, g, &st);
        if (it <= HINV_NEWTON_MAXREC) info->gnorm[it] = nrm(c, n, g);
    }
    P.linearize(m, u, p);
    HINV_HIP(hipStreamSynchronize(c->stream));
    info->status = status;
    info->solves.status = st.converged ? HINV_OK : HINV_ENOCONV;
    info->solves.solves = st.solves;
    info->solves.iterations = st.iterations;
    info->solves.refinements = st.refinements;
    info->solves.fallbacks = st.fallbacks;
    info->solves.max_relres = st.max_relres;
    if (status == HINV_OK && !st.converged) status = HINV_ENOCONV;
    return status;
}

// ------------------------------------------------------- double pass ---
namespace {

// Orthonormal bases Z_j of span(Y_j) (the qr(Y) step of Algorithm 4) by
// shifted CholeskyQR3 (Fukaya, Kannan, Nakatsukasa, Zhang, Yamamoto 2020):
// one Cholesky QR on the Gram matrix shifted by 11 (n s + s (s+1)) u
// tr(Y^T Y), then two plain Cholesky QR passes.  Y_j is overwritten by Z_j.
bool orthonormalize(Ctx* c, DenseWork& w, int ni, int n, int s, double* Y, double* tmp, double* G,
                    double* Ri) {
    const size_t ts = (size_t)n * s, ss = (size_t)s * s;
    w.shift.ensure(ni);
    for (int pass = 0; pass < 3; ++pass) {
        for (int j = 0; j < ni; ++j) gram(c, w, n, s, s, Y + j * ts, n, Y + j * ts, n, G + j * ss, s);
        if (pass == 0)
            scaled_trace(c, ni, s, G, s, ss, 11.0 * ((double)n * s + (double)s * (s + 1)) * 1.1102230246251565e-16,
                         w.shift.get());
        if (!cholesky_upper(c, w, ni, s, G, s, ss, pass == 0 ? w.shift.get() : nullptr)) return false;
        tri_inverse_upper(c, w, ni, s, G, s, ss, Ri, s, ss);
        for (int j = 0; j < ni; ++j) {
            gemm_tall(c, n, s, s, 1.0, Y + j * ts, n, Ri + j * ss, s, 0.0, tmp + j * ts, n);
            dev_copy(c, n, s, tmp + j * ts, n, Y + j * ts, n);
        }
    }
    return true;
}

__global__ void k_scale_cols(int s, int r, const double* __restrict__ U, const double* __restrict__ g,
                             double* __restrict__ M) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s * r) return;
    const int col = i / s;
    M[i] = U[i] / sqrt(g[col]);
}

// qr(Y) of a block of numerical rank r < s (one instance): Y^T Y = U diag(g) U^T
// (descending), the r directions with g_i > tau g_1 kept, Z = Y U_r diag(g_r)^-1/2,
// then two Cholesky QR passes on the n x r block (its condition number is at
// most tau^-1/2).  tau = (10 rtol)^2: the solves that produced Y leave
// components of relative size rtol outside its exact range.  Returns r, 0 on
// failure.  Y <- Z (n x r, ld n).
int orthonormalize_rank(Ctx* c, DenseWork& w, int n, int s, double rtol, double* Y, double* tmp, double* G,
                        double* Ri, double* U, double* g) {
    const size_t ss = (size_t)s * s;
    gram(c, w, n, s, s, Y, n, Y, n, G, s);
    sym_eig(c, w, 1, s, G, s, ss, U, s, ss, g, s);
    std::vector<double> hg(s);
    HINV_HIP(hipMemcpyAsync(hg.data(), g, sizeof(double) * s, hipMemcpyDeviceToHost, c->stream));
    HINV_HIP(hipStreamSynchronize(c->stream));
    if (!(hg[0] > 0.0)) return 0;
    const double tau = std::max(1e-24, 100.0 * rtol * rtol);
    int r = 0;
    while (r < s && hg[r] > tau * hg[0]) ++r;
    k_scale_cols<<<ceil_div(s * r, kBlock), kBlock, 0, c->stream>>>(s, r, U, g, Ri);
    HINV_LAUNCH_CHECK();
    gemm_tall(c, n, s, r, 1.0, Y, n, Ri, s, 0.0, tmp, n);
    dev_copy(c, n, r, tmp, n, Y, n);
    const size_t rr = (size_t)r * r;
    for (int pass = 0; pass < 2; ++pass) {
        gram(c, w, n, r, r, Y, n, Y, n, G, r);
        if (!cholesky_upper(c, w, 1, r, G, r, rr, nullptr)) return 0;
        tri_inverse_upper(c, w, 1, r, G, r, rr, Ri, r, rr);
        gemm_tall(c, n, r, r, 1.0, Y, n, Ri, r, 0.0, tmp, n);
        dev_copy(c, n, r, tmp, n, Y, n);
    }
    return r;
}

}  // namespace

// PreCholQR (Algorithm 4) on each Y_j (n x s): Z = qr(Y), Zbar = B Z,
// R_Z = chol(Z^T Zbar), Q = Z R_Z^-1 written to Q_j.  Y_j is overwritten by
// Z_j; Zb is scratch.
int precholqr(Problem* const* P, int ni, DenseWork& dw, int s, double* Y, double* Zb, double* Q, double* G,
              double* Ri, bool b_identity, int* rank, double* U, double* g) {
    Ctx* c = P[0]->ctx;
    const int n = P[0]->n;
    const bool revealing = rank && ni == 1 && U && g;
    if (rank) *rank = s;
    // a copy of Y for the rank-revealing retry (Zb is not needed before Z exists)
    if (revealing) dev_copy(c, n, s, Y, n, Zb, n);
    if (!orthonormalize(c, dw, ni, n, s, Y, Q, G, Ri)) {  // Y <- Z
        if (!revealing) return HINV_EBREAK;
        dev_copy(c, n, s, Zb, n, Y, n);
        const int r = orthonormalize_rank(c, dw, n, s, P[0]->rtol, Y, Q, G, Ri, U, g);
        if (r == 0) return HINV_EBREAK;
        *rank = r;
        s = r;
    }
    const size_t ts = (size_t)n * s, ss = (size_t)s * s;
    for (int j = 0; j < ni; ++j) {
        if (b_identity)
            dev_copy(c, n, s, Y + j * ts, n, Zb + j * ts, n);                      // Zbar = Z
        else
            P[j]->prior_apply(s, Y + j * ts, n, Zb + j * ts, n);                   // Zbar = B Z
        gram(c, dw, n, s, s, Y + j * ts, n, Zb + j * ts, n, G + j * ss, s);      // Z^T Zbar
    }
    if (!cholesky_upper(c, dw, ni, s, G, s, ss)) return HINV_EBREAK;            // R_Z
    tri_inverse_upper(c, dw, ni, s, G, s, ss, Ri, s, ss);
    for (int j = 0; j < ni; ++j)
        gemm_tall(c, n, s, s, 1.0, Y + j * ts, n, Ri + j * ss, s, 0.0, Q + j * ts, n);  // Q = Z R_Z^-1
    return HINV_OK;
}

// Rayleigh-Ritz step of Algorithm 2: T = Q^T (A Q), T = S Lambda S^T (descending),
// V = Q S_k, Lambda_k to the host (synchronizes the stream).
void rayleigh_ritz(Problem* const* P, int ni, DenseWork& dw, int s, int k, int tprod, const double* Q,
                   const double* AQ, double* T, double* S, double* lam, double* const* V, int ldv,
                   double* const* lambda_host) {
    Ctx* c = P[0]->ctx;
    const int n = P[0]->n;
    const size_t ts = (size_t)n * s, ss = (size_t)s * s;
    for (int j = 0; j < ni; ++j)
        gram(c, dw, n, s, s, Q + j * ts, n, AQ + j * ts, n, T + j * ss, s, tprod == HINV_TPROD_BF16);
    sym_eig(c, dw, ni, s, T, s, ss, S, s, ss, lam, s);
    for (int j = 0; j < ni; ++j) {
        gemm_tall(c, n, s, k, 1.0, Q + j * ts, n, S + j * ss, s, 0.0, V[j], ldv);
        HINV_HIP(hipMemcpyAsync(lambda_host[j], lam + (size_t)j * s, sizeof(double) * k, hipMemcpyDeviceToHost,
                                c->stream));
    }
    HINV_HIP(hipStreamSynchronize(c->stream));
}

int lowrank_eig(Problem& P, int mode, int tprod, int s, const double* omega, int ldo, int k,
                double* lambda_host, double* V, int ldv, SolveStats* st) {
    const int n = P.n;
    P.ws_big.ensure((size_t)n * s * 3);
    P.ws_small.ensure((size_t)s * s * 4 + s);
    double* Y = P.ws_big.get();
    double* Zb = Y + (size_t)n * s;
    double* W = Zb + (size_t)n * s;
    double* G = P.ws_small.get();
    double* Ri = G + (size_t)s * s;
    double* T = Ri + (size_t)s * s;
    double* S = T + (size_t)s * s;
    double* lam = S + (size_t)s * s;
    DenseWork& dw = P.dw;
    // pass 1: Ybar = A Omega, Y = B^-1 Ybar  (A = H_misfit, B = R)
    P.hessian(mode, s, omega, ldo, W, n, st);
    P.prior_solve(s, W, n, Y, n, st);
    Problem* const pp = &P;
    int r = s;  // numerical rank of Y: below s when A has lower rank than the probe count
    const int rc = precholqr(&pp, 1, dw, s, Y, Zb, W, G, Ri, false, &r, T, lam);  // Q in W (n x r)
    if (rc != HINV_OK) return rc;
    if (r < k) return HINV_EBREAK;
    // pass 2: T = Q^T A Q
    P.hessian(mode, r, W, n, Zb, n, st);
    rayleigh_ritz(&pp, 1, dw, r, k, tprod, W, Zb, T, S, lam, &V, ldv, &lambda_host);
    return HINV_OK;
}

// ------------------------------------------------------- single pass ---
// Algorithm 3: one pass of A over Omega.  PreCholQR of Y = B^-1 A Omega gives
// Q and Qbar = B Q; T is the least-squares solution over symmetric matrices of
// T W = Z with W = Qbar^T Omega, Z = Qbar^T Y (Eq. eq:Tsinglepass).  Its
// normal equations T G + G T = C with G = W W^T, C = Z W^T + W Z^T are solved
// in the eigenbasis of G = U diag(g) U^T: (U^T T U)_ij = (U^T C U)_ij / (g_i + g_j).
int lowrank_eig_single(Problem& P, int mode, int s, const double* omega, int ldo, int k,
                       double* lambda_host, double* V, int ldv, SolveStats* st) {
    Ctx* c = P.ctx;
    const int n = P.n;
    const size_t ts = (size_t)n * s, ss = (size_t)s * s;
    P.ws_big.ensure(ts * 5);
    P.ws_small.ensure(ss * 9 + 2 * (size_t)s);
    double* Yb = P.ws_big.get();  // A Omega, later Qbar
    double* Y = Yb + ts;         // B^-1 A Omega, overwritten by Z
    double* Yk = Y + ts;         // B^-1 A Omega, kept
    double* Zb = Yk + ts;        // B Z
    double* Q = Zb + ts;
    double* G = P.ws_small.get();
    double* Ri = G + ss;
    double* Wm = Ri + ss;
    double* Zm = Wm + ss;
    double* Cm = Zm + ss;
    double* U = Cm + ss;
    double* Tm = U + ss;
    double* S = Tm + ss;
    double* tmp = S + ss;
    double* g = tmp + ss;
    double* lam = g + s;
    DenseWork& dw = P.dw;
    P.hessian(mode, s, omega, ldo, Yb, n, st);       // Ybar = A Omega
    P.prior_solve(s, Yb, n, Y, n, st);                // Y = B^-1 Ybar
    dev_copy(c, n, s, Y, n, Yk, n);
    Problem* const pp = &P;
    const int rc = precholqr(&pp, 1, dw, s, Y, Zb, Q, G, Ri);  // Q; Zb = B Z; Ri = R_Z^-1
    if (rc != HINV_OK) return rc;
    gemm_tall(c, n, s, s, 1.0, Zb, n, Ri, s, 0.0, Yb, n);        // Qbar = B Z R_Z^-1 = B Q
    gram(c, dw, n, s, s, Yb, n, omega, ldo, Wm, s);              // W = Qbar^T Omega
    gram(c, dw, n, s, s, Yb, n, Yk, n, Zm, s);                   // Z = Qbar^T Y
    small_gemm(c, false, true, s, s, s, 1.0, Wm, s, Wm, s, 0.0, G, s);    // G = W W^T
    small_gemm(c, false, true, s, s, s, 1.0, Zm, s, Wm, s, 0.0, Cm, s);   // C = Z W^T
    small_gemm(c, false, true, s, s, s, 1.0, Wm, s, Zm, s, 1.0, Cm, s);   //   + W Z^T
    sym_eig(c, dw, 1, s, G, s, ss, U, s, ss, g, s);                       // G = U diag(g) U^T
    small_gemm(c, false, false, s, s, s, 1.0, Cm, s, U, s, 0.0, tmp, s);  // C U
    small_gemm(c, true, false, s, s, s, 1.0, U, s, tmp, s, 0.0, Tm, s);   // U^T C U
    sylvester_diag(c, s, g, Tm, s);                                       // / (g_i + g_j)
    small_gemm(c, false, false, s, s, s, 1.0, U, s, Tm, s, 0.0, tmp, s);  // U X
    small_gemm(c, false, true, s, s, s, 1.0, tmp, s, U, s, 0.0, Tm, s);   // T = U X U^T
    sym_eig(c, dw, 1, s, Tm, s, ss, S, s, ss, lam, s);
    gemm_tall(c, n, s, k, 1.0, Q, n, S, s, 0.0, V, ldv);                  // V = Q S_k
    HINV_HIP(hipMemcpyAsync(lambda_host, lam, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
    HINV_HIP(hipStreamSynchronize(c->stream));
    return HINV_OK;
}

// ----------------------------------------------------- pointwise variance ---
namespace {
__global__ void k_post_var_weight(int k, const double* __restrict__ lam, double* __restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) w[i] = -lam[i] / (1.0 + lam[i]);
}
}  // namespace

// Eq. eq:prior_mvar: Algorithm 2 with A = R^-1, B = I and no oversampling
// (s probe vectors, s eigenpairs (mu, vbar)), diag(R^-1) ~ sum mu_i vbar_i^2.
int prior_variance(Problem& P, int s, const double* omega, int ldo, double* diag, double* mu_host,
                   SolveStats* st) {
    Ctx* c = P.ctx;
    const int n = P.n;
    const size_t ts = (size_t)n * s, ss = (size_t)s * s;
    P.ws_big.ensure(ts * 4);
    P.ws_small.ensure(ss * 4 + s);
    double* Y = P.ws_big.get();
    double* Zb = Y + ts;
    double* Q = Zb + ts;
    double* Vb = Q + ts;
    double* G = P.ws_small.get();
    double* Ri = G + ss;
    double* T = Ri + ss;
    double* S = T + ss;
    double* mu = S + ss;
    DenseWork& dw = P.dw;
    P.prior_solve(s, omega, ldo, Y, n, st);                   // Y = R^-1 Omega (B = I)
    Problem* const pp = &P;
    const int rc = precholqr(&pp, 1, dw, s, Y, Zb, Q, G, Ri, /*b_identity=*/true);
    if (rc != HINV_OK) return rc;
    P.prior_solve(s, Q, n, Zb, n, st);                        // R^-1 Q
    gram(c, dw, n, s, s, Q, n, Zb, n, T, s);                  // T = Q^T R^-1 Q
    sym_eig(c, dw, 1, s, T, s, ss, S, s, ss, mu, s);
    gemm_tall(c, n, s, s, 1.0, Q, n, S, s, 0.0, Vb, n);       // vbar = Q S
    weighted_squares(c, n, s, Vb, n, mu, nullptr, diag);
    if (mu_host) HINV_HIP(hipMemcpyAsync(mu_host, mu, sizeof(double) * s, hipMemcpyDeviceToHost, c->stream));
    HINV_HIP(hipStreamSynchronize(c->stream));
    return HINV_OK;
}

// Eq. eq:post_mvar: diag = prior_diag - sum lambda_i / (1 + lambda_i) v_i^2.
void posterior_variance(Problem& P, const double* prior_diag, int k, const double* lambda_host, const double* V,
                        int ldv, double* diag) {
    Ctx* c = P.ctx;
    P.ws_small.ensure(2 * (size_t)std::max(k, 1));
    double* lam = P.ws_small.get();
    double* w = lam + std::max(k, 1);
    if (k > 0) {
        HINV_HIP(hipMemcpyAsync(lam, lambda_host, sizeof(double) * k, hipMemcpyHostToDevice, c->stream));
        k_post_var_weight<<<ceil_div(k, 256), 256, 0, c->stream>>>(k, lam, w);
        HINV_LAUNCH_CHECK();
    }
    weighted_squares(c, P.n, k, V, ldv, w, prior_diag, diag);
    HINV_HIP(hipStreamSynchronize(c->stream));
}

// ------------------------------------------------------ posterior sample ---
namespace {

// Device state of the low-rank update y = x - V S V^T R x shared by the
// samples of one call: W = R V (n x k, in ws_big) and the scales
// S = 1 - (1 + lambda)^-1/2 (k, in ws_small after the k x ns coefficients).
struct LowRankUpdate {
    const double* W = nullptr;
    double* C = nullptr;
    const double* sc = nullptr;
};

LowRankUpdate prepare_update(Problem& P, int k, const double* lambda_host, const double* V, int ldv, int ns) {
    Ctx* c = P.ctx;
    const int n = P.n;
    LowRankUpdate u;
    if (k == 0) return u;
    P.ws_big.ensure((size_t)n * k);
    P.ws_small.ensure((size_t)k * ns + 2 * (size_t)k);
    double* W = P.ws_big.get();
    double* C = P.ws_small.get();
    double* lam = C + (size_t)k * ns;
    double* sc = lam + k;
    P.prior_apply(k, V, ldv, W, n);  // W = R V, once for every sample of the call
    HINV_HIP(hipMemcpyAsync(lam, lambda_host, sizeof(double) * k, hipMemcpyHostToDevice, c->stream));
    k_post_scale<<<ceil_div(k, 256), 256, 0, c->stream>>>(k, lam, sc);
    HINV_LAUNCH_CHECK();
    u.W = W;
    u.C = C;
    u.sc = sc;
    return u;
}

// out[:, j] = m_map + x_j - V S V^T R x_j for the ns prior draws x_j in out.
void apply_update(Problem& P, const LowRankUpdate& u, const double* m_map, int k, const double* V, int ldv,
                  int ns, double* out, int ldo) {
    Ctx* c = P.ctx;
    const int n = P.n;
    if (k > 0) {
        gram(c, P.dw, n, k, ns, u.W, n, out, ldo, u.C, k);           // W^T x = V^T R x
        scale_rows(c, k, ns, u.sc, u.C, k);                          // S V^T R x
        gemm_tall(c, n, k, ns, -1.0, V, ldv, u.C, k, 1.0, out, ldo);  // x - V S V^T R x
    }
    k_add_vec<<<dim3(ceil_div(n, 256), ns), 256, 0, c->stream>>>(n, m_map, out, ldo);
    HINV_LAUNCH_CHECK();
}

}  // namespace

void posterior_sample(Problem& P, const double* m_map, int k, const double* lambda_host,
                      const double* V, int ldv, int ns, const double* eta, int ldeta, double* out,
                      int ldo, SolveStats* st) {
    // x = K_A^-1 C_M eta (zero-mean prior draws)
    P.prior_sample(ns, eta, ldeta, out, ldo, false, st);
    const LowRankUpdate u = prepare_update(P, k, lambda_host, V, ldv, ns);
    apply_update(P, u, m_map, k, V, ldv, ns, out, ldo);
    HINV_HIP(hipStreamSynchronize(P.ctx->stream));
}

void posterior_sample_seeded(Problem& P, const double* m_map, int k, const double* lambda_host, const double* V,
                             int ldv, uint64_t seed, uint64_t stream, long long first, int ns, double* out, int ldo,
                             SolveStats* st) {
    const int chunk = std::min(ns, kSampleChunk);
    const size_t L = (size_t)6 * P.N * P.N;
    P.ws_eta.ensure(L * chunk);
    const LowRankUpdate u = prepare_update(P, k, lambda_host, V, ldv, chunk);
    for (int s0 = 0; s0 < ns; s0 += chunk) {
        const int cnt = std::min(chunk, ns - s0);
        double* o = out + (size_t)s0 * ldo;
        P.white_noise(seed, stream, first + s0, cnt, P.ws_eta.get(), (int)L);
        P.prior_sample(cnt, P.ws_eta.get(), (int)L, o, ldo, false, st);
        apply_update(P, u, m_map, k, V, ldv, cnt, o, ldo);
    }
    HINV_HIP(hipStreamSynchronize(P.ctx->stream));
}

}  // namespace hinv
