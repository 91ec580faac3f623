// Batched multigrid-preconditioned conjugate gradients on the structured mesh.
//
// Every state-equation solve of the method (forward, adjoint, incremental
// forward and adjoint -- each Hessian action needs two, App. A) and every
// prior solve K_A^{-1} runs through Hierarchy::solve:
//
//   * operators: the five-point state stiffness A(m) (Dirichlet rows j = 0, N
//     removed) or the seven-point prior operator K_A (all nodes);
//   * preconditioner: one V-cycle of geometric multigrid on the nested
//     right-diagonal meshes N, N/2, ..., <= 8.  Coarse state operators use
//     the mean of the four child triangle coefficients, which makes them equal
//     to the Galerkin products P^T A P with P1 interpolation P; the prior
//     operator has constant coefficients and its rediscretization is Galerkin
//     as well.  Smoothing: degree-2 Chebyshev on the Jacobi-scaled operator
//     over [0.5, 2], pre and post (symmetric, so the V-cycle is an SPD
//     preconditioner).  The coarsest level is solved with a dense inverse.
//   * columns: all right-hand sides of a call advance together; every kernel
//     takes blockIdx.y as the column and skips columns that have converged.
//   * precision: the outer loop is FP64 iterative refinement,
//     r = b - A x in FP64, inner PCG in FP64 or FP32 on r / |r|, x += |r| d,
//     until |r| <= rtol |b| per column.
#include <cstdio>
#include <cstdlib>

#include "grid.h"
#include "solver.h"

namespace hinv {

namespace {

// Chebyshev degree-2 constants for the interval [kChebLo, kChebHi].
struct Cheb {
    double theta, delta, rho0, rho1;
    Cheb() {
        theta = 0.5 * (kChebHi + kChebLo);
        delta = 0.5 * (kChebHi - kChebLo);
        const double sigma = theta / delta;
        rho0 = 1.0 / sigma;
        rho1 = 1.0 / (2.0 * sigma - rho0);
    }
};

inline dim3 grid2(int n, int nc) { return dim3(ceil_div(n, kBlock), nc); }

template <typename T>
__device__ inline T* col(T* p, int ld) {
    return p + (size_t)blockIdx.y * ld;
}
template <typename T>
__device__ inline const T* col(const T* p, int ld) {
    return p + (size_t)blockIdx.y * ld;
}

// ------------------------------------------------------ coefficient setup ---
__global__ void k_coef_fine(int N, const double* __restrict__ m, double* __restrict__ cT) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * N * N) return;
    const int cell = t >> 1, s = t & 1;
    const int ci = cell % N, cj = cell / N;
    int ka, kr, kb;
    tri_nodes(N, ci, cj, s, ka, kr, kb);
    cT[t] = exp((m[ka] + m[kr] + m[kb]) * (1.0 / 3.0));
}

// Coarse triangle coefficient = mean of its four children.
__global__ void k_coarsen(int Nc, const double* __restrict__ cf, double* __restrict__ cc) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * Nc * Nc) return;
    const int cell = t >> 1, s = t & 1;
    const int I = cell % Nc, J = cell / Nc;
    const int Nf = 2 * Nc;
    auto tf = [&](int ci, int cj, int ss) { return cf[2 * (cj * Nf + ci) + ss]; };
    double v;
    if (s == 0)
        v = tf(2 * I, 2 * J, 0) + tf(2 * I + 1, 2 * J, 0) + tf(2 * I + 1, 2 * J, 1) +
            tf(2 * I + 1, 2 * J + 1, 0);
    else
        v = tf(2 * I, 2 * J, 1) + tf(2 * I, 2 * J + 1, 1) + tf(2 * I, 2 * J + 1, 0) +
            tf(2 * I + 1, 2 * J + 1, 1);
    cc[t] = 0.25 * v;
}

__global__ void k_weights(int N, const double* __restrict__ cT, double* wE64, double* wN64,
                          double* dinv64, float* wE32, float* wN32, float* dinv32) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int N1 = N + 1;
    if (k >= N1 * N1) return;
    const int i = k % N1, j = k / N1;
    auto cL = [&](int ci, int cj) {
        return (ci >= 0 && ci < N && cj >= 0 && cj < N) ? cT[2 * (cj * N + ci)] : 0.0;
    };
    auto cU = [&](int ci, int cj) {
        return (ci >= 0 && ci < N && cj >= 0 && cj < N) ? cT[2 * (cj * N + ci) + 1] : 0.0;
    };
    const double wE = i < N ? 0.5 * (cL(i, j) + cU(i, j - 1)) : 0.0;
    const double wN = j < N ? 0.5 * (cU(i, j) + cL(i - 1, j)) : 0.0;
    const double wW = i > 0 ? 0.5 * (cL(i - 1, j) + cU(i - 1, j - 1)) : 0.0;
    const double wS = j > 0 ? 0.5 * (cU(i, j - 1) + cL(i - 1, j - 1)) : 0.0;
    const bool fr = j > 0 && j < N;
    const double di = fr ? 1.0 / (wE + wN + wW + wS) : 0.0;
    wE64[k] = wE;
    wN64[k] = wN;
    dinv64[k] = di;
    wE32[k] = (float)wE;
    wN32[k] = (float)wN;
    dinv32[k] = (float)di;
}

// ------------------------------------------------------------ operators ---
template <typename T, class Op>
__global__ void k_apply(Op op, const T* __restrict__ x, int ldx, T* __restrict__ y, int ldy,
                        const int* __restrict__ act, double* __restrict__ partial) {
    if (act && !act[blockIdx.y]) return;
    const int N = op.N, N1 = N + 1, n = N1 * N1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const T* xc = col(x, ldx);
    T* yc = col(y, ldy);
    double dot = 0.0;
    if (k < n) {
        const int i = k % N1, j = k / N1;
        T v = 0;
        if (op.is_free(i, j)) v = op.apply(i, j, k, [&](int, int, int kk) { return xc[kk]; });
        yc[k] = v;
        dot = (double)v * (double)xc[k];
    }
    if (partial) {
        const double s = block_sum(dot);
        if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

// Pre-smoothing from a zero initial guess (two Chebyshev steps in one pass):
// d0 = D^-1 b / theta, r1 = b - A d0, x = (1 + rho1 rho0) d0 + (2 rho1 / delta) D^-1 r1.
template <typename T, class Op>
__global__ void k_smooth_pre(Op op, const T* __restrict__ b, T* __restrict__ x, int ld,
                             const int* __restrict__ act, T cA, T cB, T inv_theta) {
    if (act && !act[blockIdx.y]) return;
    const int N = op.N, N1 = N + 1, n = N1 * N1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int i = k % N1, j = k / N1;
    const T* bc = col(b, ld);
    T* xc = col(x, ld);
    if (!op.is_free(i, j)) {
        xc[k] = 0;
        return;
    }
    auto d0 = [&](int ii, int jj, int kk) { return op.inv_diag(ii, jj, kk) * bc[kk] * inv_theta; };
    const T dk = d0(i, j, k);
    const T r1 = bc[k] - op.apply(i, j, k, d0);
    xc[k] = cA * dk + cB * op.inv_diag(i, j, k) * r1;
}

template <typename T, class Op>
__global__ void k_residual(Op op, const T* __restrict__ b, const T* __restrict__ x,
                           T* __restrict__ r, int ld, const int* __restrict__ act) {
    if (act && !act[blockIdx.y]) return;
    const int N = op.N, N1 = N + 1, n = N1 * N1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int i = k % N1, j = k / N1;
    const T* bc = col(b, ld);
    const T* xc = col(x, ld);
    T v = 0;
    if (op.is_free(i, j)) v = bc[k] - op.apply(i, j, k, [&](int, int, int kk) { return xc[kk]; });
    col(r, ld)[k] = v;
}

// Restriction P^T: coarse node (I,J) gathers fine (2I,2J) with weight 1 and its
// six P1 neighbours (2I+-1,2J), (2I,2J+-1), (2I+1,2J+1), (2I-1,2J-1) with 1/2.
template <typename T>
__global__ void k_restrict(int Nc, const T* __restrict__ rf, int ldf, T* __restrict__ bc,
                           int ldc, int dirichlet, const int* __restrict__ act) {
    if (act && !act[blockIdx.y]) return;
    const int Nc1 = Nc + 1, nc = Nc1 * Nc1;
    const int K = blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    const int I = K % Nc1, J = K / Nc1;
    T* out = col(bc, ldc);
    if (dirichlet && (J == 0 || J == Nc)) {
        out[K] = 0;
        return;
    }
    const int Nf = 2 * Nc, Nf1 = Nf + 1;
    const T* f = col(rf, ldf);
    const int i = 2 * I, j = 2 * J, k = j * Nf1 + i;
    T s = 0;
    if (i > 0) s += f[k - 1];
    if (i < Nf) s += f[k + 1];
    if (j > 0) s += f[k - Nf1];
    if (j < Nf) s += f[k + Nf1];
    if (i < Nf && j < Nf) s += f[k + Nf1 + 1];
    if (i > 0 && j > 0) s += f[k - Nf1 - 1];
    out[K] = f[k] + (T)0.5 * s;
}

// x_fine += P x_coarse (P1 interpolation on the nested meshes).
template <typename T>
__global__ void k_prolong_add(int Nc, const T* __restrict__ xc, int ldc, T* __restrict__ xf,
                              int ldf, int dirichlet, const int* __restrict__ act) {
    if (act && !act[blockIdx.y]) return;
    const int Nf = 2 * Nc, Nf1 = Nf + 1, nf = Nf1 * Nf1, Nc1 = Nc + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nf) return;
    const int i = k % Nf1, j = k / Nf1;
    if (dirichlet && (j == 0 || j == Nf)) return;
    const T* c = col(xc, ldc);
    T v;
    const int I = i >> 1, J = j >> 1;
    if (!(i & 1) && !(j & 1))
        v = c[J * Nc1 + I];
    else if (!(j & 1))
        v = (T)0.5 * (c[J * Nc1 + I] + c[J * Nc1 + I + 1]);
    else if (!(i & 1))
        v = (T)0.5 * (c[J * Nc1 + I] + c[(J + 1) * Nc1 + I]);
    else
        v = (T)0.5 * (c[J * Nc1 + I] + c[(J + 1) * Nc1 + I + 1]);
    col(xf, ldf)[k] += v;
}

// Post-smoothing, first Chebyshev step: r0 = b - A x, d0 = D^-1 r0 / theta, x += d0; t = d0.
template <typename T, class Op>
__global__ void k_post1(Op op, const T* __restrict__ b, T* __restrict__ x, T* __restrict__ t,
                        int ld, const int* __restrict__ act, T inv_theta) {
    if (act && !act[blockIdx.y]) return;
    const int N = op.N, N1 = N + 1, n = N1 * N1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int i = k % N1, j = k / N1;
    const T* bc = col(b, ld);
    const T* xc = col((const T*)x, ld);
    T d = 0;
    if (op.is_free(i, j)) {
        const T r0 = bc[k] - op.apply(i, j, k, [&](int, int, int kk) { return xc[kk]; });
        d = op.inv_diag(i, j, k) * r0 * inv_theta;
    }
    col(t, ld)[k] = d;
}

// Second step (x still holds the value before the first step): r1 = r0 - A d0 with
// r0 = theta D d0, x2 = x + d0 + rho1 rho0 d0 + (2 rho1/delta) D^-1 r1.
// Optionally accumulates sum_k rv_k x_k per column (r^T z of the PCG).
template <typename T, class Op>
__global__ void k_post2(Op op, T* __restrict__ x, const T* __restrict__ t, int ld,
                        const int* __restrict__ act, T theta, T c1, T c2,
                        const T* __restrict__ rv, double* __restrict__ partial) {
    if (act && !act[blockIdx.y]) return;
    const int N = op.N, N1 = N + 1, n = N1 * N1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const T* tc = col(t, ld);
    T* xc = col(x, ld);
    double dot = 0.0;
    if (k < n) {
        const int i = k % N1, j = k / N1;
        if (op.is_free(i, j)) {
            const T dk = tc[k];
            const T di = op.inv_diag(i, j, k);
            const T r0 = theta * dk / di;
            const T r1 = r0 - op.apply(i, j, k, [&](int, int, int kk) { return tc[kk]; });
            const T v = xc[k] + ((T)1 + c1) * dk + c2 * di * r1;
            xc[k] = v;
            if (rv) dot = (double)v * (double)col(rv, ld)[k];
        }
    }
    if (partial) {
        const double s = block_sum(dot);
        if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

// ------------------------------------------------------------- coarse ---
// Dense matrix of the coarsest operator; Dirichlet rows/columns become identity.
template <class Op>
__global__ void k_coarse_matrix(Op op, double* __restrict__ M) {
    const int N1 = op.N + 1, n = N1 * N1;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n * n) return;
    const int row = id / n, c = id % n;
    const int i = row % N1, j = row / N1;
    const int ic = c % N1, jc = c / N1;
    double v;
    if (!op.is_free(i, j) || !op.is_free(ic, jc))
        v = (row == c) ? 1.0 : 0.0;
    else
        v = op.apply(i, j, row, [&](int, int, int kk) { return kk == c ? 1.0 : 0.0; });
    M[id] = v;
}

// In-place Gauss-Jordan inversion of an SPD matrix (no pivoting), one workgroup.
// Pivot step p:  a = M[p][p];  M[i][j] -= M[i][p] M[p][j] / a (i, j != p);
// M[p][j] /= a;  M[i][p] = -M[i][p] / a;  M[p][p] = 1 / a.
__global__ void k_gauss_jordan(int n, double* __restrict__ M) {
    extern __shared__ double sm[];
    double* A = sm;            // n*n
    double* rowp = sm + n * n;  // n
    double* colp = rowp + n;    // n
    for (int id = threadIdx.x; id < n * n; id += blockDim.x) A[id] = M[id];
    __syncthreads();
    for (int p = 0; p < n; ++p) {
        for (int id = threadIdx.x; id < n; id += blockDim.x) {
            rowp[id] = A[p * n + id];
            colp[id] = A[id * n + p];
        }
        __syncthreads();
        const double a = rowp[p];
        const double ia = 1.0 / a;
        for (int id = threadIdx.x; id < n * n; id += blockDim.x) {
            const int i = id / n, j = id % n;
            double v;
            if (i == p && j == p)
                v = ia;
            else if (i == p)
                v = rowp[j] * ia;
            else if (j == p)
                v = -colp[i] * ia;
            else
                v = A[id] - colp[i] * rowp[j] * ia;
            A[id] = v;
        }
        __syncthreads();
    }
    for (int id = threadIdx.x; id < n * n; id += blockDim.x) M[id] = A[id];
}

__global__ void k_cast_d2f(const double* a, float* b, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) b[k] = (float)a[k];
}

// x = Cinv b for the coarsest level, one workgroup per column.
template <typename T>
__global__ void k_coarse_solve(int nc, const T* __restrict__ cinv, const T* __restrict__ b,
                               T* __restrict__ x, int ld, const int* __restrict__ act) {
    if (act && !act[blockIdx.y]) return;
    __shared__ T bs[128];
    const T* bc = col(b, ld);
    for (int k = threadIdx.x; k < nc; k += blockDim.x) bs[k] = bc[k];
    __syncthreads();
    for (int r = threadIdx.x; r < nc; r += blockDim.x) {
        T s = 0;
        for (int c = 0; c < nc; ++c) s += cinv[r * nc + c] * bs[c];
        col(x, ld)[r] = s;
    }
}

// ------------------------------------------------------------------ PCG ---
// p = z + beta p (beta = 0 on the first iteration).
template <typename T>
__global__ void k_update_p(const T* __restrict__ z, T* __restrict__ p, int ld, int n,
                           const int* __restrict__ act, const ColState* __restrict__ st,
                           int first) {
    if (!act[blockIdx.y]) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    T* pc = col(p, ld);
    // p is not read on the first iteration: it may hold stale values
    pc[k] = first ? col(z, ld)[k] : col(z, ld)[k] + (T)st[blockIdx.y].beta * pc[k];
}

// x += alpha p; r -= alpha q; partial |r|^2.
template <typename T>
__global__ void k_update_xr(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                            const T* __restrict__ q, int ld, int n, const int* __restrict__ act,
                            const ColState* __restrict__ st, double* __restrict__ partial) {
    if (!act[blockIdx.y]) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0;
    if (k < n) {
        const T a = (T)st[blockIdx.y].alpha;
        col(x, ld)[k] += a * col(p, ld)[k];
        const T rv = col(r, ld)[k] - a * col(q, ld)[k];
        col(r, ld)[k] = rv;
        rr = (double)rv * (double)rv;
    }
    const double s = block_sum(rr);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

template <typename T>
__global__ void k_dot(const T* __restrict__ a, const T* __restrict__ b, int ld, int n,
                      const int* __restrict__ act, double* __restrict__ partial) {
    if (act && !act[blockIdx.y]) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (k < n) v = (double)col(a, ld)[k] * (double)col(b, ld)[k];
    const double s = block_sum(v);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

template <typename T>
__global__ void k_zero(T* x, int ld, int n, const int* __restrict__ act) {
    if (act && !act[blockIdx.y]) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) col(x, ld)[k] = 0;
}

// Column sums of the partials of one reduction, one workgroup per column.
__device__ inline double column_total(const double* partial, int nblk) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += partial[(size_t)blockIdx.x * nblk + b];
    return block_sum(v);
}

enum FinKind { kFinRz0 = 0, kFinRz = 1, kFinAlpha = 2, kFinRr = 3 };

__global__ void k_finalize(int kind, const double* __restrict__ partial, int nblk,
                           ColState* __restrict__ st, int* __restrict__ act) {
    if (!act[blockIdx.x]) return;
    const double s = column_total(partial, nblk);
    if (threadIdx.x != 0) return;
    ColState& c = st[blockIdx.x];
    switch (kind) {
        case kFinRz0:
            c.rz = s;
            c.beta = 0.0;
            break;
        case kFinRz:
            c.beta = s / c.rz;
            c.rz = s;
            break;
        case kFinAlpha:
            c.pq = s;
            c.alpha = s > 0.0 ? c.rz / s : 0.0;
            if (!(s > 0.0)) act[blockIdx.x] = 0;  // breakdown: stop this column
            break;
        case kFinRr:
            c.rr = s;
            if (s <= c.tol2 * c.bb) act[blockIdx.x] = 0;
            break;
    }
}

// --------------------------------------------------- FP64 refinement loop ---
// r64 = masked b, x64 = 0, partial |r64|^2.
template <class Op>
__global__ void k_ir_init(Op op, const double* __restrict__ b, int ldb, double* __restrict__ x64,
                          double* __restrict__ r64, int ld, double* __restrict__ partial) {
    const int N1 = op.N + 1, n = N1 * N1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double v2 = 0.0;
    if (k < n) {
        const int i = k % N1, j = k / N1;
        const double v = op.is_free(i, j) ? col(b, ldb)[k] : 0.0;
        col(r64, ld)[k] = v;
        col(x64, ld)[k] = 0.0;
        v2 = v * v;
    }
    const double s = block_sum(v2);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// r64 = b - A x64 on active columns, partial |r64|^2.
template <class Op>
__global__ void k_ir_residual(Op op, const double* __restrict__ b, int ldb,
                              const double* __restrict__ x64, double* __restrict__ r64, int ld,
                              const int* __restrict__ act, double* __restrict__ partial) {
    if (!act[blockIdx.y]) return;
    const int N1 = op.N + 1, n = N1 * N1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double v2 = 0.0;
    if (k < n) {
        const int i = k % N1, j = k / N1;
        double v = 0.0;
        if (op.is_free(i, j)) {
            const double* xc = col(x64, ld);
            v = col(b, ldb)[k] - op.apply(i, j, k, [&](int, int, int kk) { return xc[kk]; });
        }
        col(r64, ld)[k] = v;
        v2 = v * v;
    }
    const double s = block_sum(v2);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// Outer bookkeeping per column.  first: bb = s (|b|^2).  Always: rr = s;
// column stays active while rr > rtol^2 bb; colnorm = |r|; inner tolerance.
__global__ void k_ir_finalize(int first, const double* __restrict__ partial, int nblk,
                              ColState* __restrict__ st, int* __restrict__ oact,
                              double* __restrict__ colnorm, double rtol, double tol_floor) {
    if (!first && !oact[blockIdx.x]) return;
    const double s = column_total(partial, nblk);
    if (threadIdx.x != 0) return;
    ColState& c = st[blockIdx.x];
    if (first) c.obb = s;
    c.rr = s;
    const bool a = s > rtol * rtol * c.obb && s > 0.0;
    oact[blockIdx.x] = a ? 1 : 0;
    colnorm[blockIdx.x] = sqrt(s);
    if (a) {
        // inner target: the remaining factor to rtol |b|, with margin, floored
        double t = 0.5 * rtol * sqrt(c.obb / s);
        if (t < tol_floor) t = tol_floor;
        c.tol2 = t * t;  // relative to the inner right-hand side (unit norm)
    }
}

// Inner right-hand side r / |r| in precision T; zero initial guess.
template <typename T>
__global__ void k_ir_scale(const double* __restrict__ r64, T* __restrict__ r, T* __restrict__ x,
                           int ld, int n, const int* __restrict__ oact,
                           const double* __restrict__ colnorm) {
    if (!oact[blockIdx.y]) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double s = 1.0 / colnorm[blockIdx.y];
    col(r, ld)[k] = (T)(col(r64, ld)[k] * s);
    col(x, ld)[k] = 0;
}

template <typename T>
__global__ void k_ir_update(double* __restrict__ x64, const T* __restrict__ d, int ld, int n,
                            const int* __restrict__ oact, const double* __restrict__ colnorm) {
    if (!oact[blockIdx.y]) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    col(x64, ld)[k] += colnorm[blockIdx.y] * (double)col(d, ld)[k];
}

__global__ void k_copy_cols(const double* __restrict__ a, int lda, double* __restrict__ b, int ldb,
                            int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) col(b, ldb)[k] = col(a, lda)[k];
}

__global__ void k_bb_init(ColState* st, int nc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nc) st[c].bb = 1.0;
}

template <typename T>
OpA<T> make_opA(const Level& L) {
    OpA<T> op;
    op.N = L.N;
    if constexpr (sizeof(T) == 8) {
        op.wE = L.wE64.get();
        op.wN = L.wN64.get();
        op.dinv = L.dinv64.get();
    } else {
        op.wE = L.wE32.get();
        op.wN = L.wN32.get();
        op.dinv = L.dinv32.get();
    }
    return op;
}

template <typename T>
OpKA<T> make_opKA(int N, const PriorParams& pp) {
    OpKA<T> op;
    op.N = N;
    op.h = 1.0 / N;
    op.g = pp.gamma;
    op.dl = pp.delta;
    op.bt = pp.beta;
    return op;
}

}  // namespace

// ================================================================== host ===
static bool trace_on() { return std::getenv("HINV_TRACE") != nullptr; }

static void trace_cols(hipStream_t s, const char* tag, int it, const ColState* st, const int* act, int nc) {
    std::vector<ColState> h(nc);
    std::vector<int> a(nc);
    (void)hipMemcpyAsync(h.data(), st, sizeof(ColState) * nc, hipMemcpyDeviceToHost, s);
    (void)hipMemcpyAsync(a.data(), act, sizeof(int) * nc, hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    std::fprintf(stderr, "[hinv] %s it=%d:", tag, it);
    for (int c = 0; c < nc; ++c)
        std::fprintf(stderr, " c%d(a=%d rz=%.3e pq=%.3e rr=%.3e obb=%.3e tol2=%.1e)", c, a[c], h[c].rz,
                     h[c].pq, h[c].rr, h[c].obb, h[c].tol2);
    std::fprintf(stderr, "\n");
}
Hierarchy::Hierarchy(Ctx* ctx, OpKind kind, int N, PriorParams pp)
    : ctx_(ctx), kind_(kind), N_(N), n_((N + 1) * (N + 1)), pp_(pp) {
    int Nl = N;
    while (true) {
        auto L = std::make_unique<Level>();
        L->N = Nl;
        L->n = (Nl + 1) * (Nl + 1);
        if (kind_ == kOpState) {
            L->cT.ensure((size_t)2 * Nl * Nl);
            L->wE64.ensure(L->n);
            L->wN64.ensure(L->n);
            L->dinv64.ensure(L->n);
            L->wE32.ensure(L->n);
            L->wN32.ensure(L->n);
            L->dinv32.ensure(L->n);
        }
        lev_.push_back(std::move(L));
        if (Nl <= kCoarseMaxN || (Nl & 1)) break;
        Nl /= 2;
    }
    nc_coarse_ = lev_.back()->n;
    if (nc_coarse_ > 128) fail(HINV_EINVAL, "coarsest multigrid level too large (N must be a power of two)");
    cinv64_.ensure((size_t)nc_coarse_ * nc_coarse_);
    cinv32_.ensure((size_t)nc_coarse_ * nc_coarse_);
    HINV_HIP(hipHostMalloc((void**)&host_flags_, sizeof(int) * 4096, hipHostMallocDefault));
    if (kind_ == kOpPrior) {
        build_coarse();
        ready_ = true;
    }
}

Hierarchy::~Hierarchy() {
    if (host_flags_) (void)hipHostFree(host_flags_);
}

void Hierarchy::build_coarse() {
    hipStream_t s = ctx_->stream;
    const int nc = nc_coarse_;
    const Level& L = *lev_.back();
    const int tot = nc * nc;
    if (kind_ == kOpState)
        k_coarse_matrix<<<ceil_div(tot, kBlock), kBlock, 0, s>>>(make_opA<double>(L), cinv64_.get());
    else
        k_coarse_matrix<<<ceil_div(tot, kBlock), kBlock, 0, s>>>(make_opKA<double>(L.N, pp_),
                                                                  cinv64_.get());
    HINV_LAUNCH_CHECK();
    const size_t shm = sizeof(double) * ((size_t)nc * nc + 2 * nc);
    k_gauss_jordan<<<1, 1024, shm, s>>>(nc, cinv64_.get());
    HINV_LAUNCH_CHECK();
    k_cast_d2f<<<ceil_div(tot, kBlock), kBlock, 0, s>>>(cinv64_.get(), cinv32_.get(), tot);
    HINV_LAUNCH_CHECK();
}

void Hierarchy::set_state_coefficient(const double* m) {
    if (kind_ != kOpState) fail(HINV_EINVAL, "set_state_coefficient on a prior hierarchy");
    hipStream_t s = ctx_->stream;
    const int N = lev_[0]->N;
    k_coef_fine<<<ceil_div(2 * N * N, kBlock), kBlock, 0, s>>>(N, m, lev_[0]->cT.get());
    HINV_LAUNCH_CHECK();
    for (size_t l = 0; l < lev_.size(); ++l) {
        Level& L = *lev_[l];
        if (l > 0) {
            k_coarsen<<<ceil_div(2 * L.N * L.N, kBlock), kBlock, 0, s>>>(L.N, lev_[l - 1]->cT.get(),
                                                                         L.cT.get());
            HINV_LAUNCH_CHECK();
        }
        k_weights<<<ceil_div(L.n, kBlock), kBlock, 0, s>>>(L.N, L.cT.get(), L.wE64.get(),
                                                           L.wN64.get(), L.dinv64.get(),
                                                           L.wE32.get(), L.wN32.get(),
                                                           L.dinv32.get());
        HINV_LAUNCH_CHECK();
    }
    build_coarse();
    ready_ = true;
}

template <>
PcgWork<double>& Hierarchy::work<double>() {
    return w64_;
}
template <>
PcgWork<float>& Hierarchy::work<float>() {
    return w32_;
}

void Hierarchy::ensure_cols(int nc) {
    if (nc <= cap_) return;
    const size_t n = n_;
    x64_.ensure(n * nc);
    r64_.ensure(n * nc);
    partial_.ensure((size_t)ceil_div(n, kBlock) * nc);
    st_.ensure(nc);
    act_.ensure(nc);
    oact_.ensure(nc);
    colnorm_.ensure(nc);
    if (nc > 4096) fail(HINV_EINVAL, "more than 4096 right-hand sides in one call");
    cap_ = nc;
}

template <typename T>
static void ensure_work(PcgWork<T>& w, const std::vector<std::unique_ptr<Level>>& lev, int nc) {
    if (nc <= w.cap) return;
    const size_t n = lev[0]->n;
    w.x.ensure(n * nc);
    w.r.ensure(n * nc);
    w.z.ensure(n * nc);
    w.p.ensure(n * nc);
    w.q.ensure(n * nc);
    w.lb.clear();
    w.lx.clear();
    w.lt.clear();
    for (size_t l = 0; l < lev.size(); ++l) {
        const size_t nl = lev[l]->n;
        w.lb.push_back(std::make_unique<DBuf<T>>());
        w.lx.push_back(std::make_unique<DBuf<T>>());
        w.lt.push_back(std::make_unique<DBuf<T>>());
        if (l > 0) {
            w.lb.back()->ensure(nl * nc);
            w.lx.back()->ensure(nl * nc);
        }
        w.lt.back()->ensure(nl * nc);
    }
    w.cap = nc;
}

template <typename T>
void Hierarchy::vcycle(int l, int nc) {
    hipStream_t s = ctx_->stream;
    PcgWork<T>& w = work<T>();
    const int nlev = (int)lev_.size();
    const Level& L = *lev_[l];
    const int ld = L.n;
    T* b = l == 0 ? w.r.get() : w.lb[l]->get();
    T* x = l == 0 ? w.z.get() : w.lx[l]->get();
    T* t = w.lt[l]->get();
    const int* act = act_.get();
    const int dir = kind_ == kOpState;
    if (l == nlev - 1) {
        const T* ci;
        if constexpr (sizeof(T) == 8)
            ci = cinv64_.get();
        else
            ci = cinv32_.get();
        k_coarse_solve<T><<<dim3(1, nc), 128, 0, s>>>(nc_coarse_, ci, b, x, ld, act);
        HINV_LAUNCH_CHECK();
        return;
    }
    static const Cheb ch;
    const T inv_theta = (T)(1.0 / ch.theta);
    const T cA = (T)(1.0 + ch.rho1 * ch.rho0), cB = (T)(2.0 * ch.rho1 / ch.delta);
    const T c1 = (T)(ch.rho1 * ch.rho0), c2 = cB, theta = (T)ch.theta;
    const dim3 g = grid2(L.n, nc);
    auto run = [&](auto op) {
        k_smooth_pre<T><<<g, kBlock, 0, s>>>(op, b, x, ld, act, cA, cB, inv_theta);
        HINV_LAUNCH_CHECK();
        k_residual<T><<<g, kBlock, 0, s>>>(op, b, x, t, ld, act);
        HINV_LAUNCH_CHECK();
        const Level& C = *lev_[l + 1];
        k_restrict<T><<<grid2(C.n, nc), kBlock, 0, s>>>(C.N, t, ld, w.lb[l + 1]->get(), C.n, dir, act);
        HINV_LAUNCH_CHECK();
        vcycle<T>(l + 1, nc);
        k_prolong_add<T><<<g, kBlock, 0, s>>>(C.N, w.lx[l + 1]->get(), C.n, x, ld, dir, act);
        HINV_LAUNCH_CHECK();
        k_post1<T><<<g, kBlock, 0, s>>>(op, b, x, t, ld, act, inv_theta);
        HINV_LAUNCH_CHECK();
        k_post2<T><<<g, kBlock, 0, s>>>(op, x, t, ld, act, theta, c1, c2,
                                        l == 0 ? (const T*)b : (const T*)nullptr,
                                        l == 0 ? partial_.get() : nullptr);
        HINV_LAUNCH_CHECK();
    };
    if (kind_ == kOpState)
        run(make_opA<T>(L));
    else
        run(make_opKA<T>(L.N, pp_));
}

// Inner PCG on w.r (right-hand side, overwritten by the residual) -> w.x.
// Column set: act_ (modified as columns converge); tolerances in st_.tol2, bb in st_.bb.
template <typename T>
void Hierarchy::pcg(int nc, int max_iter, int* iters) {
    hipStream_t s = ctx_->stream;
    PcgWork<T>& w = work<T>();
    const Level& L = *lev_[0];
    const int n = L.n, ld = n;
    const int nblk = ceil_div(n, kBlock);
    const dim3 g = grid2(n, nc);
    int* act = act_.get();
    const bool single = lev_.size() == 1;
    auto apply_dot = [&](auto op) {
        k_apply<T><<<g, kBlock, 0, s>>>(op, (const T*)w.p.get(), ld, w.q.get(), ld, act, partial_.get());
    };
    // z = M r, rz
    vcycle<T>(0, nc);
    if (single) k_dot<T><<<g, kBlock, 0, s>>>(w.r.get(), w.z.get(), ld, n, act, partial_.get());
    HINV_LAUNCH_CHECK();
    k_finalize<<<nc, kBlock, 0, s>>>(kFinRz0, partial_.get(), nblk, st_.get(), act);
    HINV_LAUNCH_CHECK();
    k_update_p<T><<<g, kBlock, 0, s>>>(w.z.get(), w.p.get(), ld, n, act, st_.get(), 1);
    HINV_LAUNCH_CHECK();
    int it = 0;
    for (; it < max_iter;) {
        if (kind_ == kOpState)
            apply_dot(make_opA<T>(L));
        else
            apply_dot(make_opKA<T>(L.N, pp_));
        HINV_LAUNCH_CHECK();
        k_finalize<<<nc, kBlock, 0, s>>>(kFinAlpha, partial_.get(), nblk, st_.get(), act);
        HINV_LAUNCH_CHECK();
        k_update_xr<T><<<g, kBlock, 0, s>>>(w.x.get(), w.r.get(), w.p.get(), w.q.get(), ld, n, act,
                                            st_.get(), partial_.get());
        HINV_LAUNCH_CHECK();
        k_finalize<<<nc, kBlock, 0, s>>>(kFinRr, partial_.get(), nblk, st_.get(), act);
        HINV_LAUNCH_CHECK();
        ++it;
        if (trace_on()) trace_cols(s, "pcg", it, st_.get(), act, nc);
        HINV_HIP(hipMemcpyAsync(host_flags_, act, sizeof(int) * nc, hipMemcpyDeviceToHost, s));
        HINV_HIP(hipStreamSynchronize(s));
        int live = 0;
        for (int c = 0; c < nc; ++c) live += host_flags_[c];
        if (!live) break;
        vcycle<T>(0, nc);
        if (single) k_dot<T><<<g, kBlock, 0, s>>>(w.r.get(), w.z.get(), ld, n, act, partial_.get());
        HINV_LAUNCH_CHECK();
        k_finalize<<<nc, kBlock, 0, s>>>(kFinRz, partial_.get(), nblk, st_.get(), act);
        HINV_LAUNCH_CHECK();
        k_update_p<T><<<g, kBlock, 0, s>>>(w.z.get(), w.p.get(), ld, n, act, st_.get(), 0);
        HINV_LAUNCH_CHECK();
    }
    *iters += it;
}

void Hierarchy::apply(int nc, const double* x, int ldx, double* y, int ldy) {
    if (!ready_) fail(HINV_ESTATE, "operator used before its coefficient was set");
    hipStream_t s = ctx_->stream;
    const dim3 g = grid2(n_, nc);
    if (kind_ == kOpState)
        k_apply<double><<<g, kBlock, 0, s>>>(make_opA<double>(*lev_[0]), x, ldx, y, ldy, nullptr, nullptr);
    else
        k_apply<double><<<g, kBlock, 0, s>>>(make_opKA<double>(N_, pp_), x, ldx, y, ldy, nullptr, nullptr);
    HINV_LAUNCH_CHECK();
}

void Hierarchy::solve(int nc, const double* b, int ldb, double* x, int ldx, int precision,
                      double rtol, int max_iter, SolveStats* stats) {
    if (!ready_) fail(HINV_ESTATE, "solve before the operator coefficient was set");
    if (nc <= 0) return;
    hipStream_t s = ctx_->stream;
    ensure_cols(nc);
    const bool fp32 = precision == HINV_PREC_FP32_IR;
    if (fp32)
        ensure_work(w32_, lev_, nc);
    else
        ensure_work(w64_, lev_, nc);
    const int n = n_, ld = n, nblk = ceil_div(n, kBlock);
    const dim3 g = grid2(n, nc);
    const Level& L0 = *lev_[0];
    auto launch_init = [&](auto op) {
        k_ir_init<<<g, kBlock, 0, s>>>(op, b, ldb, x64_.get(), r64_.get(), ld, partial_.get());
    };
    auto launch_res = [&](auto op) {
        k_ir_residual<<<g, kBlock, 0, s>>>(op, b, ldb, x64_.get(), r64_.get(), ld, oact_.get(),
                                           partial_.get());
    };
    if (kind_ == kOpState)
        launch_init(make_opA<double>(L0));
    else
        launch_init(make_opKA<double>(N_, pp_));
    HINV_LAUNCH_CHECK();
    const double floor32 = inner_tol32, floor64 = 1e-14;
    k_ir_finalize<<<nc, kBlock, 0, s>>>(1, partial_.get(), nblk, st_.get(), oact_.get(),
                                        colnorm_.get(), rtol, fp32 ? floor32 : floor64);
    HINV_LAUNCH_CHECK();
    int iters = 0, outer = 0, fallbacks = 0;
    const int max_outer = fp32 ? 16 : 4;
    bool use32 = fp32;
    std::vector<double> prev_rr(nc, 0.0);
    std::vector<ColState> hst(nc);
    bool converged = false;
    while (true) {
        HINV_HIP(hipMemcpyAsync(host_flags_, oact_.get(), sizeof(int) * nc, hipMemcpyDeviceToHost, s));
        if (use32)
            HINV_HIP(hipMemcpyAsync(hst.data(), st_.get(), sizeof(ColState) * nc, hipMemcpyDeviceToHost, s));
        HINV_HIP(hipStreamSynchronize(s));
        int live = 0;
        for (int c = 0; c < nc; ++c) live += host_flags_[c];
        if (!live) {
            converged = true;
            break;
        }
        if (outer >= max_outer || iters >= max_iter) break;
        if (use32) {
            // FP32 refinement stagnates when the condition number of the operator
            // approaches 1/eps_fp32: a step that cuts a residual by less than 10x
            // sends the remaining steps to FP64.
            bool stalled = false;
            for (int c = 0; c < nc; ++c)
                if (host_flags_[c] && outer > 0 && hst[c].rr > 1e-2 * prev_rr[c]) stalled = true;
            for (int c = 0; c < nc; ++c) prev_rr[c] = hst[c].rr;
            if (stalled) {
                use32 = false;
                ++fallbacks;
                ensure_work(w64_, lev_, nc);
                // recompute the inner tolerances for FP64 from the current residuals
                k_ir_finalize<<<nc, kBlock, 0, s>>>(0, partial_.get(), nblk, st_.get(), oact_.get(),
                                                    colnorm_.get(), rtol, floor64);
                HINV_LAUNCH_CHECK();
            }
        }
        HINV_HIP(hipMemcpyAsync(act_.get(), oact_.get(), sizeof(int) * nc, hipMemcpyDeviceToDevice, s));
        // the inner right-hand side has unit norm; its tolerance sits in tol2
        k_bb_init<<<ceil_div(nc, 64), 64, 0, s>>>(st_.get(), nc);
        HINV_LAUNCH_CHECK();
        if (use32) {
            k_ir_scale<float><<<g, kBlock, 0, s>>>(r64_.get(), w32_.r.get(), w32_.x.get(), ld, n,
                                                   oact_.get(), colnorm_.get());
            HINV_LAUNCH_CHECK();
            pcg<float>(nc, max_iter - iters, &iters);
            k_ir_update<float><<<g, kBlock, 0, s>>>(x64_.get(), w32_.x.get(), ld, n, oact_.get(),
                                                    colnorm_.get());
        } else {
            k_ir_scale<double><<<g, kBlock, 0, s>>>(r64_.get(), w64_.r.get(), w64_.x.get(), ld, n,
                                                    oact_.get(), colnorm_.get());
            HINV_LAUNCH_CHECK();
            pcg<double>(nc, max_iter - iters, &iters);
            k_ir_update<double><<<g, kBlock, 0, s>>>(x64_.get(), w64_.x.get(), ld, n, oact_.get(),
                                                     colnorm_.get());
        }
        HINV_LAUNCH_CHECK();
        if (kind_ == kOpState)
            launch_res(make_opA<double>(L0));
        else
            launch_res(make_opKA<double>(N_, pp_));
        HINV_LAUNCH_CHECK();
        k_ir_finalize<<<nc, kBlock, 0, s>>>(0, partial_.get(), nblk, st_.get(), oact_.get(),
                                            colnorm_.get(), rtol, use32 ? floor32 : floor64);
        HINV_LAUNCH_CHECK();
        ++outer;
        if (trace_on()) trace_cols(s, "outer", outer, st_.get(), oact_.get(), nc);
    }
    k_copy_cols<<<g, kBlock, 0, s>>>(x64_.get(), ld, x, ldx, n);
    HINV_LAUNCH_CHECK();
    // final relative residuals
    std::vector<ColState> hs(nc);
    HINV_HIP(hipMemcpyAsync(hs.data(), st_.get(), sizeof(ColState) * nc, hipMemcpyDeviceToHost, s));
    HINV_HIP(hipStreamSynchronize(s));
    double worst = 0.0;
    for (int c = 0; c < nc; ++c) {
        const double rel = hs[c].obb > 0 ? std::sqrt(hs[c].rr / hs[c].obb) : 0.0;
        worst = rel > worst ? rel : worst;
    }
    if (stats) {
        stats->solves += nc;
        stats->iterations += iters;
        stats->refinements += outer;
        stats->fallbacks += fallbacks;
        stats->max_relres = worst > stats->max_relres ? worst : stats->max_relres;
        stats->converged = stats->converged && converged;
    }
}

}  // namespace hinv
