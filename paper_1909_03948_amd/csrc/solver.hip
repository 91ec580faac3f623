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
#include <algorithm>
#include <limits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <type_traits>

#include "mgkernels.h"

namespace hinv {

namespace {

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
__global__ void k_apply(Op op_, const T* __restrict__ x, int ldx, T* __restrict__ y, int ldy,
                        const int* __restrict__ act, double* __restrict__ partial) {
    if (act && !act[blockIdx.y]) return;
    const auto& op = op_.at(blockIdx.y);
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

// Gauss-Jordan inversion of an SPD matrix (no pivoting), one workgroup of
// 1024 threads, n <= kGJMaxN, in place in M.  Pivot step p:  a = M[p][p];
// M[i][j] -= M[i][p] M[p][j] / a (i, j != p);  M[p][j] /= a;
// M[i][p] = -M[i][p] / a;  M[p][p] = 1 / a.  The matrix is held twice in LDS:
// step p reads one copy and writes the other, so a step needs one barrier
// and no staging of the pivot row and column.  Thread t owns the entries
// t, t + 1024, ... of the row-major matrix (indices divided once, up front).
constexpr int kGJMaxN = 81;
constexpr int kGJOwn = (kGJMaxN * kGJMaxN + 1023) / 1024;
__global__ __launch_bounds__(1024) void k_gauss_jordan(int n, double* __restrict__ M) {
    extern __shared__ double sm[];
    const int nn = n * n;
    int oi[kGJOwn], oj[kGJOwn];
#pragma unroll
    for (int e = 0; e < kGJOwn; ++e) {
        const int id = threadIdx.x + 1024 * e;
        oi[e] = id < nn ? id / n : 0;
        oj[e] = id < nn ? id - oi[e] * n : 0;
        if (id < nn) sm[id] = M[id];
    }
    __syncthreads();
    for (int p = 0; p < n; ++p) {
        const double* A = sm + (p & 1) * nn;
        double* B = sm + (1 - (p & 1)) * nn;
        const double ia = 1.0 / A[p * n + p];
#pragma unroll
        for (int e = 0; e < kGJOwn; ++e) {
            const int id = threadIdx.x + 1024 * e;
            if (id >= nn) break;
            const int i = oi[e], j = oj[e];
            double v;
            if (i == p && j == p)
                v = ia;
            else if (i == p)
                v = A[id] * ia;
            else if (j == p)
                v = -A[id] * ia;
            else
                v = A[id] - A[i * n + p] * A[p * n + j] * ia;
            B[id] = v;
        }
        __syncthreads();
    }
    const double* A = sm + (n & 1) * nn;
    for (int id = threadIdx.x; id < nn; id += 1024) M[id] = A[id];
}

__global__ void k_cast_d2f(const double* a, float* b, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) b[k] = (float)a[k];
}

// --------------------------------------------------- FP64 refinement loop ---
// r64 = masked b, x64 = 0, partial |r64|^2.
template <class Op>
__global__ void k_ir_init(Op op_, const double* __restrict__ b, int ldb, double* __restrict__ x64,
                          double* __restrict__ r64, int ld, double* __restrict__ partial) {
    const auto& op = op_.at(blockIdx.y);
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

// Gate of the refinement step of column c.  The step runs for an outer-active
// column; with the inner flags given (a step enqueued before the host knows
// whether the inner solve has finished) only once its inner solve has
// finished and only once per outer pass (tdone, set by k_ir_finalize).
__device__ inline bool ir_step_on(int c, const int* oact, const int* inner, const int* tdone) {
    return oact[c] && !(inner && inner[c]) && !(tdone && tdone[c]);
}

// r64 = b - A x64 on the gated columns, partial |r64|^2.
template <class Op>
__global__ void k_ir_residual(Op op_, const double* __restrict__ b, int ldb,
                              const double* __restrict__ x64, double* __restrict__ r64, int ld,
                              const int* __restrict__ act, const int* __restrict__ inner,
                              const int* __restrict__ tdone, double* __restrict__ partial) {
    if (!ir_step_on(blockIdx.y, act, inner, tdone)) return;
    const auto& op = op_.at(blockIdx.y);
    const int N1 = op.N + 1, n = N1 * N1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double v2 = 0.0;
    if constexpr (ApplyForm<std::decay_t<decltype(op)>>::kTable) {
        // prior operators: node by node (the LDS row table costs a barrier
        // that one node per thread does not repay; measured)
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
    } else {
        // state operator: straight-line form (the PCG apply kernel's), the
        // node's row, stencil values and b loaded before the first product
        const bool in = k < n;
        const int j = in ? k / N1 : 0, i = k - j * N1;
        typename std::decay_t<decltype(op)>::Row rw{};
        typename std::decay_t<decltype(op)>::Nb nb{};
        double bk = 0.0;
        if (in) {
            rw = op.row(i, j, k);
            nb = op.gather(i, j, k, col(x64, ld));
            bk = col(b, ldb)[k];
            double v = 0.0;
            if (op.is_free(i, j)) v = bk - op.combine(i, j, rw, nb);
            col(r64, ld)[k] = v;
            v2 = v * v;
        }
    }
    const double s = block_sum(v2);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

// Column sums of the partials of one reduction, one workgroup per column.
__device__ inline double column_total(const double* partial, int nblk) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += partial[(size_t)blockIdx.x * nblk + b];
    return block_sum(v);
}

// Outer bookkeeping per column.  first: bb = s (|b|^2).  Always: rr = s;
// column stays active while rr > rtol^2 bb; colnorm = |r|; inner tolerance.
__global__ void k_ir_finalize(int first, const double* __restrict__ partial, int nblk,
                              ColState* __restrict__ st, int* __restrict__ oact,
                              double* __restrict__ colnorm, double rtol, double tol_floor,
                              const int* __restrict__ inner, int* __restrict__ tdone) {
    if (!first && !ir_step_on(blockIdx.x, oact, inner, tdone)) return;
    const double s = column_total(partial, nblk);
    if (threadIdx.x != 0) return;
    if (tdone) tdone[blockIdx.x] = 1;
    ColState& c = st[blockIdx.x];
    if (first) c.obb = s;
    c.rr = s;
    // a non-finite residual (NaN or infinity in b, or met in the solve) stops
    // the column; the host reports it as not converged
    const bool a = isfinite(s) && isfinite(c.obb) && s > rtol * rtol * c.obb && s > 0.0;
    oact[blockIdx.x] = a ? 1 : 0;
    colnorm[blockIdx.x] = sqrt(s);
    if (a) {
        // inner target: the remaining factor to rtol |b|, with margin, floored
        double t = 0.5 * rtol * sqrt(c.obb / s);
        if (t < tol_floor) t = tol_floor;
        c.tol2 = t * t;  // relative to the inner right-hand side (unit norm)
    }
}

// Inner right-hand side r / |r| in precision T; zero initial guess.  The first
// workgroup of each column also starts the pass's column state: inner flag =
// outer flag, unit |b|^2, no PCG iterations, refinement step not yet taken.
template <typename T>
__global__ void k_ir_scale(const double* __restrict__ r64, T* __restrict__ r, T* __restrict__ x,
                           int ld, int n, const int* __restrict__ oact,
                           const double* __restrict__ colnorm, int* __restrict__ act,
                           ColState* __restrict__ st, int* __restrict__ tdone) {
    const int c = blockIdx.y;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        act[c] = oact[c];
        st[c].bb = 1.0;
        st[c].its = 0.0;
        tdone[c] = 0;
    }
    if (!oact[c]) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double s = 1.0 / colnorm[blockIdx.y];
    col(r, ld)[k] = (T)(col(r64, ld)[k] * s);
    col(x, ld)[k] = 0;
}

template <typename T>
__global__ void k_ir_update(double* __restrict__ x64, const T* __restrict__ d, int ld, int n,
                            const int* __restrict__ oact, const double* __restrict__ colnorm,
                            const int* __restrict__ inner, const int* __restrict__ tdone) {
    if (!ir_step_on(blockIdx.y, oact, inner, tdone)) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    col(x64, ld)[k] += colnorm[blockIdx.y] * (double)col(d, ld)[k];
}

__global__ void k_copy_cols(const double* __restrict__ a, int lda, double* __restrict__ b, int ldb,
                            int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) col(b, ldb)[k] = col(a, lda)[k];
}

// dst = src on free rows, 0 on Dirichlet rows.
template <class Op>
__global__ void k_masked_copy(Op op_, const double* __restrict__ src, int lds, double* __restrict__ dst,
                              int ldd) {
    const auto& op = op_.at(blockIdx.y);
    const int N1 = op.N + 1, n = N1 * N1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    col(dst, ldd)[k] = op.is_free(k % N1, k / N1) ? col(src, lds)[k] : 0.0;
}

__global__ void k_fill_int(int n, int v, int* __restrict__ a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}


// State operator of level L for instance inst alone.
template <typename T>
OpA<T> make_opA(const Level& L, int inst = 0) {
    OpA<T> op;
    op.N = L.N;
    const size_t off = (size_t)inst * L.n;
    if constexpr (sizeof(T) == 8) {
        op.wE = L.wE64.get() + off;
        op.wN = L.wN64.get() + off;
        op.dinv = L.dinv64.get() + off;
    } else {
        op.wE = L.wE32.get() + off;
        op.wN = L.wN32.get() + off;
        op.dinv = L.dinv32.get() + off;
    }
    return op;
}

template <typename T>
OpKA<T> make_opKA(int N, const PriorParams& pp) {
    return make_prior_op<T>(N, pp);
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
Hierarchy::Hierarchy(Ctx* ctx, OpKind kind, int N, PriorParams pp, int ninst,
                     const PriorParams* inst_pp)
    : ctx_(ctx), kind_(kind), N_(N), n_((N + 1) * (N + 1)), pp_(pp), ninst_(ninst) {
    if (ninst < 1) fail(HINV_EINVAL, "a hierarchy needs at least one instance");
    HINV_HIP(hipDeviceGetAttribute(&cus_, hipDeviceAttributeMultiprocessorCount, ctx->device));
    inst_pp_.assign(ninst, pp);
    if (inst_pp)
        for (int i = 0; i < ninst; ++i) inst_pp_[i] = inst_pp[i];
    inst_ready_.assign(ninst, 0);
    const size_t ni = ninst;
    int Nl = N;
    while (true) {
        auto L = std::make_unique<Level>();
        L->N = Nl;
        L->n = (Nl + 1) * (Nl + 1);
        if (kind_ == kOpState) {
            L->cT.ensure(ni * 2 * Nl * Nl);
            L->wE64.ensure(ni * L->n);
            L->wN64.ensure(ni * L->n);
            L->dinv64.ensure(ni * L->n);
            L->wE32.ensure(ni * L->n);
            L->wN32.ensure(ni * L->n);
            L->dinv32.ensure(ni * L->n);
        }
        lev_.push_back(std::move(L));
        if (Nl <= kCoarseMaxN || (Nl & 1)) break;
        Nl /= 2;
    }
    nc_coarse_ = lev_.back()->n;
    // the bottom kernel solves the coarsest level (N_c <= 8 for a power of two
    // N) with 12 threads per row and at most 8 entries per thread
    if (nc_coarse_ > 81) fail(HINV_EINVAL, "coarsest multigrid level too large (N must be a power of two)");
    cinv64_.ensure(ni * nc_coarse_ * nc_coarse_);
    cinv32_.ensure(ni * nc_coarse_ * nc_coarse_);
    HINV_HIP(hipHostMalloc((void**)&hblk_, (sizeof(ColState) + 3 * sizeof(int)) * 4096, hipHostMallocDefault));
    HINV_HIP(hipStreamCreateWithFlags(&gs_, hipStreamNonBlocking));
    launch_stream_ = ctx_->stream;
    if (kind_ == kOpPrior) {
        if (ninst_ > 1) {
            // row tables of every level and instance, [level][instance][class]
            const size_t nl = lev_.size();
            std::vector<KARow<double>> h64(nl * ni * 9);
            std::vector<KARow<float>> h32(nl * ni * 9);
            for (size_t l = 0; l < nl; ++l)
                for (size_t i = 0; i < ni; ++i) {
                    const PriorParams& q = inst_pp_[i];
                    const OpKA<double> o64 = make_prior_op<double>(lev_[l]->N, q);
                    const OpKA<float> o32 = make_prior_op<float>(lev_[l]->N, q);
                    for (int c = 0; c < 9; ++c) {
                        h64[(l * ni + i) * 9 + c] = o64.rows[c];
                        h32[(l * ni + i) * 9 + c] = o32.rows[c];
                    }
                }
            karow64_.ensure(h64.size());
            karow32_.ensure(h32.size());
            HINV_HIP(hipMemcpyAsync(karow64_.get(), h64.data(), sizeof(KARow<double>) * h64.size(),
                                    hipMemcpyHostToDevice, ctx_->stream));
            HINV_HIP(hipMemcpyAsync(karow32_.get(), h32.data(), sizeof(KARow<float>) * h32.size(),
                                    hipMemcpyHostToDevice, ctx_->stream));
            HINV_HIP(hipStreamSynchronize(ctx_->stream));
        }
        for (int i = 0; i < ninst_; ++i) build_coarse(i);
        ready_ = true;
    }
}

Hierarchy::~Hierarchy() {
    drop_graphs();
    if (gs_) (void)hipStreamDestroy(gs_);
    if (hblk_) (void)hipHostFree(hblk_);
}

void Hierarchy::build_coarse(int inst) {
    hipStream_t s = ctx_->stream;
    const int nc = nc_coarse_;
    const Level& L = *lev_.back();
    const int tot = nc * nc;
    double* c64 = cinv64_.get() + (size_t)inst * tot;
    if (kind_ == kOpState)
        k_coarse_matrix<<<ceil_div(tot, kBlock), kBlock, 0, s>>>(make_opA<double>(L, inst), c64);
    else
        k_coarse_matrix<<<ceil_div(tot, kBlock), kBlock, 0, s>>>(
            make_prior_op<double>(L.N, inst_pp_[inst]), c64);
    HINV_LAUNCH_CHECK();
    if (nc > kGJMaxN) fail(HINV_EINVAL, "coarse level too large for the dense inverse");
    const size_t shm = sizeof(double) * 2 * (size_t)nc * nc;
    k_gauss_jordan<<<1, 1024, shm, s>>>(nc, c64);
    HINV_LAUNCH_CHECK();
    k_cast_d2f<<<ceil_div(tot, kBlock), kBlock, 0, s>>>(c64, cinv32_.get() + (size_t)inst * tot, tot);
    HINV_LAUNCH_CHECK();
}

void Hierarchy::set_state_coefficient(const double* m, int inst) {
    if (kind_ != kOpState) fail(HINV_EINVAL, "set_state_coefficient on a prior hierarchy");
    if (inst < 0 || inst >= ninst_) fail(HINV_EINVAL, "instance index out of range");
    hipStream_t s = ctx_->stream;
    const int N = lev_[0]->N;
    auto cT = [&](int l) { return lev_[l]->cT.get() + (size_t)inst * 2 * lev_[l]->N * lev_[l]->N; };
    k_coef_fine<<<ceil_div(2 * N * N, kBlock), kBlock, 0, s>>>(N, m, cT(0));
    HINV_LAUNCH_CHECK();
    for (size_t l = 0; l < lev_.size(); ++l) {
        Level& L = *lev_[l];
        const size_t o = (size_t)inst * L.n;
        if (l > 0) {
            k_coarsen<<<ceil_div(2 * L.N * L.N, kBlock), kBlock, 0, s>>>(L.N, cT(l - 1), cT(l));
            HINV_LAUNCH_CHECK();
        }
        k_weights<<<ceil_div(L.n, kBlock), kBlock, 0, s>>>(L.N, cT(l), L.wE64.get() + o,
                                                           L.wN64.get() + o, L.dinv64.get() + o,
                                                           L.wE32.get() + o, L.wN32.get() + o,
                                                           L.dinv32.get() + o);
        HINV_LAUNCH_CHECK();
    }
    build_coarse(inst);
    inst_ready_[inst] = 1;
    ready_ = true;
    for (int i = 0; i < ninst_; ++i) ready_ = ready_ && inst_ready_[i];
}

template <typename T, class F>
void Hierarchy::with_op(int l, F fn) {
    const Level& L = *lev_[l];
    if (kind_ == kOpState) {
        OpA<T> o = make_opA<T>(L);
        if (ninst_ > 1) {
            o.cs = L.n;
            o.cpi = cpi_;
        }
        fn(o);
    } else if (ninst_ == 1) {
        fn(make_opKA<T>(L.N, pp_));
    } else {
        OpKARef<T> o;
        o.N = L.N;
        o.cpi = cpi_;
        const size_t off = (size_t)l * ninst_ * 9;
        if constexpr (sizeof(T) == 8)
            o.rows = karow64_.get() + off;
        else
            o.rows = karow32_.get() + off;
        fn(o);
    }
}

// Columns of a call: with stacked instances, nc / ninst consecutive columns each.
void Hierarchy::set_columns(int nc) {
    if (ninst_ == 1) {
        cpi_ = 1;
        return;
    }
    if (nc % ninst_) fail(HINV_EINVAL, "column count must be a multiple of the number of instances");
    cpi_ = nc / ninst_;
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
    drop_graphs();
    const size_t n = n_;
    x64_.ensure(n * nc);
    r64_.ensure(n * nc);
    // one partial per workgroup: vector kernels use ceil(n / kBlock) workgroups,
    // the fine-level V-cycle kernel one per tile (the small tiles give the most)
    const int tiles = ceil_div(N_ + 1, kTFSmall) * ceil_div(N_ + 1, kTFSmall);
    red_stride_ = std::max(ceil_div(n, kBlock), tiles);
    partial_.ensure((size_t)red_stride_ * nc);
    pcg_part_.ensure((size_t)red_stride_ * nc * 3);
    if (nc > 4096) fail(HINV_EINVAL, "more than 4096 right-hand sides in one call");
    sblk_.ensure((sizeof(ColState) + 3 * sizeof(int)) * (size_t)nc);
    st_.p = reinterpret_cast<ColState*>(sblk_.get());
    act_.p = reinterpret_cast<int*>(sblk_.get() + sizeof(ColState) * nc);
    oact_.p = act_.p + nc;
    tdone_.p = oact_.p + nc;
    colnorm_.ensure(nc);
    cap_ = nc;
}

void Hierarchy::read_state(hipStream_t s, int nc, int nflags) {
    const size_t bytes = sizeof(ColState) * cap_ + sizeof(int) * ((size_t)cap_ * (nflags - 1) + nc);
    HINV_HIP(hipMemcpyAsync(hblk_, sblk_.get(), bytes, hipMemcpyDeviceToHost, s));
}

template <typename T>
static void ensure_work(PcgWork<T>& w, const std::vector<std::unique_ptr<Level>>& lev, int nc) {
    if (nc <= w.cap) return;
    const size_t n = lev[0]->n;
    w.x.ensure(n * nc);
    w.r.ensure(n * nc);
    w.z.ensure(n * nc);
    w.p.ensure(n * nc);
    w.p2.ensure(n * nc);
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

// The finest level of a small-tile cycle takes 9 x 9 coarse / 18 x 18 fine
// tiles at eight waves a SIMD when its 8 x 8 / 16 x 16 tiles (seven
// workgroups a compute unit) would need more than two rounds of workgroups:
// at N = 1024, 4 225 workgroups in three rounds against 3 249 in two, 20%
// more halo work each (measured: one-column actions 3% faster there, 2%
// slower at N = 256, where one round holds the smaller tiles).
bool Hierarchy::finest_wide(int nc) const {
    if (!shape_.small || lev_.size() < 2 || lev_[0]->N <= kBottomN) return false;
    const long long t = ceil_div(lev_[1]->N + 1, kTCSmall);
    return t * t * ceil_div(nc, shape_.cb) > 2LL * 7 * cus_;
}

static ChebCoef cheb_coef() {
    const double theta = 0.5 * (kChebHi + kChebLo), delta = 0.5 * (kChebHi - kChebLo);
    const double sigma = theta / delta, rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
    ChebCoef c;
    c.inv_theta = 1.0 / theta;
    c.theta = theta;
    c.cA = 1.0 + rho1 * rho0;
    c.cB = 2.0 * rho1 / delta;
    c.c1 = rho1 * rho0;
    return c;
}

// z = V-cycle(r) on the PCG vectors of precision T; the last kernel finishes
// r^T z per column (beta, rz in ColState).
PcgRed Hierarchy::pcg_red(int nc) const {
    PcgRed r;
    r.stride = red_stride_;
    r.rz = pcg_part_.get();
    r.pq = r.rz + (size_t)red_stride_ * cap_;
    r.rr = r.pq + (size_t)red_stride_ * cap_;
    int Lb = 0;
    while (lev_[Lb]->N > kBottomN) ++Lb;
    const int tf = finest_wide(nc) ? kTFWide : small_tiles(0) ? kTFSmall : kTFBig;
    r.nrz = Lb == 0 ? 1 : ceil_div(lev_[0]->N + 1, tf) * ceil_div(lev_[0]->N + 1, tf);
    r.per = shape_.per;
    r.chunk = shape_.chunk > 0 ? shape_.chunk : kBlock * r.per;
    r.nvec = ceil_div(n_, r.chunk);
    return r;
}

// Fixed rule: small tiles below kSmallTileCols columns (more workgroups when
// few columns make the V-cycle latency bound); batched calls give each
// workgroup of the PCG vector kernels several node blocks, since every
// workgroup sums all partials of its column.
Hierarchy::LaunchShape Hierarchy::default_shape(int nc) const {
    const int nb = ceil_div(n_, kBlock);
    LaunchShape sh;
    sh.small = nc < kSmallTileCols;
    sh.per = nc < kSmallTileCols ? 1 : std::min(16, std::max(1, ceil_div(nb, 64)));
    sh.per = std::max(sh.per, min_per());
    sh.cb = 1;
    return sh;
}

// Every workgroup of the kernels after a reduction sums all of its partials,
// so their count enters squared: the PCG vector kernels keep it at or below
// kMaxVecPartials by giving each workgroup 1, 4, 8 or 16 node blocks (the
// tuner, which times the apply kernel alone, would otherwise pick more
// workgroups than pay inside the iteration).
int Hierarchy::min_per() const {
    const int nb = ceil_div(n_, kBlock);
    for (int per : {1, 4, 8, 16})
        if (ceil_div(nb, per) <= kMaxVecPartials) return per;
    return 16;
}

// ---- persistent tuner cache ------------------------------------------------
// Launch shapes the tuner picked, kept in the file named by HINV_TUNE_CACHE
// (JSON lines, one object a shape, appended as shapes are tuned; the last
// line of a key wins), so that later processes on the same kind of device
// reuse them instead of timing again.  Key: device architecture and compute
// unit count, operator kind, mesh size, stacked instances, columns, solve
// precision, and the version of the kernels' launch-shape rules.
namespace {
constexpr int kTuneVersion = 3;
std::mutex g_tune_mu;
bool g_tune_loaded = false;
struct TuneRec {
    std::string arch;
    int kind, N, ninst, nc, fp32, small, small_max, per, cb, chunk;
};
std::vector<TuneRec> g_tune;
long g_tune_timed = 0, g_tune_cached = 0;

std::string device_tag(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("HINV_TUNE_CACHE");
    if (!path || !*path) return;
    std::FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512], arch[128];
    while (std::fgets(line, sizeof line, f)) {
        TuneRec r;
        int ver = 0;
        if (std::sscanf(line,
                        "{\"version\": %d, \"device\": \"%127[^\"]\", \"kind\": %d, \"N\": %d, "
                        "\"instances\": %d, \"columns\": %d, \"fp32\": %d, \"small\": %d, "
                        "\"small_max\": %d, \"per\": %d, \"cb\": %d, \"chunk\": %d}",
                        &ver, arch, &r.kind, &r.N, &r.ninst, &r.nc, &r.fp32, &r.small, &r.small_max, &r.per,
                        &r.cb, &r.chunk) == 12 &&
            ver == kTuneVersion && r.per >= 1 && r.per <= 16 && r.cb >= 1 && r.cb <= 64 && r.chunk >= 0 &&
            r.chunk % 64 == 0 && r.chunk <= kVecNodes * vec_threads(r.per)) {
            r.arch = arch;
            g_tune.push_back(r);
        }
    }
    std::fclose(f);
}
}  // namespace

void tuner_counts(long* timed, long* cached) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    *timed = g_tune_timed;
    *cached = g_tune_cached;
}

// Times the candidate shapes on the call's own right-hand sides (w.r is set):
// the V-cycle with each tile choice, then the PCG apply kernel in its general
// form (beta from the r^T z partials) with 1, 4, 8 and 16 node blocks per
// workgroup.  Neither touches the solve's state: the apply kernel's outputs
// (p_new, q, the recorded r^T z) are rewritten by the first real iteration.
template <typename T>
void Hierarchy::tune_shape(int nc) {
    const long long key = 2LL * nc + (sizeof(T) == 4);
    for (const auto& kv : tuned_)
        if (kv.first == key) {
            shape_ = kv.second;
            return;
        }
    shape_ = default_shape(nc);
    // HINV_SHAPE forces a shape (tests of every launch path)
    if (const char* f = std::getenv("HINV_SHAPE")) {
        // HINV_SHAPE=<s|l><per>[c<cb>][k<chunk>]
        if ((f[0] == 's' || f[0] == 'l') && std::atoi(f + 1) >= 1) {
            shape_.small = f[0] == 's';
            shape_.small_max = 0;
            shape_.per = std::min(16, std::atoi(f + 1));
            const char* c = std::strchr(f, 'c');
            shape_.cb = c ? std::max(1, std::min(64, std::atoi(c + 1))) : 1;
            const char* k = std::strchr(f, 'k');
            shape_.chunk = k ? std::atoi(k + 1) : 0;
            if (shape_.chunk && (shape_.chunk % 64 || shape_.chunk > kVecNodes * vec_threads(shape_.per) ||
                                 ceil_div(n_, shape_.chunk) > red_stride_))
                fail(HINV_EINVAL, "HINV_SHAPE: chunk must be a multiple of 64 that the per's threads cover");
            return;
        }
    }
    const char* env = std::getenv("HINV_AUTOTUNE");
    if (env && env[0] == '0') return;
    const std::string arch = device_tag(ctx_->device);
    const int fp32 = sizeof(T) == 4;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
            if (it->arch == arch && it->kind == (int)kind_ && it->N == N_ && it->ninst == ninst_ && it->nc == nc &&
                it->fp32 == fp32 && it->per >= min_per()) {
                shape_.small = it->small != 0;
                shape_.small_max = it->small_max;
                shape_.per = it->per;
                shape_.cb = it->cb;
                shape_.chunk = it->chunk;
                tuned_.push_back({key, shape_});
                ++g_tune_cached;
                return;
            }
    }
    hipStream_t s = ctx_->stream;
    launch_stream_ = s;
    hipEvent_t e0, e1;
    HINV_HIP(hipEventCreate(&e0));
    HINV_HIP(hipEventCreate(&e1));
    const bool timer_was = ctx_->timer.paused;
    ctx_->timer.paused = true;
    auto timed = [&](auto fn) {
        fn();  // warm
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            HINV_HIP(hipEventRecord(e0, s));
            fn();
            HINV_HIP(hipEventRecord(e1, s));
            HINV_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            HINV_HIP(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return best;
    };
    LaunchShape best = shape_;
    float best_ms = 1e30f;
    // tiles: small on every level, or large above N_l = small_max (0: every
    // level large; 128, 256: the coarser levels keep the shorter workgroups)
    // Below kSmallTileCols columns every level keeps small tiles: timed back
    // to back, the V-cycle's vectors stay in cache and favour large tiles
    // (less halo), while inside PCG iterations they do not.
    const int N0 = lev_[0]->N;
    // cb: the RHS-block width, columns one workgroup of the V-cycle kernels sweeps
    for (int small_max : {-1, 0, 128, 256})
        for (int cb : {1, 2, 4, 8, 16}) {
            if (nc < kSmallTileCols && (cb > 1 || small_max >= 0)) continue;
            if (small_max > 0 && small_max >= N0) continue;
            shape_.small = small_max < 0;
            shape_.small_max = std::max(0, small_max);
            shape_.cb = cb;
            const float ms = timed([&] { vcycle<T>(nc, 0); });
            if (ms < best_ms) {
                best_ms = ms;
                best.small = shape_.small;
                best.small_max = shape_.small_max;
                best.cb = cb;
            }
        }
    shape_.small = best.small;
    shape_.small_max = best.small_max;
    shape_.cb = best.cb;
    PcgWork<T>& w = work<T>();
    const int n = n_;
    best_ms = 1e30f;
    // Few columns whose node blocks fit the partial cap one per workgroup keep
    // one block per workgroup: measured fastest inside the solves, while timing
    // the apply kernel alone has picked 4 in some runs (3% slower solves).
    const bool fixed_per = nc < kSmallTileCols && min_per() == 1;
    if (fixed_per) best.per = 1;
    // candidates (per, chunk): whole 256-node blocks, and for few columns the
    // column split into one or two workgroups of 1024 threads per compute unit
    // (a partial last round of workgroups costs as much as a full one)
    std::vector<std::pair<int, int>> cand;
    for (int per : {1, 4, 8, 16})
        if (!fixed_per && per >= min_per()) cand.push_back({per, 0});
    if (!fixed_per && nc < kSmallTileCols) {
        hipDeviceProp_t prop;
        HINV_HIP(hipGetDeviceProperties(&prop, ctx_->device));
        for (int w : {1, 2}) {
            const int want = prop.multiProcessorCount * w;
            const int chunk = ceil_div(ceil_div(n, want), 64) * 64;
            if (chunk <= kVecNodes * 1024 && ceil_div(n, chunk) <= kMaxVecPartials) cand.push_back({16, chunk});
        }
    }
    best.chunk = 0;
    for (const auto& pc : cand) {
        shape_.per = pc.first;
        shape_.chunk = pc.second;
        const PcgRed red = pcg_red(nc);
        const float ms = timed([&] {
            with_op<T>(0, [&](auto op) {
                k_pcg_apply<T, decltype(op), false><<<dim3(red.nvec, nc), vec_threads(red.per), 0, s>>>(
                    op, w.z.get(), w.p.get(), w.p2.get(), w.q.get(), n, act_.get(), st_.get(), red);
            });
            HINV_LAUNCH_CHECK();
        });
        if (ms < best_ms) {
            best_ms = ms;
            best.per = pc.first;
            best.chunk = pc.second;
        }
    }
    ctx_->timer.paused = timer_was;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    shape_ = best;
    tuned_.push_back({key, best});
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        ++g_tune_timed;
        TuneRec r{arch, (int)kind_, N_, ninst_, nc, fp32, best.small ? 1 : 0, best.small_max, best.per, best.cb,
                  best.chunk};
        g_tune.push_back(r);
        const char* path = std::getenv("HINV_TUNE_CACHE");
        if (path && *path)
            if (std::FILE* f = std::fopen(path, "a")) {
                std::fprintf(f,
                             "{\"version\": %d, \"device\": \"%s\", \"kind\": %d, \"N\": %d, \"instances\": %d, "
                             "\"columns\": %d, \"fp32\": %d, \"small\": %d, \"small_max\": %d, \"per\": %d, "
                             "\"cb\": %d, \"chunk\": %d}\n",
                             kTuneVersion, r.arch.c_str(), r.kind, r.N, r.ninst, r.nc, r.fp32, r.small, r.small_max,
                             r.per, r.cb, r.chunk);
                std::fclose(f);
            }
    }
    if (std::getenv("HINV_TRACE_SHAPES"))
        std::fprintf(stderr, "[hinv] launch shape N=%d nc=%d %s: %s tiles, %d columns per V-cycle workgroup, "
                     "%d node blocks per workgroup, chunk %d\n", N_, nc, sizeof(T) == 8 ? "fp64" : "fp32",
                     best.small ? "small" : (best.small_max ? "large above N=256/128, small" : "large"), best.cb,
                     best.per, best.chunk);
}

// z = V-cycle(r) for the PCG of precision T.  An FP64 PCG runs its V-cycle
// in FP32 (a preconditioner: its rounding changes the preconditioner, not the
// solve's result, which the PCG and the refinement test hold to their
// tolerance in FP64): the finest-level kernels read r and write z in FP64,
// every other vector of the cycle is FP32.
template <typename T>
void Hierarchy::vcycle(int nc, int check) {
    vcycle_impl<T, float>(nc, check);
}

// k_up_chain for NL levels with nt threads per workgroup (template dispatch).
template <typename T, class Op, int NL, int NT>
static void launch_chain1(dim3 g, hipStream_t s, const ChainArgs<T, Op>& ca, int dir, const int* act,
                          const ChebCoef& cc, int nc, int cb) {
    hipLaunchKernelGGL((k_up_chain<T, Op, kTFChain, NL, NT>), g, dim3(NT), 0, s, ca, dir, act, cc, nc, cb);
}
template <typename T, class Op, int NL>
static void launch_chain_nt(int nt, dim3 g, hipStream_t s, const ChainArgs<T, Op>& ca, int dir, const int* act,
                            const ChebCoef& cc, int nc, int cb) {
    if (nt == 512)
        launch_chain1<T, Op, NL, 512>(g, s, ca, dir, act, cc, nc, cb);
    else
        launch_chain1<T, Op, NL, 256>(g, s, ca, dir, act, cc, nc, cb);
}
template <typename T, class Op>
static void launch_chain(int NL, int nt, dim3 g, hipStream_t s, const ChainArgs<T, Op>& ca, int dir,
                         const int* act, const ChebCoef& cc, int nc, int cb) {
    switch (NL) {
        case 2: launch_chain_nt<T, Op, 2>(nt, g, s, ca, dir, act, cc, nc, cb); break;
        case 3: launch_chain_nt<T, Op, 3>(nt, g, s, ca, dir, act, cc, nc, cb); break;
        default: launch_chain_nt<T, Op, 4>(nt, g, s, ca, dir, act, cc, nc, cb); break;
    }
}

template <typename T, typename TI>
void Hierarchy::vcycle_impl(int nc, int check) {
    hipStream_t s = launch_stream_;
    PcgWork<T>& wt = work<T>();
    PcgWork<TI>& wi = work<TI>();
    const int nlev = (int)lev_.size();
    int Lb = 0;
    while (lev_[Lb]->N > kBottomN) ++Lb;
    int* act = act_.get();
    const int dir = kind_ == kOpState;
    const ChebCoef cc = cheb_coef();
    PcgRed red = pcg_red(nc);
    constexpr double st = sizeof(T), si = sizeof(TI);
    // Few columns: pair[l] = levels l and l + 1 take one k_down2 launch
    // (coarse levels paired from the bottom up while the finer of the two has
    // N_l <= kPairMaxN: above it the larger tiles cost what the launch saves),
    // and chain[l] = n: the up steps of levels l-n+1 .. l one k_up_chain launch.
    std::vector<char> pair(nlev, 0);
    std::vector<int> chain(nlev, 0);
    if (pair_levels()) {
        for (int l = Lb - 2; l >= 1 && lev_[l]->N <= kPairMaxN; l -= 2) pair[l] = true;
        // chains of up to kChainLen levels from the bottom up; a last one of
        // a single level stays a plain k_up
        for (int top = Lb - 1; top >= 2; top -= kChainLen) chain[top] = std::min(kChainLen, top);
    }
    // workgroups of 512 threads where a launch has fewer tiles than compute
    // units (each workgroup's passes are then the whole launch's latency)
    auto threads_for = [&](int tiles) { return tiles < cus_ ? 512 : 256; };

    for (int l = 0; l < Lb; ++l) {
        const Level& L = *lev_[l];
        const Level& C = *lev_[l + 1];
        if (pair[l]) {
            const Level& Cc = *lev_[l + 2];
            with_op<TI>(l, [&](auto opF) {
                with_op<TI>(l + 1, [&](auto opM) {
                    if constexpr (std::is_same_v<decltype(opF), decltype(opM)>) {
                        using Op = decltype(opF);
                        const int tc = ceil_div(Cc.N + 1, kTPair), gz = ceil_div(nc, shape_.cb);
                        auto go = [&](auto kern, int nt) {
                            timed_launch(ctx_, -1, 0.0, kern, dim3(tc, tc, gz), dim3(nt), s, opF, opM,
                                         (const TI*)wi.lb[l]->get(), wi.lt[l]->get(), L.n, wi.lb[l + 1]->get(),
                                         wi.lt[l + 1]->get(), C.n, wi.lb[l + 2]->get(), Cc.n, dir,
                                         (const int*)act, cc, nc, shape_.cb);
                        };
                        if (threads_for(tc * tc) == 512)
                            go(k_down2<TI, Op, kTPair, 512>, 512);
                        else
                            go(k_down2<TI, Op, kTPair, 256>, 256);
                    }
                });
            });
            HINV_LAUNCH_CHECK();
            ++l;
            continue;
        }
        // algorithmic bytes: read b, write x2 and b_coarse per column; the state
        // operator's three coefficient arrays once per launch and instance
        const double bytes_down = nc * ((l == 0 ? st : si) * L.n + si * (L.n + C.n)) + (dir ? si * 3.0 * L.n * ninst_ : 0.0);
        const int kcls = l == 0 ? kclass_for(kKDown, nc) : -1;
        with_op<TI>(l, [&](auto op) {
            using Op = decltype(op);
            const int chk = l == 0 ? check : 0;
            const int cb = shape_.cb, gz = ceil_div(nc, cb);
            TI* xl = wi.lt[l]->get();
            TI* bcl = wi.lb[l + 1]->get();
            ColState* stp = st_.get();
            auto launch = [&](auto kern, int tcs, const auto* bl) {
                const int tc = ceil_div(C.N + 1, tcs);
                timed_launch(ctx_, kcls, bytes_down, kern, dim3(tc, tc, gz), dim3(256), s, op, bl, xl, L.n, bcl, C.n,
                             dir, act, cc, red, stp, chk, nc, cb);
            };
            if (l == 0) {
                if (finest_wide(nc))
                    launch(k_down<TI, Op, kTCWide, T, 8>, kTCWide, (const T*)wt.r.get());
                else if (small_tiles(l))
                    launch(k_down<TI, Op, kTCSmall, T>, kTCSmall, (const T*)wt.r.get());
                else
                    launch(k_down<TI, Op, kTCBig, T>, kTCBig, (const T*)wt.r.get());
            } else {
                if (small_tiles(l))
                    launch(k_down<TI, Op, kTCSmall>, kTCSmall, (const TI*)wi.lb[l]->get());
                else
                    launch(k_down<TI, Op, kTCBig>, kTCBig, (const TI*)wi.lb[l]->get());
            }
        });
        HINV_LAUNCH_CHECK();
    }
    {
        // the bottom computes in FP32 (its coefficients, coarse inverse and
        // prior rows are the FP32 copies) on the cycle's vectors
        BottomArgs a{};
        a.nlev = nlev - Lb;
        if (a.nlev > kBottomLevels) fail(HINV_EINVAL, "internal: too many bottom levels");
        for (int l = 0; l < a.nlev; ++l) {
            const Level& L = *lev_[Lb + l];
            a.N[l] = L.N;
            if (kind_ == kOpState) {
                a.wE[l] = L.wE32.get();
                a.wN[l] = L.wN32.get();
                a.dinv[l] = L.dinv32.get();
            }
        }
        a.cinv = cinv32_.get();
        a.nc = nc_coarse_;
        if (kind_ == kOpPrior && ninst_ == 1)
            for (int l = 0; l < a.nlev; ++l) {
                const OpKA<float> o = make_opKA<float>(a.N[l], pp_);
                for (int c = 0; c < 9; ++c) a.ka[l][c] = o.rows[c];
            }
        if (ninst_ > 1) {
            a.cpi = cpi_;
            a.cinv_stride = (long long)nc_coarse_ * nc_coarse_;
            for (int l = 0; l < a.nlev; ++l) {
                a.cs[l] = lev_[Lb + l]->n;
                const size_t off = (size_t)(Lb + l) * ninst_ * 9;
                a.karows[l] = karow32_.get() ? karow32_.get() + off : nullptr;
            }
        }
        const int chk = Lb == 0 ? check : 0;
        // per column: read b (and r for r^T z), write x; once per launch: the
        // state coefficients of every bottom level and the dense coarse inverse
        const double nb = (double)(lev_[Lb]->n);
        double ncoef = 0.0;
        for (int l = Lb; l < nlev; ++l) ncoef += lev_[l]->n;
        const double coef_bytes = sizeof(float) * ninst_ * ((dir ? 3.0 * ncoef : 0.0) + (double)nc_coarse_ * nc_coarse_);
        ColState* stp = st_.get();
        const int ldb = lev_[Lb]->n;
        auto launch = [&](auto kern, const auto* bb, auto* xb, const auto* rv, double vb) {
            timed_launch(ctx_, kKBottom, nc * vb * (2.0 * nb + (rv ? nb : 0.0)) + coef_bytes, kern, dim3(nc),
                         dim3(1024), s, a, bb, xb, ldb, act, cc, rv, red, stp, chk);
        };
        if (Lb == 0) {
            // the whole hierarchy: r in, z out, and the r^T z partial
            const T* r = wt.r.get();
            if (kind_ == kOpState)
                launch(k_bottom<T, kOpState, kBottomN>, r, wt.z.get(), r, st);
            else
                launch(k_bottom<T, kOpPrior, kBottomN>, r, wt.z.get(), r, st);
        } else {
            const TI* none = nullptr;
            if (kind_ == kOpState)
                launch(k_bottom<TI, kOpState, kBottomN>, (const TI*)wi.lb[Lb]->get(), wi.lx[Lb]->get(), none, si);
            else
                launch(k_bottom<TI, kOpPrior, kBottomN>, (const TI*)wi.lb[Lb]->get(), wi.lx[Lb]->get(), none, si);
        }
        HINV_LAUNCH_CHECK();
    }
    for (int l = Lb - 1; l >= 0; --l) {
        const Level& L = *lev_[l];
        const Level& C = *lev_[l + 1];
        if (chain[l] >= 2) {
            const int NL = chain[l], lo = l - NL + 1;
            with_op<TI>(lo, [&](auto op0) {
                using Op = decltype(op0);
                ChainArgs<TI, Op> ca{};
                bool same = true;
                for (int k = 0; k < NL; ++k) {
                    const int lk = lo + k;
                    with_op<TI>(lk, [&](auto opk) {
                        if constexpr (std::is_same_v<decltype(opk), Op>)
                            ca.op[k] = opk;
                        else
                            same = false;
                    });
                    ca.b[k] = wi.lb[lk]->get();
                    ca.x2[k] = wi.lt[lk]->get();
                    ca.ld[k] = lev_[lk]->n;
                }
                if (!same) fail(HINV_EINVAL, "internal: mixed operator types in a chain");
                ca.x = wi.lx[lo]->get();
                ca.xc = wi.lx[l + 1]->get();
                ca.ldc = lev_[l + 1]->n;
                const int tf = ceil_div(lev_[lo]->N + 1, kTFChain), gz = ceil_div(nc, shape_.cb);
                launch_chain<TI, Op>(NL, threads_for(tf * tf), dim3(tf, tf, gz), s, ca, dir, act, cc, nc,
                                     shape_.cb);
            });
            HINV_LAUNCH_CHECK();
            l = lo;  // the loop's decrement continues below the chain
            continue;
        }
        // read b, x2, x_coarse (and r for r^T z), write x; coefficients once per instance
        const double bytes_up = nc * ((l == 0 ? 3.0 * st : 2.0 * si) * L.n + si * (L.n + C.n)) +
                                (dir ? si * 3.0 * L.n * ninst_ : 0.0);
        const int kcls = l == 0 ? kclass_for(kKUp, nc) : -1;
        with_op<TI>(l, [&](auto op) {
            using Op = decltype(op);
            const int cb = shape_.cb, gz = ceil_div(nc, cb);
            const TI* x2l = wi.lt[l]->get();
            const TI* xcl = wi.lx[l + 1]->get();
            const int* actc = act;
            auto launch = [&](auto kern, int tfs, const auto* bl, auto* xl, const auto* rv) {
                const int tf = ceil_div(L.N + 1, tfs);
                timed_launch(ctx_, kcls, bytes_up, kern, dim3(tf, tf, gz), dim3(256), s, op, bl, x2l, xl, L.n, xcl,
                             C.n, dir, actc, cc, rv, red, nc, cb);
            };
            if (l == 0) {
                const T* r = wt.r.get();
                if (finest_wide(nc))
                    launch(k_up<TI, Op, kTFWide, T, T, 8>, kTFWide, r, wt.z.get(), r);
                else if (small_tiles(l))
                    launch(k_up<TI, Op, kTFSmall, T, T>, kTFSmall, r, wt.z.get(), r);
                else
                    launch(k_up<TI, Op, kTFBig, T, T>, kTFBig, r, wt.z.get(), r);
            } else {
                const TI* bl = wi.lb[l]->get();
                const TI* none = nullptr;
                if (small_tiles(l))
                    launch(k_up<TI, Op, kTFSmall>, kTFSmall, bl, wi.lx[l]->get(), none);
                else
                    launch(k_up<TI, Op, kTFBig>, kTFBig, bl, wi.lx[l]->get(), none);
            }
        });
        HINV_LAUNCH_CHECK();
    }
}

// One PCG iteration (apply, update, V-cycle) on launch_stream_: p moves from
// P[cur] to P[1 - cur].
template <typename T>
void Hierarchy::pcg_iteration(int nc, int cur, int first) {
    hipStream_t s = launch_stream_;
    PcgWork<T>& w = work<T>();
    const Level& L = *lev_[0];
    const int n = L.n, ld = n;
    int* act = act_.get();
    const PcgRed red = pcg_red(nc);
    const dim3 g(red.nvec, nc);
    T* P[2] = {w.p.get(), w.p2.get()};
    {
        // read z, p_old, write p_new, q; state coefficients once per instance
        const double bytes_apply =
            sizeof(T) * ((double)nc * 4.0 * n + (kind_ == kOpState ? 2.0 * n * ninst_ : 0.0));
        with_op<T>(0, [&](auto op) {
            using Op = decltype(op);
            const T* zc = w.z.get();
            const T* pold = P[cur];
            const int* actc = act;
            ColState* stc = st_.get();
            timed_launch(ctx_, kclass_for(kKPcgApply, nc), bytes_apply, first ? k_pcg_apply<T, Op, true> : k_pcg_apply<T, Op, false>, g,
                         dim3(vec_threads(red.per)), s, op, zc, pold, P[1 - cur], w.q.get(), ld, actc, stc, red);
        });
        HINV_LAUNCH_CHECK();
    }
    {
        // x, r in/out, p, q in
        const T* pn = P[1 - cur];
        const T* qc = w.q.get();
        timed_launch(ctx_, kclass_for(kKPcgUpdate, nc), sizeof(T) * (double)nc * 6.0 * n, k_pcg_update<T>, g,
                     dim3(vec_threads(red.per)), s,
                     w.x.get(), w.r.get(), pn, qc, ld, n, act, st_.get(), red);
        HINV_LAUNCH_CHECK();
    }
    vcycle<T>(nc, 1);
}

// Graph of 2 reps PCG iterations starting from P[1], or of the prologue
// (captured once per precision and column count; replayed on the caller's
// stream).
template <typename T>
hipGraphExec_t Hierarchy::capture(int nc, bool prologue, int reps) {
    hipGraph_t graph = nullptr;
    HINV_HIP(hipStreamBeginCapture(gs_, hipStreamCaptureModeRelaxed));
    launch_stream_ = gs_;
    ctx_->timer.paused = true;
    try {
        if (prologue) {
            vcycle<T>(nc, 0);
            pcg_iteration<T>(nc, 0, 1);
        }
        for (int r = 0; r < reps; ++r) {
            pcg_iteration<T>(nc, 1, 0);
            pcg_iteration<T>(nc, 0, 0);
        }
    } catch (...) {
        ctx_->timer.paused = false;
        launch_stream_ = ctx_->stream;
        (void)hipStreamEndCapture(gs_, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    ctx_->timer.paused = false;
    launch_stream_ = ctx_->stream;
    HINV_HIP(hipStreamEndCapture(gs_, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HINV_HIP(e);
    return exec;
}

// Graph of 2 reps PCG iterations starting from P[1] (1 <= reps <= kMaxReps).
template <typename T>
hipGraphExec_t Hierarchy::pcg_graph(int nc, int reps) {
    const int slot = sizeof(T) == 8 ? 0 : 1, r = reps - 1;
    if (reps < 1 || reps > kMaxReps) fail(HINV_EINVAL, "PCG graph length out of range");
    hipGraphExec_t& g = gexec_[slot][r];
    if (g && gexec_nc_[slot][r] == nc) return g;
    if (g) {
        HINV_HIP(hipGraphExecDestroy(g));
        g = nullptr;
    }
    g = capture<T>(nc, false, reps);
    gexec_nc_[slot][r] = nc;
    return g;
}

// Graph of the start of a solve: the V-cycle of the initial residual, the
// first PCG iteration and 2 reps more (0 <= reps <= kMaxReps; ends with p in
// P[1]).
template <typename T>
hipGraphExec_t Hierarchy::prologue_graph(int nc, int reps) {
    const int slot = sizeof(T) == 8 ? 0 : 1;
    if (reps < 0 || reps > kMaxReps) fail(HINV_EINVAL, "PCG graph length out of range");
    hipGraphExec_t& g = gpro_[slot][reps];
    if (g && gpro_nc_[slot][reps] == nc) return g;
    if (g) {
        HINV_HIP(hipGraphExecDestroy(g));
        g = nullptr;
    }
    g = capture<T>(nc, true, reps);
    gpro_nc_[slot][reps] = nc;
    return g;
}

void Hierarchy::drop_graphs() {
    for (int i = 0; i < 2; ++i) {
        for (auto& g : gexec_[i])
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
        for (auto& g : gpro_[i])
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
}

// Inner PCG on w.r (right-hand side, overwritten by the residual) -> w.x.
// Columns: act_ (cleared on the device as columns converge); tolerances in
// st_.tol2 relative to st_.bb.  The start (V-cycle of the residual, first
// iteration) and the run of iterations up to the first completion check are
// one launch of a captured graph, later runs two iterations each; the host
// checks for completion after each run (kernels of finished columns return
// at once).
template <typename T>
bool Hierarchy::pcg(int nc, int max_iter, int* iters, const std::function<void()>* tail) {
    hipStream_t s = ctx_->stream;
    launch_stream_ = s;
    int* act = act_.get();
    tune_shape<T>(nc);
    const bool graphs = !std::getenv("HINV_NO_GRAPHS");
    // The prologue (V-cycle of the initial residual, first iteration) is a
    // graph too.  While the kernel timer runs, every 16th solve of few columns
    // and every batched solve launch their second and third iterations eagerly
    // with every launch sampled: like the replayed iterations they find the
    // operator in cache (the prologue's first V-cycle does not); graph replays
    // are counted only.  (Batched kernels run for a millisecond or more, so
    // their eager launches cost nothing measurable, and sampling each batched
    // solve keeps the mix of operators in the class averages fixed.)
    int it = 0;
    bool sampled = ctx_->timer.any_on() && (nc >= kSmallTileCols || solves_++ % 16 == 0);
    // Iterations before the first completion check follow the iteration count of
    // the last solve of this shape: the columns count their own iterations in
    // the column state, so the estimate is the slowest column's count, not the
    // replays (kernels of finished columns return at once, so a late check
    // costs launches, not work).  At most 13 iterations run before the first
    // check, 2 between later ones.
    const long long key = 2LL * nc + (sizeof(T) == 4);
    int expect = 0;
    for (const auto& kv : last_iters_)
        if (kv.first == key) expect = kv.second;
    // iterations after the prologue up to the first check: with graphs (and
    // no eager sampled iterations) they are part of the prologue's launch
    int pre = 0;
    if (graphs && max_iter > 0) {
        if (!sampled) pre = expect > 3 ? std::min(kMaxReps, expect / 2) : 1;
        while (pre > 0 && 1 + 2 * pre > max_iter) --pre;
        HINV_HIP(hipGraphLaunch(prologue_graph<T>(nc, pre), s));
        it = 1 + 2 * pre;
        for (int k : {kclass_for(kKDown, nc), kclass_for(kKUp, nc), (int)kKBottom}) ctx_->timer.count_only(k, 2 + 2 * pre);
        for (int k : {kclass_for(kKPcgApply, nc), kclass_for(kKPcgUpdate, nc)}) ctx_->timer.count_only(k, 1 + 2 * pre);
    } else {
        vcycle<T>(nc, 0);
        if (max_iter > 0) {
            pcg_iteration<T>(nc, 0, 1);
            it = 1;
        }
    }
    bool first_check = true, tail_state = false;
    const ColState* hst = host_st();  // pinned, so the read-backs need no staging copy
    const int* hact = host_act();
    bool pre_ran = pre > 0;
    while (it < max_iter || pre_ran) {
        if (pre_ran) {
            pre_ran = false;  // the first run came with the prologue
        } else {
            int reps = 1;
            if (first_check && expect > it + 2) reps = std::min(kMaxReps, (expect - it + 1) / 2);
            while (reps > 0 && it + 2 * reps > max_iter) --reps;
            if (sampled && it + 2 <= max_iter) {
                ctx_->timer.force = true;
                pcg_iteration<T>(nc, 1, 0);
                pcg_iteration<T>(nc, 0, 0);
                ctx_->timer.force = false;
                sampled = false;
                it += 2;
                if (reps > 1 && graphs) {
                    HINV_HIP(hipGraphLaunch(pcg_graph<T>(nc, reps - 1), s));
                    it += 2 * (reps - 1);
                    for (int k : {kclass_for(kKDown, nc), kclass_for(kKUp, nc), (int)kKBottom,
                                  kclass_for(kKPcgApply, nc), kclass_for(kKPcgUpdate, nc)})
                        ctx_->timer.count_only(k, 2 * (reps - 1));
                }
            } else if (graphs && reps > 0) {
                HINV_HIP(hipGraphLaunch(pcg_graph<T>(nc, reps), s));
                it += 2 * reps;
                // two iterations per replay: two launches of each finest-level class
                for (int k : {kclass_for(kKDown, nc), kclass_for(kKUp, nc), (int)kKBottom,
                                  kclass_for(kKPcgApply, nc), kclass_for(kKPcgUpdate, nc)})
                    ctx_->timer.count_only(k, 2 * reps);
            } else {
                // odd tail: one eager iteration keeps the ping-pong parity at P[1]
                pcg_iteration<T>(nc, 1, 0);
                pcg_iteration<T>(nc, 0, 0);
                it += 2;
            }
        }
        if (trace_on()) trace_cols(s, "pcg", it, st_.get(), act, nc);
        if (tail) (*tail)();
        read_state(s, nc, tail ? 2 : 1);
        HINV_HIP(hipStreamSynchronize(s));
        first_check = false;
        int live = 0;
        for (int c = 0; c < nc; ++c) live += hact[c];
        if (!live) {
            tail_state = tail != nullptr;
            break;
        }
    }
    int taken = 0;
    for (int c = 0; c < nc; ++c) taken = std::max(taken, (int)hst[c].its);
    if (first_check) taken = it;  // no completion check ran
    *iters += taken;
    bool found = false;
    for (auto& kv : last_iters_)
        if (kv.first == key) {
            kv.second = taken;
            found = true;
        }
    if (!found) last_iters_.push_back({key, taken});
    return tail_state;
}

void Hierarchy::apply(int nc, const double* x, int ldx, double* y, int ldy) {
    if (!ready_) fail(HINV_ESTATE, "operator used before its coefficient was set");
    if (nc <= 0) return;
    hipStream_t s = ctx_->stream;
    set_columns(nc);
    const dim3 g = grid2(n_, nc);
    with_op<double>(0, [&](auto op) {
        k_apply<double><<<g, kBlock, 0, s>>>(op, x, ldx, y, ldy, nullptr, nullptr);
    });
    HINV_LAUNCH_CHECK();
}

void Hierarchy::precondition(int nc, const double* r, int ldr, double* z, int ldz) {
    if (!ready_) fail(HINV_ESTATE, "operator used before its coefficient was set");
    if (nc <= 0) return;
    hipStream_t s = ctx_->stream;
    set_columns(nc);
    ensure_cols(nc);
    if (w64_.cap < nc || w32_.cap < nc) drop_graphs();
    ensure_work(w64_, lev_, nc);
    ensure_work(w32_, lev_, nc);
    const dim3 g = grid2(n_, nc);
    with_op<double>(0, [&](auto op) {
        k_masked_copy<<<g, kBlock, 0, s>>>(op, r, ldr, w64_.r.get(), n_);
    });
    HINV_LAUNCH_CHECK();
    k_fill_int<<<ceil_div(nc, 64), 64, 0, s>>>(nc, 1, act_.get());
    HINV_LAUNCH_CHECK();
    launch_stream_ = s;
    tune_shape<double>(nc);
    vcycle<double>(nc, 0);
    with_op<double>(0, [&](auto op) {
        k_masked_copy<<<g, kBlock, 0, s>>>(op, w64_.z.get(), n_, z, ldz);
    });
    HINV_LAUNCH_CHECK();
}

void Hierarchy::solve(int nc, const double* b, int ldb, double* x, int ldx, int precision,
                      double rtol, int max_iter, SolveStats* stats, double accept) {
    if (!ready_) fail(HINV_ESTATE, "solve before the operator coefficient was set");
    if (nc <= 0) return;
    hipStream_t s = ctx_->stream;
    set_columns(nc);
    ensure_cols(nc);
    if (precision == HINV_PREC_AUTO) precision = nc >= kAutoBatch ? HINV_PREC_FP32_IR : HINV_PREC_FP64;
    const bool fp32 = precision == HINV_PREC_FP32_IR;
    // the FP32 work serves every V-cycle, the FP64 work the FP64 PCG
    if (w32_.cap < nc || (!fp32 && w64_.cap < nc)) drop_graphs();
    ensure_work(w32_, lev_, nc);
    if (!fp32) ensure_work(w64_, lev_, nc);
    const int n = n_, ld = n, nblk = ceil_div(n, kBlock);
    const dim3 g = grid2(n, nc);
    // the FP64 iterate lives in the caller's x when its columns are contiguous
    // and do not overlap b (x is output only), else in x64_ and is copied out
    const auto lo = [](const void* p) { return reinterpret_cast<uintptr_t>(p); };
    const bool disjoint = lo(x + (size_t)ldx * nc) <= lo(b) || lo(b + (size_t)ldb * nc) <= lo(x);
    double* const xw = (ldx == n && disjoint) ? x : x64_.get();
    auto launch_init = [&](auto op) {
        k_ir_init<<<g, kBlock, 0, s>>>(op, b, ldb, xw, r64_.get(), ld, partial_.get());
    };
    with_op<double>(0, launch_init);
    HINV_LAUNCH_CHECK();
    // FP32 refinement: a pass reduces the true residual by no more than about
    // kappa eps_32, whatever the inner tolerance, so the inner PCG stops at half
    // the reduction the passes of the last FP32 solve achieved (never below
    // inner_tol32, never above 0.1); it adapts within the solve as passes are seen.
    const auto floor_for = [&](double rho) { return std::min(0.1, std::max(inner_tol32, 0.5 * rho)); };
    double floor32 = floor_for(rho32_), rho_seen = 0.0;
    const double floor64 = 1e-14;
    k_ir_finalize<<<nc, kBlock, 0, s>>>(1, partial_.get(), nblk, st_.get(), oact_.get(),
                                        colnorm_.get(), rtol, fp32 ? floor32 : floor64, nullptr, nullptr);
    HINV_LAUNCH_CHECK();
    int iters = 0, outer = 0, fallbacks = 0;
    bool have_state = false;  // the host block already holds this pass's outer state
    const int max_outer = fp32 ? 16 : 4;
    bool use32 = fp32;
    std::vector<double> prev_rr(nc, INFINITY);  // unknown before the first pass
    std::vector<int> prev_on(nc, 0);             // outer flags at the start of the last pass
    std::vector<double> rr_before(nc, INFINITY);  // residuals at the start of the last FP64 pass
    bool last64 = false;                          // the last pass ran in FP64
    const ColState* hst = host_st();  // pinned, so the read-backs need no staging copy
    const int* hoact = host_oact();
    bool converged = false;
    while (true) {
        // the first pass starts without reading the flags back: its kernels
        // skip the columns that are already converged (b = 0)
        if (outer > 0) {
            if (!have_state) {
                read_state(s, nc, 2);
                HINV_HIP(hipStreamSynchronize(s));
            }
            have_state = false;
            int live = 0;
            for (int c = 0; c < nc; ++c) live += hoact[c];
            if (!live) {
                converged = true;
                break;
            }
            // a goal below the acceptable tolerance: an FP64 pass that left every
            // remaining residual where it was (within 2x) has met the columns'
            // rounding floor; stop if all of them are acceptable
            if (accept > rtol && last64) {
                bool ok = true, moved = false;
                for (int c = 0; c < nc && ok; ++c) {
                    if (!hoact[c]) continue;
                    const double rr = hst[c].rr, obb = hst[c].obb;
                    ok = std::isfinite(rr) && obb > 0 && rr <= accept * accept * obb;
                    moved = moved || rr < 0.25 * rr_before[c];
                }
                if (ok && !moved) {
                    converged = true;
                    break;
                }
            }
            for (int c = 0; c < nc; ++c) rr_before[c] = hst[c].rr;
        }
        if (outer >= max_outer || iters >= max_iter) {
            if (outer == 0) {
                read_state(s, nc, 1);
                HINV_HIP(hipStreamSynchronize(s));
            }
            break;
        }
        if (use32) {
            // FP32 refinement stagnates when the condition number of the operator
            // approaches 1/eps_fp32: a step that cuts a residual by less than 10x
            // sends the remaining steps to FP64.
            bool stalled = false;
            if (outer > 0) {
                for (int c = 0; c < nc; ++c)
                    if (hoact[c] && hst[c].rr > 1e-2 * prev_rr[c]) stalled = true;
                if (outer >= 2)
                    for (int c = 0; c < nc; ++c)
                        if (prev_on[c] && prev_rr[c] > 0.0)
                            rho_seen = std::max(rho_seen, std::sqrt(hst[c].rr / prev_rr[c]));
                for (int c = 0; c < nc; ++c) {
                    prev_rr[c] = hst[c].rr;
                    prev_on[c] = hoact[c];
                }
                // the inner tolerances of the coming pass from the reductions seen
                const double f = floor_for(rho_seen);
                if (!stalled && f > 2.0 * floor32) {
                    floor32 = f;
                    k_ir_finalize<<<nc, kBlock, 0, s>>>(0, partial_.get(), nblk, st_.get(), oact_.get(),
                                                        colnorm_.get(), rtol, floor32, nullptr, nullptr);
                    HINV_LAUNCH_CHECK();
                }
            }
            if (stalled) {
                use32 = false;
                ++fallbacks;
                if (w64_.cap < nc) drop_graphs();
                ensure_work(w64_, lev_, nc);
                // recompute the inner tolerances for FP64 from the current residuals
                k_ir_finalize<<<nc, kBlock, 0, s>>>(0, partial_.get(), nblk, st_.get(), oact_.get(),
                                                    colnorm_.get(), rtol, floor64, nullptr, nullptr);
                HINV_LAUNCH_CHECK();
            }
        }
        // (k_ir_scale starts the pass's column state: the inner right-hand
        // side has unit norm, its tolerance sits in tol2)
        // refinement step x64 += |r| x_inner, r64 = b - A x64, outer bookkeeping;
        // with inner flags given, only for the columns whose PCG has finished
        // (and once per pass)
        auto step = [&](auto* xin, const int* inner) {
            using TI = std::remove_pointer_t<decltype(xin)>;
            k_ir_update<TI><<<g, kBlock, 0, s>>>(xw, xin, ld, n, oact_.get(), colnorm_.get(), inner, tdone_.get());
            HINV_LAUNCH_CHECK();
            with_op<double>(0, [&](auto op) {
                k_ir_residual<<<g, kBlock, 0, s>>>(op, b, ldb, xw, r64_.get(), ld, oact_.get(), inner, tdone_.get(),
                                                   partial_.get());
            });
            HINV_LAUNCH_CHECK();
            k_ir_finalize<<<nc, kBlock, 0, s>>>(0, partial_.get(), nblk, st_.get(), oact_.get(), colnorm_.get(),
                                                rtol, use32 ? floor32 : floor64, inner, tdone_.get());
            HINV_LAUNCH_CHECK();
        };
        if (use32) {
            k_ir_scale<float><<<g, kBlock, 0, s>>>(r64_.get(), w32_.r.get(), w32_.x.get(), ld, n, oact_.get(),
                                                   colnorm_.get(), act_.get(), st_.get(), tdone_.get());
            HINV_LAUNCH_CHECK();
            pcg<float>(nc, max_iter - iters, &iters);
            step(w32_.x.get(), nullptr);
            last64 = false;
        } else {
            k_ir_scale<double><<<g, kBlock, 0, s>>>(r64_.get(), w64_.r.get(), w64_.x.get(), ld, n, oact_.get(),
                                                    colnorm_.get(), act_.get(), st_.get(), tdone_.get());
            HINV_LAUNCH_CHECK();
            // the step is enqueued before each completion check of the PCG, so
            // that one read-back serves both checks when the PCG has finished
            const std::function<void()> tail = [&] { step(w64_.x.get(), act_.get()); };
            have_state = pcg<double>(nc, max_iter - iters, &iters, &tail);
            // stopped at the iteration limit: unfinished columns take the step they have
            if (!have_state) step(w64_.x.get(), nullptr);
            last64 = true;
        }
        ++outer;
        if (trace_on()) trace_cols(s, "outer", outer, st_.get(), oact_.get(), nc);
    }
    if (xw != x) {
        k_copy_cols<<<g, kBlock, 0, s>>>(xw, ld, x, ldx, n);
        HINV_LAUNCH_CHECK();
    }
    if (fp32 && rho_seen > 0.0) rho32_ = rho_seen;
    // final relative residuals: the column states read with the last flags
    // (no refinement step ran after that read)
    double worst = 0.0;
    bool finite = true;
    for (int c = 0; c < nc; ++c) {
        const double rr = hst[c].rr, obb = hst[c].obb;
        if (!std::isfinite(rr) || !std::isfinite(obb)) {
            finite = false;
            continue;
        }
        const double rel = obb > 0 ? std::sqrt(rr / obb) : 0.0;
        worst = rel > worst ? rel : worst;
    }
    if (!finite) worst = std::numeric_limits<double>::quiet_NaN();
    if (stats) {
        stats->solves += nc;
        stats->iterations += iters;
        stats->refinements += outer;
        stats->fallbacks += fallbacks;
        // a NaN stays NaN for the rest of the call's accumulated solves
        if (std::isnan(worst) || worst > stats->max_relres) stats->max_relres = worst;
        stats->converged = stats->converged && converged && finite;
    }
}

}  // namespace hinv
