// Quadratic (P2) state space: operator, two-level PCG, observation, gradient
// and Hessian-output kernels (see p2.h).
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "grid.h"
#include "p2.h"

namespace hinv {

namespace {

inline dim3 grid2(int n, int nc) { return dim3(ceil_div(n, kBlock), nc); }

// Fine-grid offset (dx, dy) in [0, 2]^2 of local dof j of triangle s of a cell.
__host__ __device__ inline void p2_offset(int s, int j, int& dx, int& dy) {
    // lower: a (0,0) r (2,0) b (2,2) | mid(a,r) (1,0) mid(r,b) (2,1) mid(a,b) (1,1)
    // upper: a (0,0) r (0,2) b (2,2) | mid(a,r) (0,1) mid(r,b) (1,2) mid(a,b) (1,1)
    constexpr int lx[6] = {0, 2, 2, 1, 2, 1}, ly[6] = {0, 0, 2, 0, 1, 1};
    dx = s == 0 ? lx[j] : ly[j];
    dy = s == 0 ? ly[j] : lx[j];
}

// Local dof of triangle s at cell offset (dx, dy), or -1.
__device__ inline int p2_local(int s, int dx, int dy) {
    if (s == 1) {  // the upper triangle mirrors the lower one across the diagonal
        const int t = dx;
        dx = dy;
        dy = t;
    }
    // lower triangle: dy <= dx
    if (dy > dx) return -1;
    constexpr int tab[3][3] = {{0, 3, 1}, {-1, 5, 4}, {-1, -1, 2}};  // [dy][dx]
    return tab[dy][dx];
}

__device__ inline int p2_dof(int side, int ci, int cj, int s, int j) {
    int dx, dy;
    p2_offset(s, j, dx, dy);
    return (2 * cj + dy) * side + 2 * ci + dx;
}

// Visits the triangles that hold fine node (I, J): f(ci, cj, s, local dof).
template <class F>
__device__ inline void p2_for_triangles(int N, int I, int J, F f) {
    const int ci0 = I > 0 ? max(0, (I - 1) / 2) : 0, ci1 = min(N - 1, I / 2);
    const int cj0 = J > 0 ? max(0, (J - 1) / 2) : 0, cj1 = min(N - 1, J / 2);
    for (int cj = cj0; cj <= cj1; ++cj)
        for (int ci = ci0; ci <= ci1; ++ci)
            for (int s = 0; s < 2; ++s) {
                const int loc = p2_local(s, I - 2 * ci, J - 2 * cj);
                if (loc >= 0) f(ci, cj, s, loc);
            }
}

template <typename T>
__device__ inline T* colp(T* p, int ld) {
    return p + (size_t)blockIdx.y * ld;
}

// Per-triangle coefficient: c_T, or the sensitivity s_T = (c_T/3) sum mhat.
__device__ inline double tri_coef(int N, const double* cT, const double* mh, int ci, int cj, int s) {
    const double c = cT[2 * (cj * N + ci) + s];
    if (!mh) return c;
    int ka, kr, kb;
    tri_nodes(N, ci, cj, s, ka, kr, kb);
    return c * (1.0 / 3.0) * (mh[ka] + mh[kr] + mh[kb]);
}

// y = scale K[coef] x (or y = b - K[coef] x when b is given) on the free rows,
// 0 on the Dirichlet rows.  mhat != null: coefficient s_T(mhat) per column.
// ldx = 0: the same x for every column.  act: columns to skip (may be null).
__global__ void k_p2_apply(int N, P2Elem el, const double* __restrict__ cT, const double* __restrict__ mhat,
                           int ldm, const double* __restrict__ x, int ldx, const double* __restrict__ b,
                           int ldb, double scale, double* __restrict__ y, int ldy,
                           const int* __restrict__ act) {
    const int side = 2 * N + 1, ns = side * side;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns || (act && !act[blockIdx.y])) return;
    const int J = k / side, I = k - J * side;
    double v = 0.0;
    if (J > 0 && J < 2 * N) {
        const double* xc = x + (size_t)blockIdx.y * ldx;
        const double* mh = mhat ? colp(mhat, ldm) : nullptr;
        double acc = 0.0;
        p2_for_triangles(N, I, J, [&](int ci, int cj, int s, int loc) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < 6; ++j) t += el.K[s][loc][j] * xc[p2_dof(side, ci, cj, s, j)];
            acc += tri_coef(N, cT, mh, ci, cj, s) * t;
        });
        v = b ? colp(b, ldb)[k] - acc : scale * acc;
    }
    colp(y, ldy)[k] = v;
}

// 1 / diag(A_2) on the free rows, 0 on the Dirichlet rows.
__global__ void k_p2_dinv(int N, P2Elem el, const double* __restrict__ cT, double* __restrict__ dinv) {
    const int side = 2 * N + 1, ns = side * side;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns) return;
    const int J = k / side, I = k - J * side;
    double dg = 0.0;
    p2_for_triangles(N, I, J, [&](int ci, int cj, int s, int loc) {
        dg += cT[2 * (cj * N + ci) + s] * el.K[s][loc][loc];
    });
    dinv[k] = (J > 0 && J < 2 * N && dg > 0.0) ? 1.0 / dg : 0.0;
}

__global__ void k_p2_top(int N, double* __restrict__ u) {
    const int side = 2 * N + 1;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I < side) u[(size_t)(2 * N) * side + I] = 1.0;
}

// rc = P^T r (P1 vertex v: its own value plus half of the midpoints of the
// edges at v: horizontal, vertical and the SW-NE diagonal), 0 on the P1
// Dirichlet rows.
__global__ void k_p2_restrict(int N, const double* __restrict__ r, int ldr, double* __restrict__ rc, int ldc,
                              const int* __restrict__ act) {
    const int N1 = N + 1, side = 2 * N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1 || (act && !act[blockIdx.y])) return;
    const int j = k / N1, i = k - j * N1;
    double v = 0.0;
    if (j > 0 && j < N) {
        const double* rr = colp(r, ldr);
        const int I = 2 * i, J = 2 * j, c = J * side + I;
        double h = 0.0;
        if (I > 0) h += rr[c - 1];
        if (I < 2 * N) h += rr[c + 1];
        h += rr[c - side] + rr[c + side];
        if (I < 2 * N) h += rr[c + side + 1];
        if (I > 0) h += rr[c - side - 1];
        v = rr[c] + 0.5 * h;
    }
    colp(rc, ldc)[k] = v;
}

// x += P e on the free rows (the P1 function e evaluated at the P2 nodes).
__global__ void k_p2_prolong_add(int N, const double* __restrict__ e, int lde, double* __restrict__ x, int ldx,
                                 const int* __restrict__ act) {
    const int N1 = N + 1, side = 2 * N + 1, ns = side * side;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns || (act && !act[blockIdx.y])) return;
    const int J = k / side, I = k - J * side;
    if (J == 0 || J == 2 * N) return;
    const double* ec = colp(e, lde);
    const int i0 = I >> 1, j0 = J >> 1, i1 = (I + 1) >> 1, j1 = (J + 1) >> 1;
    // even coordinates give i0 == i1; odd ones the two ends of the edge
    const double v = (I & 1) || (J & 1) ? 0.5 * (ec[j0 * N1 + i0] + ec[j1 * N1 + i1]) : ec[j0 * N1 + i0];
    colp(x, ldx)[k] += v;
}

// First Chebyshev step: d = dinv r / theta; x = d (from_zero) or x += d.
__global__ void k_p2_cheb_init(int ns, const double* __restrict__ dinv, const double* __restrict__ r, int ld,
                               double inv_theta, double* __restrict__ d, double* __restrict__ x, int ldx,
                               int from_zero, const int* __restrict__ act) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns || (act && !act[blockIdx.y])) return;
    const size_t o = (size_t)blockIdx.y * ld + k;
    const double v = dinv[k] * r[o] * inv_theta;
    d[o] = v;
    double* xp = x + (size_t)blockIdx.y * ldx + k;
    *xp = from_zero ? v : *xp + v;
}

// Next Chebyshev step after q = A d: r -= q; d = c1 d + c2 dinv r; x += d.
__global__ void k_p2_cheb_step(int ns, const double* __restrict__ dinv, const double* __restrict__ q,
                               double* __restrict__ r, double* __restrict__ d, int ld, double* __restrict__ x,
                               int ldx, double c1, double c2, const int* __restrict__ act) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns || (act && !act[blockIdx.y])) return;
    const size_t o = (size_t)blockIdx.y * ld + k;
    const double rv = r[o] - q[o];
    const double dv = c1 * d[o] + c2 * dinv[k] * rv;
    r[o] = rv;
    d[o] = dv;
    x[(size_t)blockIdx.y * ldx + k] += dv;
}

__global__ void k_p2_masked_copy(int N, const double* __restrict__ a, int lda, double* __restrict__ b, int ldb) {
    const int side = 2 * N + 1, ns = side * side;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ns) return;
    const int J = k / side;
    colp(b, ldb)[k] = (J > 0 && J < 2 * N) ? colp(a, lda)[k] : 0.0;
}

__global__ void k_p2_dot_partial(int n, const double* __restrict__ a, int lda, const double* __restrict__ b,
                                 int ldb, double* __restrict__ part) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const double v = k < n ? colp(a, lda)[k] * colp(b, ldb)[k] : 0.0;
    const double s = block_sum(v);
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ void k_p2_dot_finish(const double* __restrict__ part, int nblk, double* __restrict__ out) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += part[(size_t)blockIdx.x * nblk + b];
    const double s = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// alpha = rz / pq; x += alpha p; r -= alpha q (pq <= 0: no step)
__global__ void k_p2_pcg_step(int ns, const double* __restrict__ rz, const double* __restrict__ pq,
                              double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                              const double* __restrict__ q, int ld, int ldx, const int* __restrict__ act) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (k >= ns || !act[c]) return;
    const double a = pq[c] > 0.0 ? rz[c] / pq[c] : 0.0;
    const size_t o = (size_t)c * ld + k;
    x[(size_t)c * ldx + k] += a * p[o];
    r[o] -= a * q[o];
}

// p = z + beta p with beta = rz_new / rz_old (first: p = z)
__global__ void k_p2_pcg_dir(int ns, const double* __restrict__ rzn, const double* __restrict__ rzo,
                             const double* __restrict__ z, double* __restrict__ p, int ld, int first,
                             const int* __restrict__ act) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (k >= ns || !act[c]) return;
    const size_t o = (size_t)c * ld + k;
    p[o] = first ? z[o] : z[o] + (rzn[c] / rzo[c]) * p[o];
}

__global__ void k_p2_zero(int ns, double* __restrict__ x, int ld) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < ns) colp(x, ld)[k] = 0.0;
}

// u_T^T K_T w_T of triangle (ci, cj, s)
__device__ inline double p2_form(const P2Elem& el, int side, int ci, int cj, int s, const double* u,
                                 const double* w) {
    double uv[6], wv[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const int d = p2_dof(side, ci, cj, s, j);
        uv[j] = u[d];
        wv[j] = w[d];
    }
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
        double t = 0.0;
#pragma unroll
        for (int b = 0; b < 6; ++b) t += el.K[s][a][b] * wv[b];
        acc += uv[a] * t;
    }
    return acc;
}

// g_v = sum_{T ni v} (c_T/3) u_T^T K p_T
__global__ void k_p2_grad(int N, P2Elem el, const double* __restrict__ cT, const double* __restrict__ u,
                          const double* __restrict__ p, double* __restrict__ g) {
    const int N1 = N + 1, side = 2 * N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int j = k / N1, i = k - j * N1;
    double acc = 0.0;
    for_incident_triangles(N, i, j, [&](int ci, int cj, int s, int) {
        acc += cT[2 * (cj * N + ci) + s] * (1.0 / 3.0) * p2_form(el, side, ci, cj, s, u, p);
    });
    g[k] = acc;
}

// (H mhat)_v without the prior: sum_{T ni v} (c_T/3) [u K phat + uhat K p + (1/3) sum_T mhat u K p]
// (Gauss-Newton: the first term only)
__global__ void k_p2_hess_out(int N, P2Elem el, const double* __restrict__ cT, const double* __restrict__ u,
                              const double* __restrict__ p, const double* __restrict__ uh, int ldu,
                              const double* __restrict__ ph, int ldp, const double* __restrict__ mh, int ldm,
                              double* __restrict__ out, int ldo, int gn, const double* __restrict__ add,
                              int ldadd) {
    const int N1 = N + 1, side = 2 * N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int j = k / N1, i = k - j * N1;
    const double* uhc = colp(uh, ldu);
    const double* phc = colp(ph, ldp);
    const double* mhc = colp(mh, ldm);
    double acc = 0.0;
    for_incident_triangles(N, i, j, [&](int ci, int cj, int s, int) {
        double v = p2_form(el, side, ci, cj, s, u, phc);
        if (!gn) {
            int ka, kr, kb;
            tri_nodes(N, ci, cj, s, ka, kr, kb);
            v += p2_form(el, side, ci, cj, s, uhc, p);
            v += (1.0 / 3.0) * (mhc[ka] + mhc[kr] + mhc[kb]) * p2_form(el, side, ci, cj, s, u, p);
        }
        acc += cT[2 * (cj * N + ci) + s] * (1.0 / 3.0) * v;
    });
    if (add) acc = colp(add, ldadd)[k] + acc;
    colp(out, ldo)[k] = acc;
}

// Observation point o in cell (i, j), triangle as for P1 (lower when the
// local x offset is >= the local y offset), barycentric (lam_a, lam_r, lam_b);
// the six P2 basis values there.
__global__ void k_p2_obs_setup(int N, int q, const double* __restrict__ xy, int* __restrict__ node,
                               double* __restrict__ w) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= q) return;
    const int side = 2 * N + 1;
    const double x = xy[2 * o] * N, y = xy[2 * o + 1] * N;
    int i = (int)floor(x), j = (int)floor(y);
    i = i < 0 ? 0 : (i > N - 1 ? N - 1 : i);
    j = j < 0 ? 0 : (j > N - 1 ? N - 1 : j);
    const double xi = x - i, ze = y - j;
    const int s = xi >= ze ? 0 : 1;
    const double la = s == 0 ? 1.0 - xi : 1.0 - ze;
    const double lr = s == 0 ? xi - ze : ze - xi;
    const double lb = s == 0 ? ze : xi;
    const double psi[6] = {la * (2.0 * la - 1.0), lr * (2.0 * lr - 1.0), lb * (2.0 * lb - 1.0),
                           4.0 * la * lr,         4.0 * lr * lb,         4.0 * la * lb};
    for (int a = 0; a < 6; ++a) {
        node[6 * o + a] = p2_dof(side, i, j, s, a);
        w[6 * o + a] = psi[a];
    }
}

__global__ void k_p2_obs_gather(int q, const int* __restrict__ node, const double* __restrict__ w,
                                const double* __restrict__ u, int ldu, const double* __restrict__ d,
                                double* __restrict__ out, int ldo) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= q) return;
    const double* uc = colp(u, ldu);
    double v = 0.0;
    for (int a = 0; a < 6; ++a) v += w[6 * o + a] * uc[node[6 * o + a]];
    if (d) v -= d[o];
    colp(out, ldo)[o] = v;
}

// y[dof] += scale (B^T v)[dof] over the dofs touched by observations (CSR, fixed order)
__global__ void k_p2_obs_scatter(int nt, const int* __restrict__ tnode, const int* __restrict__ tptr,
                                 const int* __restrict__ tent, const double* __restrict__ w,
                                 const double* __restrict__ v, int ldv, double scale, double* __restrict__ y,
                                 int ldy) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const double* vc = colp(v, ldv);
    double s = 0.0;
    for (int e = tptr[t]; e < tptr[t + 1]; ++e) {
        const int ent = tent[e];
        s += w[ent] * vc[ent / 6];
    }
    colp(y, ldy)[tnode[t]] += scale * s;
}

}  // namespace

// ---------------------------------------------------------------- host ---
P2Elem p2_element() {
    // cell with legs 1; lower: a (0,0), r (1,0), b (1,1); upper: a (0,0), r (0,1), b (1,1).
    // Barycentric gradients: lower lam_a = 1 - x, lam_r = x - y, lam_b = y;
    // upper lam_a = 1 - y, lam_r = y - x, lam_b = x.  Area 1/2.
    const double G[2][3][2] = {{{-1, 0}, {1, -1}, {0, 1}}, {{0, -1}, {-1, 1}, {1, 0}}};
    const int ev[3][2] = {{0, 1}, {1, 2}, {0, 2}};  // local edges of the midpoint dofs
    P2Elem el{};
    for (int s = 0; s < 2; ++s)
        for (int qp = 0; qp < 3; ++qp) {
            double lam[3] = {0, 0, 0};
            lam[ev[qp][0]] = lam[ev[qp][1]] = 0.5;
            double g[6][2];
            for (int v = 0; v < 3; ++v)
                for (int d = 0; d < 2; ++d) g[v][d] = (4.0 * lam[v] - 1.0) * G[s][v][d];
            for (int e = 0; e < 3; ++e) {
                const int v = ev[e][0], w = ev[e][1];
                for (int d = 0; d < 2; ++d) g[3 + e][d] = 4.0 * (lam[w] * G[s][v][d] + lam[v] * G[s][w][d]);
            }
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b)
                    el.K[s][a][b] += (0.5 / 3.0) * (g[a][0] * g[b][0] + g[a][1] * g[b][1]);
        }
    return el;
}

namespace {
// Largest eigenvalue of D^-1/2 K D^-1/2 of the element (power iteration on a
// 6 x 6 matrix whose spectrum is nonnegative).  A = sum c_T K_T and
// D = sum c_T diag(K_T) give x^T A x <= mu x^T D x for all x, so mu bounds the
// spectrum of D^-1 A_2 from above.
double element_bound(const P2Elem& el) {
    double mu = 0.0;
    for (int s = 0; s < 2; ++s) {
        double M[6][6];
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) M[a][b] = el.K[s][a][b] / std::sqrt(el.K[s][a][a] * el.K[s][b][b]);
        double v[6] = {1, -0.7, 0.4, -0.9, 0.6, -0.3}, lam = 0.0;
        for (int it = 0; it < 500; ++it) {
            double w[6] = {0, 0, 0, 0, 0, 0}, nw = 0.0;
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b) w[a] += M[a][b] * v[b];
            for (int a = 0; a < 6; ++a) nw += w[a] * w[a];
            nw = std::sqrt(nw);
            for (int a = 0; a < 6; ++a) v[a] = w[a] / nw;
            lam = nw;
        }
        mu = std::max(mu, lam);
    }
    return mu;
}
}  // namespace

P2Space::P2Space(Ctx* ctx, int N_) : N(N_), side(2 * N_ + 1), ns((2 * N_ + 1) * (2 * N_ + 1)), ctx_(ctx) {
    el_ = p2_element();
    lmax_ = element_bound(el_) * 1.0001;  // power iteration converges from below
    dinv_.ensure(ns);
}

void P2Space::set_coefficient(const double* cT) {
    cT_ = cT;
    k_p2_dinv<<<ceil_div(ns, kBlock), kBlock, 0, ctx_->stream>>>(N, el_, cT, dinv_.get());
    HINV_LAUNCH_CHECK();
}

void P2Space::apply(int nc, const double* x, int ldx, double* y, int ldy, double scale) {
    if (!cT_) fail(HINV_ESTATE, "P2 operator used before its coefficient was set");
    k_p2_apply<<<grid2(ns, nc), kBlock, 0, ctx_->stream>>>(N, el_, cT_, nullptr, 0, x, ldx, nullptr, 0, scale,
                                                           y, ldy, nullptr);
    HINV_LAUNCH_CHECK();
}

void P2Space::sens(int nc, const double* mhat, int ldm, const double* w, double scale, double* y, int ldy) {
    if (!cT_) fail(HINV_ESTATE, "P2 operator used before its coefficient was set");
    k_p2_apply<<<grid2(ns, nc), kBlock, 0, ctx_->stream>>>(N, el_, cT_, mhat, ldm, w, 0, nullptr, 0, scale, y,
                                                           ldy, nullptr);
    HINV_LAUNCH_CHECK();
}

void P2Space::set_top(double* u) {
    k_p2_top<<<ceil_div(side, kBlock), kBlock, 0, ctx_->stream>>>(N, u);
    HINV_LAUNCH_CHECK();
}

void P2Space::forward_rhs(double* rhs) {
    ensure(1);
    double* uD = t1_.get();
    k_p2_zero<<<ceil_div(ns, kBlock), kBlock, 0, ctx_->stream>>>(ns, uD, ns);
    HINV_LAUNCH_CHECK();
    set_top(uD);
    apply(1, uD, ns, rhs, ns, -1.0);
}

void P2Space::ensure(int nc) {
    if (nc <= cap_) return;
    const size_t len = (size_t)ns * nc;
    for (auto* b : {&r_, &z_, &p_, &q_v_, &t1_, &t2_, &t3_}) b->ensure(len);
    const size_t n1 = (size_t)(N + 1) * (N + 1) * nc;
    rc_.ensure(n1);
    ec_.ensure(n1);
    part_.ensure((size_t)ceil_div(ns, kBlock) * nc);
    scal_.ensure(6 * (size_t)nc);
    act_.ensure(nc);
    cap_ = nc;
}

void P2Space::dots(int nc, const double* a, int lda, const double* b, int ldb, double* out) {
    const int nblk = ceil_div(ns, kBlock);
    k_p2_dot_partial<<<grid2(ns, nc), kBlock, 0, ctx_->stream>>>(ns, a, lda, b, ldb, part_.get());
    HINV_LAUNCH_CHECK();
    k_p2_dot_finish<<<nc, kBlock, 0, ctx_->stream>>>(part_.get(), nblk, out);
    HINV_LAUNCH_CHECK();
}

// z = two-level cycle applied to r (all in ns-strided columns, act marks the
// live columns): degree-2 Chebyshev-Jacobi on [lmax / 4, lmax] from zero,
// P^T of the residual through one V-cycle of the P1 hierarchy, P back, and
// the same smoother again from the corrected iterate.
void P2Space::precondition(int nc, const double* r, int ldr, double* z, int ldz, Hierarchy& coarse) {
    hipStream_t s = ctx_->stream;
    const int* act = act_.get();
    const double hi = lmax_, lo = 0.25 * lmax_;
    const double theta = 0.5 * (hi + lo), dl = 0.5 * (hi - lo), sigma1 = theta / dl;
    const double rho0 = 1.0 / sigma1, rho1 = 1.0 / (2.0 * sigma1 - rho0);
    const double c1 = rho1 * rho0, c2 = 2.0 * rho1 / dl;
    const dim3 g = grid2(ns, nc);
    double* rs = t1_.get();
    double* d = t2_.get();
    double* q = t3_.get();
    const int N1 = N + 1, n1 = N1 * N1;
    auto smooth = [&](bool from_zero) {
        // rs = r (from zero) or r - A z; d = D^-1 rs / theta, z = d or z += d
        if (from_zero)
            k_p2_masked_copy<<<g, kBlock, 0, s>>>(N, r, ldr, rs, ns);
        else
            k_p2_apply<<<g, kBlock, 0, s>>>(N, el_, cT_, nullptr, 0, z, ldz, r, ldr, 1.0, rs, ns, act);
        HINV_LAUNCH_CHECK();
        k_p2_cheb_init<<<g, kBlock, 0, s>>>(ns, dinv_.get(), rs, ns, 1.0 / theta, d, z, ldz, from_zero ? 1 : 0,
                                            act);
        HINV_LAUNCH_CHECK();
        // second step: rs -= A d, d = c1 d + c2 D^-1 rs, z += d
        k_p2_apply<<<g, kBlock, 0, s>>>(N, el_, cT_, nullptr, 0, d, ns, nullptr, 0, 1.0, q, ns, act);
        HINV_LAUNCH_CHECK();
        k_p2_cheb_step<<<g, kBlock, 0, s>>>(ns, dinv_.get(), q, rs, d, ns, z, ldz, c1, c2, act);
        HINV_LAUNCH_CHECK();
    };
    smooth(true);
    // coarse correction
    k_p2_apply<<<g, kBlock, 0, s>>>(N, el_, cT_, nullptr, 0, z, ldz, r, ldr, 1.0, rs, ns, act);
    HINV_LAUNCH_CHECK();
    k_p2_restrict<<<grid2(n1, nc), kBlock, 0, s>>>(N, rs, ns, rc_.get(), n1, act);
    HINV_LAUNCH_CHECK();
    coarse.precondition(nc, rc_.get(), n1, ec_.get(), n1);
    k_p2_prolong_add<<<g, kBlock, 0, s>>>(N, ec_.get(), n1, z, ldz, act);
    HINV_LAUNCH_CHECK();
    smooth(false);
}

void P2Space::solve(int nc, const double* b, int ldb, double* x, int ldx, Hierarchy& coarse, double rtol,
                    int max_iter, SolveStats* st) {
    if (!cT_) fail(HINV_ESTATE, "P2 solve before the coefficient was set");
    if (nc <= 0) return;
    ensure(nc);
    hipStream_t s = ctx_->stream;
    const dim3 g = grid2(ns, nc);
    double* bb = scal_.get();
    double* rz = bb + nc;
    double* rzn = rz + nc;
    double* pq = rzn + nc;
    double* rr = pq + nc;
    // r = b on the free rows; x = 0
    k_p2_masked_copy<<<g, kBlock, 0, s>>>(N, b, ldb, r_.get(), ns);
    HINV_LAUNCH_CHECK();
    k_p2_zero<<<g, kBlock, 0, s>>>(ns, x, ldx);
    HINV_LAUNCH_CHECK();
    dots(nc, r_.get(), ns, r_.get(), ns, bb);
    std::vector<double> hbb(nc), hrr(nc);
    HINV_HIP(hipMemcpyAsync(hbb.data(), bb, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
    HINV_HIP(hipStreamSynchronize(s));
    std::vector<int> hact(nc);
    int live = 0;
    bool finite = true;
    for (int c = 0; c < nc; ++c) {
        hact[c] = hbb[c] > 0.0 && std::isfinite(hbb[c]);
        if (!std::isfinite(hbb[c])) finite = false;
        live += hact[c];
        hrr[c] = hbb[c];
    }
    HINV_HIP(hipMemcpyAsync(act_.get(), hact.data(), sizeof(int) * nc, hipMemcpyHostToDevice, s));
    int its = 0;
    if (live) {
        precondition(nc, r_.get(), ns, z_.get(), ns, coarse);
        dots(nc, r_.get(), ns, z_.get(), ns, rz);
        k_p2_pcg_dir<<<g, kBlock, 0, s>>>(ns, rz, rz, z_.get(), p_.get(), ns, 1, act_.get());
        HINV_LAUNCH_CHECK();
    }
    while (live && its < max_iter) {
        k_p2_apply<<<g, kBlock, 0, s>>>(N, el_, cT_, nullptr, 0, p_.get(), ns, nullptr, 0, 1.0, q_v_.get(), ns,
                                        act_.get());
        HINV_LAUNCH_CHECK();
        dots(nc, p_.get(), ns, q_v_.get(), ns, pq);
        k_p2_pcg_step<<<g, kBlock, 0, s>>>(ns, rz, pq, x, r_.get(), p_.get(), q_v_.get(), ns, ldx, act_.get());
        HINV_LAUNCH_CHECK();
        dots(nc, r_.get(), ns, r_.get(), ns, rr);
        ++its;
        HINV_HIP(hipMemcpyAsync(hrr.data(), rr, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
        HINV_HIP(hipStreamSynchronize(s));
        bool changed = false;
        for (int c = 0; c < nc; ++c) {
            if (!hact[c]) continue;
            const bool done = !(hrr[c] > rtol * rtol * hbb[c]);  // NaN stops the column too
            if (!std::isfinite(hrr[c])) finite = false;
            if (done) {
                hact[c] = 0;
                --live;
                changed = true;
            }
        }
        if (changed) HINV_HIP(hipMemcpyAsync(act_.get(), hact.data(), sizeof(int) * nc, hipMemcpyHostToDevice, s));
        if (!live) break;
        precondition(nc, r_.get(), ns, z_.get(), ns, coarse);
        dots(nc, r_.get(), ns, z_.get(), ns, rzn);
        k_p2_pcg_dir<<<g, kBlock, 0, s>>>(ns, rzn, rz, z_.get(), p_.get(), ns, 0, act_.get());
        HINV_LAUNCH_CHECK();
        std::swap(rz, rzn);
    }
    // the pinned host copies of act_ are read by the stream: keep them alive
    HINV_HIP(hipStreamSynchronize(s));
    double worst = 0.0;
    for (int c = 0; c < nc; ++c) {
        if (!(hbb[c] > 0.0)) continue;
        const double rel = std::sqrt(hrr[c] / hbb[c]);
        if (!std::isfinite(rel)) finite = false;
        else worst = std::max(worst, rel);
    }
    if (!finite) worst = std::numeric_limits<double>::quiet_NaN();
    if (st) {
        st->solves += nc;
        st->iterations += its;
        st->refinements += 1;
        if (std::isnan(worst) || worst > st->max_relres) st->max_relres = worst;
        st->converged = st->converged && live == 0 && finite;
    }
}

void P2Space::grad(const double* u, const double* p, double* g) {
    const int n1 = (N + 1) * (N + 1);
    k_p2_grad<<<ceil_div(n1, kBlock), kBlock, 0, ctx_->stream>>>(N, el_, cT_, u, p, g);
    HINV_LAUNCH_CHECK();
}

void P2Space::hess_out(int nc, bool gn, const double* u, const double* p, const double* uh, int ldu,
                       const double* ph, int ldp, const double* mh, int ldm, double* out, int ldo,
                       const double* add, int ldadd) {
    const int n1 = (N + 1) * (N + 1);
    k_p2_hess_out<<<grid2(n1, nc), kBlock, 0, ctx_->stream>>>(N, el_, cT_, u, p, uh, ldu, ph, ldp, mh, ldm, out,
                                                              ldo, gn ? 1 : 0, add, ldadd);
    HINV_LAUNCH_CHECK();
}

void P2Space::set_observations(int q, const double* xy_dev) {
    q_ = q;
    if (q == 0) return;
    hipStream_t s = ctx_->stream;
    obs_node_.ensure(6 * (size_t)q);
    obs_w_.ensure(6 * (size_t)q);
    k_p2_obs_setup<<<ceil_div(q, kBlock), kBlock, 0, s>>>(N, q, xy_dev, obs_node_.get(), obs_w_.get());
    HINV_LAUNCH_CHECK();
    // transpose structure: dof -> list of (6 o + a), from the device's dof indices
    std::vector<int> hn(6 * (size_t)q);
    HINV_HIP(hipMemcpyAsync(hn.data(), obs_node_.get(), sizeof(int) * 6 * q, hipMemcpyDeviceToHost, s));
    HINV_HIP(hipStreamSynchronize(s));
    std::vector<int> order(6 * (size_t)q);
    for (int e = 0; e < 6 * q; ++e) order[e] = e;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hn[a] < hn[b]; });
    std::vector<int> tn, tp, te;
    for (int e = 0; e < 6 * q; ++e) {
        const int nd = hn[order[e]];
        if (tn.empty() || tn.back() != nd) {
            tn.push_back(nd);
            tp.push_back(e);
        }
        te.push_back(order[e]);
    }
    tp.push_back(6 * q);
    n_touch_ = (int)tn.size();
    t_node_.ensure(tn.size());
    t_ptr_.ensure(tp.size());
    t_ent_.ensure(te.size());
    HINV_HIP(hipMemcpyAsync(t_node_.get(), tn.data(), sizeof(int) * tn.size(), hipMemcpyHostToDevice, s));
    HINV_HIP(hipMemcpyAsync(t_ptr_.get(), tp.data(), sizeof(int) * tp.size(), hipMemcpyHostToDevice, s));
    HINV_HIP(hipMemcpyAsync(t_ent_.get(), te.data(), sizeof(int) * te.size(), hipMemcpyHostToDevice, s));
    HINV_HIP(hipStreamSynchronize(s));
}

void P2Space::observe(int nc, const double* u, int ldu, const double* d, double* out, int ldo) {
    if (q_ == 0) return;
    k_p2_obs_gather<<<grid2(q_, nc), kBlock, 0, ctx_->stream>>>(q_, obs_node_.get(), obs_w_.get(), u, ldu, d, out,
                                                                ldo);
    HINV_LAUNCH_CHECK();
}

void P2Space::observe_adjoint(int nc, const double* v, int ldv, double scale, double* y, int ldy) {
    if (q_ == 0) return;
    k_p2_obs_scatter<<<grid2(n_touch_, nc), kBlock, 0, ctx_->stream>>>(n_touch_, t_node_.get(), t_ptr_.get(),
                                                                       t_ent_.get(), obs_w_.get(), v, ldv, scale, y,
                                                                       ldy);
    HINV_LAUNCH_CHECK();
}

}  // namespace hinv
