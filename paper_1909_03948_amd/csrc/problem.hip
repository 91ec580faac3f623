// Operations of the Poisson coefficient-inversion problem on the device.
//
//   forward         A(m)_FF u_F = -A(m)_FD u_D          (Sec. 5.1, Eq. eq:poisson_weak)
//   cost            1/2 sigma^-2 |B u - d|^2 + 1/2 (m - m_pr)^T R (m - m_pr)
//                                                        (Sec. 5.1, Eq. eq:cost-elliptic)
//   adjoint         A_FF p_F = -[B^T (B u - d)]_F / sigma^2              (App. A, eq:firstadj)
//   gradient        g_v = [R (m - m_pr)]_v + sum_{T ni v} (c_T / 3) |T| grad u . grad p
//                                                        (App. A, eq:firstcontrol)
//   inc. forward    A_FF uhat_F = -[K[s] u]_F, s_T = (c_T/3) sum_{w in T} mhat_w
//                                                        (App. A, eq:incrementals1)
//   inc. adjoint    A_FF phat_F = -[B^T B uhat / sigma^2 + K[s] p]_F  (eq:incrementals2)
//   Hessian         (H mhat)_v = sum_{T ni v} (c_T/3) |T| (grad u . grad phat + grad uhat . grad p)
//                    + sum_{T ni v} (c_T/9) (sum_{w in T} mhat_w) |T| grad u . grad p [+ R mhat]
//                                                        (eq:incrementals3)
//   prior           R = K_A M^-1 K_A, R^-1 = K_A^-1 M K_A^-1           (Sec. 5.1, Sec. 2.3)
//   prior draw      m_pr + K_A^-1 C_M eta, C_M C_M^T = M  (Sec. 4.3.1, App. C)
//
// c_T = exp((m_a + m_r + m_b) / 3) (centroid rule); K[s] is the stiffness with
// per-triangle coefficient s_T, a five-point stencil on this mesh.
#include <algorithm>

#include "grid.h"
#include "problem.h"

namespace hinv {

namespace {

inline dim3 grid2(int n, int nc) { return dim3(ceil_div(n, kBlock), nc); }

template <typename T>
__device__ inline T* colp(T* p, int ld) {
    return p + (size_t)blockIdx.y * ld;
}

// ---------------------------------------------------------- observations ---
// Point (x, y) lies in cell (i, j) = (min(floor(x N), N-1), min(floor(y N), N-1)),
// local offsets xi = x N - i, zeta = y N - j.  Lower triangle when xi >= zeta:
// P1 weights (1 - xi, xi - zeta, zeta) on (k(i,j), k(i+1,j), k(i+1,j+1));
// upper: (1 - zeta, zeta - xi, xi) on (k(i,j), k(i,j+1), k(i+1,j+1)).
__global__ void k_obs_setup(int N, int q, const double* __restrict__ xy, int* __restrict__ node,
                            double* __restrict__ w) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= q) return;
    const double x = xy[2 * o] * N, y = xy[2 * o + 1] * N;
    int i = (int)floor(x), j = (int)floor(y);
    i = i < 0 ? 0 : (i > N - 1 ? N - 1 : i);
    j = j < 0 ? 0 : (j > N - 1 ? N - 1 : j);
    const double xi = x - i, ze = y - j;
    node[3 * o] = knode(i, j, N);
    node[3 * o + 2] = knode(i + 1, j + 1, N);
    if (xi >= ze) {
        node[3 * o + 1] = knode(i + 1, j, N);
        w[3 * o] = 1.0 - xi;
        w[3 * o + 1] = xi - ze;
        w[3 * o + 2] = ze;
    } else {
        node[3 * o + 1] = knode(i, j + 1, N);
        w[3 * o] = 1.0 - ze;
        w[3 * o + 1] = ze - xi;
        w[3 * o + 2] = xi;
    }
}

// out[o] = (B u)_o - d_o (d may be null).
__global__ void k_obs_gather(int q, const int* __restrict__ node, const double* __restrict__ w,
                             const double* __restrict__ u, int ldu, const double* __restrict__ d,
                             double* __restrict__ out, int ldo) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= q) return;
    const double* uc = colp(u, ldu);
    double v = w[3 * o] * uc[node[3 * o]] + w[3 * o + 1] * uc[node[3 * o + 1]] +
               w[3 * o + 2] * uc[node[3 * o + 2]];
    if (d) v -= d[o];
    colp(out, ldo)[o] = v;
}

// y[node] += scale * (B^T v)[node] over the nodes touched by observations (CSR, fixed order).
__global__ void k_obs_scatter(int nt, const int* __restrict__ tnode, const int* __restrict__ tptr,
                              const int* __restrict__ tent, const double* __restrict__ w,
                              const double* __restrict__ v, int ldv, double scale,
                              double* __restrict__ y, int ldy) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const double* vc = colp(v, ldv);
    double s = 0.0;
    for (int e = tptr[t]; e < tptr[t + 1]; ++e) {
        const int ent = tent[e];
        s += w[ent] * vc[ent / 3];
    }
    colp(y, ldy)[tnode[t]] += scale * s;
}

// ----------------------------------------------------- state equation ---
// -A_FD u_D with u_D = 0 on y = 0 and 1 on y = 1: only row j = N-1 couples to
// the top boundary, through its north edge weight.
__global__ void k_forward_rhs(int N, const double* __restrict__ wN, double* __restrict__ rhs) {
    const int N1 = N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int j = k / N1;
    rhs[k] = (j == N - 1) ? wN[k] : 0.0;
}

__global__ void k_set_top(int N, double* __restrict__ u) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= N) u[knode(i, N, N)] = 1.0;
}

// Per-triangle sensitivity coefficient s_T = (c_T/3)(mhat_a + mhat_r + mhat_b).
__device__ inline double sens_coef(int N, const double* cT, const double* mh, int ci, int cj, int s) {
    if (ci < 0 || ci >= N || cj < 0 || cj >= N) return 0.0;
    int ka, kr, kb;
    tri_nodes(N, ci, cj, s, ka, kr, kb);
    return cT[2 * (cj * N + ci) + s] * (1.0 / 3.0) * (mh[ka] + mh[kr] + mh[kb]);
}

// y[:,c] = scale * (K[s(mhat[:,c])] w)_k on free rows, 0 on Dirichlet rows.
// w is one full state-space vector (its Dirichlet values take part).
__global__ void k_sens(int N, const double* __restrict__ cT, const double* __restrict__ mhat,
                       int ldm, const double* __restrict__ w, double scale, double* __restrict__ y,
                       int ldy) {
    const int N1 = N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int j = k / N1, i = k - j * N1;
    double v = 0.0;
    if (j > 0 && j < N) {
        // Straight-line form: the six triangles around C = (i, j), as in the
        // Hessian output kernel; a triangle outside the mesh (i = 0 or N)
        // reads C in place of its missing nodes and has weight 0, so every
        // load is issued before the first product.  Each edge takes the mean
        // of the coefficients of its two triangles, in the order E, W, N, S.
        const double* mh = colp(mhat, ldm);
        const bool e = i < N, wv = i > 0;
        const int kE = e ? k + 1 : k, kW = wv ? k - 1 : k, kN = k + N1, kS = k - N1;
        const int kNE = e ? k + N1 + 1 : k, kSW = wv ? k - N1 - 1 : k;
        const int c0 = j * N + i;  // cell (i, j)
        const double fe = e ? 1.0 : 0.0, fw = wv ? 1.0 : 0.0;
        const double t1 = fe * cT[e ? 2 * c0 : 0], t2 = fe * cT[e ? 2 * c0 + 1 : 0];
        const double t3 = fw * cT[wv ? 2 * (c0 - 1) : 0], t4 = fe * cT[e ? 2 * (c0 - N) + 1 : 0];
        const double t5 = fw * cT[wv ? 2 * (c0 - N - 1) : 0], t6 = fw * cT[wv ? 2 * (c0 - N - 1) + 1 : 0];
        const double mC = mh[k], mE = mh[kE], mN = mh[kN], mNE = mh[kNE], mW = mh[kW], mS = mh[kS],
                     mSW = mh[kSW];
        const double wk = w[k], wE = w[kE], wW = w[kW], wN = w[kN], wS = w[kS];
        const double s1 = t1 * (1.0 / 3.0) * (mC + mE + mNE);   // (C, E, NE)
        const double s2 = t2 * (1.0 / 3.0) * (mC + mN + mNE);   // (C, N, NE)
        const double s3 = t3 * (1.0 / 3.0) * (mW + mC + mN);    // (W, C, N)
        const double s4 = t4 * (1.0 / 3.0) * (mS + mC + mE);    // (S, C, E)
        const double s5 = t5 * (1.0 / 3.0) * (mSW + mS + mC);   // (SW, S, C)
        const double s6 = t6 * (1.0 / 3.0) * (mSW + mW + mC);   // (SW, W, C)
        if (e) v += 0.5 * (s1 + s4) * (wk - wE);
        if (wv) v += 0.5 * (s3 + s6) * (wk - wW);
        v += 0.5 * (s2 + s3) * (wk - wN);
        v += 0.5 * (s4 + s5) * (wk - wS);
        v *= scale;
    }
    colp(y, ldy)[k] = v;
}

// Hessian output without the prior term (see file header).  gn drops the
// terms that carry the adjoint p.
__global__ void k_hess_out(int N, const double* __restrict__ cT, const double* __restrict__ u,
                           const double* __restrict__ p, const double* __restrict__ uh, int ldu,
                           const double* __restrict__ ph, int ldp, const double* __restrict__ mh,
                           int ldm, double* __restrict__ out, int ldo, int gn,
                           const double* __restrict__ add, int ldadd) {
    const int N1 = N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int j = k / N1, i = k - j * N1;
    // The six triangles around node C = (i, j) (cells split along the SW-NE
    // diagonal), in the order the sum takes them:
    //   cell (i, j):         (C, E, NE), (C, N, NE)
    //   cell (i - 1, j):     (W, C, N)       cell (i, j - 1): (S, C, E)
    //   cell (i - 1, j - 1): (SW, S, C), (SW, W, C)
    // A triangle outside the mesh reads C in place of its missing nodes and
    // has weight 0, so every load is issued before the first product.
    const bool e = i < N, w = i > 0, nn = j < N, sd = j > 0;
    const int kE = e ? k + 1 : k, kW = w ? k - 1 : k, kN = nn ? k + N1 : k, kS = sd ? k - N1 : k;
    const int kNE = e && nn ? k + N1 + 1 : k, kSW = w && sd ? k - N1 - 1 : k;
    const int c0 = j * N + i;  // cell (i, j)
    const double w1 = e && nn ? 1.0 : 0.0, w3 = w && nn ? 1.0 : 0.0, w4 = e && sd ? 1.0 : 0.0,
                 w5 = w && sd ? 1.0 : 0.0;
    const double t1 = w1 * cT[e && nn ? 2 * c0 : 0], t2 = w1 * cT[e && nn ? 2 * c0 + 1 : 0];
    const double t3 = w3 * cT[w && nn ? 2 * (c0 - 1) : 0], t4 = w4 * cT[e && sd ? 2 * (c0 - N) + 1 : 0];
    const double t5 = w5 * cT[w && sd ? 2 * (c0 - N - 1) : 0], t6 = w5 * cT[w && sd ? 2 * (c0 - N - 1) + 1 : 0];
    const int nd[7] = {k, kE, kN, kNE, kW, kS, kSW};  // C E N NE W S SW
    double vu[7], vph[7], vp[7], vuh[7], vmh[7];
    const double* uhc = colp(uh, ldu);
    const double* phc = colp(ph, ldp);
    const double* mhc = colp(mh, ldm);
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        vu[q] = u[nd[q]];
        vph[q] = phc[nd[q]];
        vp[q] = vuh[q] = vmh[q] = 0.0;
    }
    if (!gn) {
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            vp[q] = p[nd[q]];
            vuh[q] = uhc[nd[q]];
            vmh[q] = mhc[nd[q]];
        }
    }
    const double addv = add ? colp(add, ldadd)[k] : 0.0;
    auto tri = [&](int a, int r, int b) {
        double v = tri_form(vu[a], vu[r], vu[b], vph[a], vph[r], vph[b]);
        if (!gn) {
            v += tri_form(vuh[a], vuh[r], vuh[b], vp[a], vp[r], vp[b]);
            v += (1.0 / 3.0) * (vmh[a] + vmh[r] + vmh[b]) * tri_form(vu[a], vu[r], vu[b], vp[a], vp[r], vp[b]);
        }
        return v;
    };
    constexpr int C = 0, E = 1, NN = 2, NE = 3, W = 4, S = 5, SW = 6;
    double acc = 0.0;
    acc += t1 * (1.0 / 3.0) * tri(C, E, NE);
    acc += t2 * (1.0 / 3.0) * tri(C, NN, NE);
    acc += t3 * (1.0 / 3.0) * tri(W, C, NN);
    acc += t4 * (1.0 / 3.0) * tri(S, C, E);
    acc += t5 * (1.0 / 3.0) * tri(SW, S, C);
    acc += t6 * (1.0 / 3.0) * tri(SW, W, C);
    if (add) acc = addv + acc;  // the prior term, as the accumulating apply adds it
    colp(out, ldo)[k] = acc;
}

// g_v = sum_{T ni v} (c_T/3) |T| grad u . grad p  (data part of the gradient).
__global__ void k_grad(int N, const double* __restrict__ cT, const double* __restrict__ u,
                       const double* __restrict__ p, double* __restrict__ g) {
    const int N1 = N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int i = k % N1, j = k / N1;
    double acc = 0.0;
    for_incident_triangles(N, i, j, [&](int ci, int cj, int s, int) {
        int a, r, b;
        tri_nodes(N, ci, cj, s, a, r, b);
        acc += cT[2 * (cj * N + ci) + s] * (1.0 / 3.0) * tri_form(u[a], u[r], u[b], p[a], p[r], p[b]);
    });
    g[k] = acc;
}

// (C_M eta)_v: every edge midpoint of a triangle carries one normal with
// quadrature weight |T|/3 and basis value 1/2 at both edge ends, so the
// entry of C_M is sqrt(|T|/3) / 2 = h / (2 sqrt 6).  Edges in (a, r, b) order:
// e0 = (a, r), e1 = (r, b), e2 = (a, b).
__global__ void k_mass_factor(int N, const double* __restrict__ eta, int lde,
                              double* __restrict__ out, int ldo) {
    const int N1 = N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int i = k % N1, j = k / N1;
    const double* ec = colp(eta, lde);
    double acc = 0.0;
    for_incident_triangles(N, i, j, [&](int ci, int cj, int s, int role) {
        const int t = 2 * (cj * N + ci) + s;
        // a: e0, e2;  r: e0, e1;  b: e1, e2
        const int ea = role == 2 ? 1 : 0;
        const int eb = role == 1 ? 1 : 2;
        acc += ec[3 * t + ea] + ec[3 * t + eb];
    });
    colp(out, ldo)[k] = acc * (0.5 / (N * sqrt(6.0)));
}

// y = op x + beta y (FP64, all rows of the prior / mass operator).
__global__ void k_prior_apply(OpKA<double> op, const double* __restrict__ x, int ldx,
                              double* __restrict__ y, int ldy, double beta) {
    const int N1 = op.N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int i = k % N1, j = k / N1;
    const double* xc = colp(x, ldx);
    double v = op.apply(i, j, k, [&](int, int, int kk) { return xc[kk]; });
    double* yc = colp(y, ldy);
    if (beta != 0.0) v += beta * yc[k];
    yc[k] = v;
}

// Chebyshev iteration for M x = b with the Jacobi-scaled spectrum in [1/2, 2]
// (x = 0, r = b, d = D^-1 b / theta; then per step r <- r - M d, x <- x + d,
// d <- c1 d + c2 D^-1 r), kMassSteps steps per launch on LDS tiles: a
// workgroup owns T x T nodes (T = 32, or 16 when the 32-tiles would leave
// most of the GPU idle) and holds r and d on a halo of kMassSteps rings, so
// step s updates the tile shrunk by s + 1 rings from values it holds.  The
// next launch reads the other copy of r and d (the halos of a tile are owned
// by its neighbours).
constexpr int kMassSteps = 8;
struct MassSteps {
    double c1[kMassSteps], c2[kMassSteps];
};

template <int T>
__global__ __launch_bounds__(256) void k_cheb_mass(OpKA<double> op, const double* __restrict__ b, int ldb,
                                                   double* __restrict__ x, const double* __restrict__ r_in,
                                                   const double* __restrict__ d_in, double* __restrict__ r_out,
                                                   double* __restrict__ d_out, int ld, MassSteps cs, int first,
                                                   double inv_theta) {
    constexpr int H = kMassSteps, W = T + 2 * H, NN = W * W, E = (NN + 255) / 256;
    constexpr int OWN = (T * T + 255) / 256;
    __shared__ double sr[NN], sd[NN];
    const int N = op.N, N1 = N + 1;
    const int ox = blockIdx.x * T - H, oy = blockIdx.y * T - H;  // node of local (0, 0)
    const size_t co = (size_t)blockIdx.z * ld;
    // loads first (r and d, or b on the first launch; x of the owned nodes)
    double vr[E], vd[E], vx[OWN];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = threadIdx.x + 256 * e;
        const int i = ox + t % W, j = oy + t / W;
        const bool in = t < NN && i >= 0 && i <= N && j >= 0 && j <= N;
        const int k = j * N1 + i;
        vr[e] = vd[e] = 0.0;
        if (in) {
            if (first) {
                const double bv = b[(size_t)blockIdx.z * ldb + k];
                vr[e] = bv;
                vd[e] = op.inv_diag(i, j, k) * bv * inv_theta;
            } else {
                vr[e] = r_in[co + k];
                vd[e] = d_in[co + k];
            }
        }
    }
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
        const int t = threadIdx.x + 256 * o;
        const int i = ox + H + t % T, j = oy + H + t / T;
        vx[o] = (!first && t < T * T && i <= N && j <= N) ? x[co + j * N1 + i] : 0.0;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = threadIdx.x + 256 * e;
        if (t < NN) {
            sr[t] = vr[e];
            sd[t] = vd[e];
        }
    }
    __syncthreads();
    // Tiles strictly inside the mesh (every node 1 <= i, j <= N - 1) have the
    // interior row everywhere: its seven couplings stay in scalar registers.
    const bool inner = ox >= 1 && oy >= 1 && ox + W <= N && oy + W <= N;
    if (inner) {
        const KARow<double>& q0 = op.rows[0];
        const double mc = q0.c, me = q0.e, mw = q0.w, mn = q0.n, ms = q0.s, mne = q0.ne, msw = q0.sw;
        const double mdv = q0.dinv;
        for (int st = 0; st < H; ++st) {
            const int lo = st + 1, hi = W - lo;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int t = threadIdx.x + 256 * e;
                const int li = t % W, lj = t / W;
                if (t >= NN || li < lo || li >= hi || lj < lo || lj >= hi) continue;
                const double Md = mc * sd[t] + me * sd[t + 1] + mw * sd[t - 1] + mn * sd[t + W] + ms * sd[t - W] +
                                  mne * sd[t + W + 1] + msw * sd[t - W - 1];
                sr[t] = sr[t] - Md;
            }
#pragma unroll
            for (int o = 0; o < OWN; ++o) {
                const int t = threadIdx.x + 256 * o;
                if (t < T * T) vx[o] += sd[(H + t / T) * W + H + t % T];
            }
            __syncthreads();
            const double c1 = cs.c1[st], c2 = cs.c2[st];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int t = threadIdx.x + 256 * e;
                const int li = t % W, lj = t / W;
                if (t >= NN || li < lo || li >= hi || lj < lo || lj >= hi) continue;
                sd[t] = c1 * sd[t] + c2 * mdv * sr[t];
            }
            __syncthreads();
        }
    }
    for (int st = 0; !inner && st < H; ++st) {
        const int lo = st + 1, hi = W - lo;  // region [lo, hi)^2
        // r <- r - M d on the region (each r read and written by one thread);
        // x <- x + d on the owned nodes, before d changes.  The loops walk the
        // whole tile (compile-time width) and skip what lies outside.
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = threadIdx.x + 256 * e;
            const int li = t % W, lj = t / W, i = ox + li, j = oy + lj;
            if (t >= NN || li < lo || li >= hi || lj < lo || lj >= hi) continue;
            if (i < 0 || i > N || j < 0 || j > N) continue;
            const double Md = op.apply(i, j, j * N1 + i, [&](int ii, int jj, int) {
                return sd[(jj - oy) * W + (ii - ox)];
            });
            sr[t] = sr[t] - Md;
        }
#pragma unroll
        for (int o = 0; o < OWN; ++o) {
            const int t = threadIdx.x + 256 * o;
            if (t < T * T) vx[o] += sd[(H + t / T) * W + H + t % T];
        }
        __syncthreads();
        const double c1 = cs.c1[st], c2 = cs.c2[st];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = threadIdx.x + 256 * e;
            const int li = t % W, lj = t / W, i = ox + li, j = oy + lj;
            if (t >= NN || li < lo || li >= hi || lj < lo || lj >= hi) continue;
            if (i < 0 || i > N || j < 0 || j > N) continue;
            sd[t] = c1 * sd[t] + c2 * op.inv_diag(i, j, j * N1 + i) * sr[t];
        }
        __syncthreads();
    }
#pragma unroll
    for (int o = 0; o < OWN; ++o) {
        const int t = threadIdx.x + 256 * o;
        const int i = ox + H + t % T, j = oy + H + t / T;
        if (t < T * T && i <= N && j <= N) {
            const int l = (H + t / T) * W + H + t % T;
            const size_t k = co + j * N1 + i;
            x[k] = vx[o];
            r_out[k] = sr[l];
            d_out[k] = sd[l];
        }
    }
}

__global__ void k_add_scalar(int n, double v, double* __restrict__ x, int ld) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) colp(x, ld)[k] += v;
}

__global__ void k_axpby(int n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) y[k] = a * x[k] + b * y[k];
}

__global__ void k_fill(int n, double v, double* __restrict__ y) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) y[k] = v;
}

__global__ void k_copy(int n, const double* __restrict__ x, int ldx, double* __restrict__ y, int ldy) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) colp(y, ldy)[k] = colp(x, ldx)[k];
}

__global__ void k_dot_partial(int n, const double* __restrict__ a, int lda,
                              const double* __restrict__ b, int ldb, double* __restrict__ partial) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (k < n) v = colp(a, lda)[k] * colp(b, ldb)[k];
    const double s = block_sum(v);
    if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ void k_dot_finish(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) v += partial[(size_t)blockIdx.x * nblk + b];
    const double s = block_sum(v);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// ------------------------------------------------------------ white noise ---
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 64x64
// multiplications with Weyl-sequence key increments.
__device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += W0;
        k1 += W1;
    }
}

// Box-Muller on one word pair: u1 in (0, 1], u2 in [0, 1).
__device__ inline void box_muller(uint64_t w0, uint64_t w1, double& z0, double& z1) {
    const double u1 = ((double)(w0 >> 11) + 1.0) * 0x1.0p-53;
    const double u2 = (double)(w1 >> 11) * 0x1.0p-53;
    const double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// eta[:, s] for samples first .. first+ns-1: sample S takes the stream words
// [S L, (S+1) L), word w from counter block w / 4 + 1 (L = 6 N^2, 4 | L).
__global__ void k_white_noise(int L, uint64_t seed, uint64_t stream, long long first,
                              double* __restrict__ eta, int ld) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;  // block within the sample
    if (4 * b >= L) return;
    const unsigned long long blk = (unsigned long long)(first + blockIdx.y) * (L / 4) + b + 1;
    uint64_t c[4] = {blk, 0, 0, 0};
    philox4x64_10(c, seed, stream);
    double* e = eta + (size_t)blockIdx.y * ld + 4 * b;
    box_muller(c[0], c[1], e[0], e[1]);
    box_muller(c[2], c[3], e[2], e[3]);
}

OpKA<double> prior_op(int N, const PriorParams& pp) { return make_prior_op<double>(N, pp); }

// The mass matrix as a prior operator (gamma = 0, delta = 1, beta = 0).
OpKA<double> mass_op(int N) { return make_prior_op<double>(N, PriorParams{0.0, 1.0, 0.0}); }

// Chebyshev iteration count for M: error factor 2 (1/3)^K = 7.1e-12 at K = 24,
// below the 1e-10 relative residual every PDE solve runs to (32 steps, to
// 2e-15, cost a fourth more in every application of R).
constexpr int kMassCheb = 24;
static_assert(kMassCheb % kMassSteps == 0, "mass Chebyshev steps come in whole launches");

}  // namespace

// ----------------------------------------------------------- vector ops ---
void dev_dots(Ctx* ctx, int n, int nc, const double* a, int lda, const double* b, int ldb,
              double* host_out) {
    const int nblk = ceil_div(n, kBlock);
    ctx->red.ensure((size_t)nblk * nc + nc);
    k_dot_partial<<<grid2(n, nc), kBlock, 0, ctx->stream>>>(n, a, lda, b, ldb, ctx->red.get());
    HINV_LAUNCH_CHECK();
    double* out = ctx->red.get() + (size_t)nblk * nc;
    k_dot_finish<<<nc, kBlock, 0, ctx->stream>>>(ctx->red.get(), nblk, out);
    HINV_LAUNCH_CHECK();
    // through pinned memory: a pageable destination adds a staging copy to
    // every read-back of the Newton-CG loop
    if (!ctx->host_red) HINV_HIP(hipHostMalloc((void**)&ctx->host_red, sizeof(double) * Ctx::kHostRed,
                                               hipHostMallocDefault));
    for (int c0 = 0; c0 < nc; c0 += Ctx::kHostRed) {
        const int m = std::min(Ctx::kHostRed, nc - c0);
        HINV_HIP(hipMemcpyAsync(ctx->host_red, out + c0, sizeof(double) * m, hipMemcpyDeviceToHost, ctx->stream));
        HINV_HIP(hipStreamSynchronize(ctx->stream));
        std::memcpy(host_out + c0, ctx->host_red, sizeof(double) * m);
    }
}

void dev_dot_to(Ctx* ctx, int n, const double* a, const double* b, double* out) {
    const int nblk = ceil_div(n, kBlock);
    ctx->red.ensure((size_t)nblk + 1);
    k_dot_partial<<<grid2(n, 1), kBlock, 0, ctx->stream>>>(n, a, n, b, n, ctx->red.get());
    HINV_LAUNCH_CHECK();
    k_dot_finish<<<1, kBlock, 0, ctx->stream>>>(ctx->red.get(), nblk, out);
    HINV_LAUNCH_CHECK();
}

double dev_dot(Ctx* ctx, int n, const double* a, const double* b) {
    double r;
    dev_dots(ctx, n, 1, a, n, b, n, &r);
    return r;
}

void dev_axpby(Ctx* ctx, int n, double a, const double* x, double b, double* y) {
    k_axpby<<<ceil_div(n, kBlock), kBlock, 0, ctx->stream>>>(n, a, x, b, y);
    HINV_LAUNCH_CHECK();
}

void dev_copy(Ctx* ctx, int n, int nc, const double* x, int ldx, double* y, int ldy) {
    if (nc <= 0) return;
    k_copy<<<grid2(n, nc), kBlock, 0, ctx->stream>>>(n, x, ldx, y, ldy);
    HINV_LAUNCH_CHECK();
}

void dev_fill(Ctx* ctx, int n, double v, double* y) {
    k_fill<<<ceil_div(n, kBlock), kBlock, 0, ctx->stream>>>(n, v, y);
    HINV_LAUNCH_CHECK();
}

// -------------------------------------------------------------- problem ---
Problem::Problem(Ctx* c, const hinv_problem_desc& desc)
    : ctx(c), N(desc.N), n((desc.N + 1) * (desc.N + 1)), q(desc.q), gamma(desc.gamma),
      delta(desc.delta), m_prior(desc.m_prior), sigma(desc.sigma), precision(desc.precision),
      rtol(desc.rtol), max_iter(desc.max_iter > 0 ? desc.max_iter : 200) {
    beta = std::isnan(desc.beta) ? std::sqrt(gamma * delta) / 1.42 : desc.beta;
    PriorParams pp{gamma, delta, beta};
    if (desc.theta1 > 0.0) {
        // Theta = theta1 v v^T + theta2 w w^T, v = (sin a, cos a), w = (cos a, -sin a):
        // the s.p.d. tensor with the eigenvalues and directions Sec. 5.1 states
        const double sa = std::sin(desc.alpha), ca = std::cos(desc.alpha);
        pp.t11 = desc.theta1 * sa * sa + desc.theta2 * ca * ca;
        pp.t12 = (desc.theta1 - desc.theta2) * sa * ca;
        pp.t22 = desc.theta1 * ca * ca + desc.theta2 * sa * sa;
    }
    prior = pp;
    deg = desc.state_degree == 2 ? 2 : 1;
    ns = deg == 2 ? (2 * N + 1) * (2 * N + 1) : n;
    HA = std::make_unique<Hierarchy>(ctx, kOpState, N, pp);
    HK = std::make_unique<Hierarchy>(ctx, kOpPrior, N, pp);
    if (deg == 2) S2 = std::make_unique<P2Space>(ctx, N);
    m_lin.ensure(n);
    u_lin.ensure(ns);
    p_lin.ensure(ns);
    hipStream_t s = ctx->stream;
    if (q > 0) {
        obs_xy.ensure(2 * (size_t)q);
        obs_w.ensure(3 * (size_t)q);
        obs_node.ensure(3 * (size_t)q);
        d.ensure(q);
        HINV_HIP(hipMemcpyAsync(obs_xy.get(), desc.obs_xy, sizeof(double) * 2 * q, hipMemcpyHostToDevice, s));
        k_obs_setup<<<ceil_div(q, kBlock), kBlock, 0, s>>>(N, q, obs_xy.get(), obs_node.get(), obs_w.get());
        HINV_LAUNCH_CHECK();
        // transpose structure: node -> list of (3 o + a), built from the device's node indices
        std::vector<int> hn(3 * (size_t)q);
        HINV_HIP(hipMemcpyAsync(hn.data(), obs_node.get(), sizeof(int) * 3 * q, hipMemcpyDeviceToHost, s));
        HINV_HIP(hipStreamSynchronize(s));
        std::vector<int> order(3 * (size_t)q);
        for (int e = 0; e < 3 * q; ++e) order[e] = e;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hn[a] < hn[b]; });
        std::vector<int> tn, tp, te;
        for (int e = 0; e < 3 * q; ++e) {
            const int nd = hn[order[e]];
            if (tn.empty() || tn.back() != nd) {
                tn.push_back(nd);
                tp.push_back(e);
            }
            te.push_back(order[e]);
        }
        tp.push_back(3 * q);
        n_touch = (int)tn.size();
        t_node.ensure(tn.size());
        t_ptr.ensure(tp.size());
        t_ent.ensure(te.size());
        HINV_HIP(hipMemcpyAsync(t_node.get(), tn.data(), sizeof(int) * tn.size(), hipMemcpyHostToDevice, s));
        HINV_HIP(hipMemcpyAsync(t_ptr.get(), tp.data(), sizeof(int) * tp.size(), hipMemcpyHostToDevice, s));
        HINV_HIP(hipMemcpyAsync(t_ent.get(), te.data(), sizeof(int) * te.size(), hipMemcpyHostToDevice, s));
        HINV_HIP(hipStreamSynchronize(s));
        if (S2) S2->set_observations(q, obs_xy.get());
        set_data(desc.d_obs, sigma);
    }
}

void Problem::set_data(const double* d_host, double sig) {
    if (sig > 0) sigma = sig;
    if (q == 0) return;
    hipStream_t s = ctx->stream;
    if (d_host) {
        HINV_HIP(hipMemcpyAsync(d.get(), d_host, sizeof(double) * q, hipMemcpyHostToDevice, s));
        HINV_HIP(hipStreamSynchronize(s));
    } else {
        k_fill<<<ceil_div(q, kBlock), kBlock, 0, s>>>(q, 0.0, d.get());
        HINV_LAUNCH_CHECK();
    }
}

double* Problem::scratch(int which, int nc) {
    if (which < 0 || which >= kScratch) fail(HINV_EINVAL, "internal: scratch index out of range");
    if (nc > cap_) {
        for (auto& w : w_) w.release();
        for (auto& w : w_) w.ensure((size_t)std::max(n, ns) * nc);
        cap_ = nc;
    }
    return w_[which].get();
}

double* Problem::obs_scratch(int nc) {
    if (nc > qcap_) {
        wq_.ensure((size_t)std::max(q, 1) * nc);
        qcap_ = nc;
    }
    return wq_.get();
}

void Problem::set_state(const double* m) {
    HA->set_state_coefficient(m);
    if (S2) S2->set_coefficient(HA->coefficient());
}

void Problem::state_solve(int nc, const double* b, int ldb, double* x, int ldx, double tol, SolveStats* st,
                          double accept) {
    if (S2)
        S2->solve(nc, b, ldb, x, ldx, *HA, tol, max_iter, st);
    else
        HA->solve(nc, b, ldb, x, ldx, precision, tol, max_iter, st, accept);
}

void Problem::state_apply(int nc, const double* x, int ldx, double* y, int ldy) {
    if (S2)
        S2->apply(nc, x, ldx, y, ldy, 1.0);
    else
        HA->apply(nc, x, ldx, y, ldy);
}

void Problem::forward(const double* m, double* u, SolveStats* st) {
    hipStream_t s = ctx->stream;
    set_state(m);
    ha_is_lin = false;
    double* rhs = scratch(0, 1);
    if (S2) {
        S2->forward_rhs(rhs);
        state_solve(1, rhs, ns, u, ns, rtol, st);
        S2->set_top(u);
        return;
    }
    k_forward_rhs<<<ceil_div(n, kBlock), kBlock, 0, s>>>(N, HA->weightsN(), rhs);
    HINV_LAUNCH_CHECK();
    HA->solve(1, rhs, n, u, n, precision, rtol, max_iter, st);
    k_set_top<<<ceil_div(N + 1, kBlock), kBlock, 0, s>>>(N, u);
    HINV_LAUNCH_CHECK();
}

void Problem::observe(const double* u, int ldu, int nc, double* out, int ldo, bool minus_data) {
    if (q == 0) return;
    if (S2) {
        S2->observe(nc, u, ldu, minus_data ? d.get() : nullptr, out, ldo);
        return;
    }
    k_obs_gather<<<grid2(q, nc), kBlock, 0, ctx->stream>>>(q, obs_node.get(), obs_w.get(), u, ldu,
                                                           minus_data ? d.get() : nullptr, out, ldo);
    HINV_LAUNCH_CHECK();
}

void Problem::cost(const double* m, const double* u, double* misfit, double* reg) {
    double mis = 0.0;
    if (q > 0) {
        double* r = obs_scratch(1);
        observe(u, ns, 1, r, q, true);
        double ss;
        dev_dots(ctx, q, 1, r, q, r, q, &ss);
        mis = 0.5 * ss / (sigma * sigma);
    }
    double* dm = scratch(0, 1);
    double* Rdm = scratch(1, 1);
    dev_copy(ctx, n, 1, m, n, dm, n);
    k_add_scalar<<<ceil_div(n, kBlock), kBlock, 0, ctx->stream>>>(n, -m_prior, dm, n);
    HINV_LAUNCH_CHECK();
    prior_apply(1, dm, n, Rdm, n);
    *misfit = mis;
    *reg = 0.5 * dev_dot(ctx, n, dm, Rdm);
}

void Problem::gradient(const double* m, const double* u, double* p, double* g, SolveStats* st) {
    hipStream_t s = ctx->stream;
    set_state(m);
    ha_is_lin = false;
    double* rhs = scratch(0, 1);
    k_fill<<<ceil_div(ns, kBlock), kBlock, 0, s>>>(ns, 0.0, rhs);
    HINV_LAUNCH_CHECK();
    if (q > 0) {
        double* r = obs_scratch(1);
        observe(u, ns, 1, r, q, true);
        if (S2) {
            S2->observe_adjoint(1, r, q, -1.0 / (sigma * sigma), rhs, ns);
        } else {
            k_obs_scatter<<<ceil_div(n_touch, kBlock), kBlock, 0, s>>>(
                n_touch, t_node.get(), t_ptr.get(), t_ent.get(), obs_w.get(), r, q,
                -1.0 / (sigma * sigma), rhs, n);
            HINV_LAUNCH_CHECK();
        }
    }
    state_solve(1, rhs, ns, p, ns, rtol, st);
    if (S2) {
        S2->grad(u, p, g);
    } else {
        k_grad<<<ceil_div(n, kBlock), kBlock, 0, s>>>(N, HA->coefficient(), u, p, g);
        HINV_LAUNCH_CHECK();
    }
    double* dm = scratch(1, 1);
    dev_copy(ctx, n, 1, m, n, dm, n);
    k_add_scalar<<<ceil_div(n, kBlock), kBlock, 0, s>>>(n, -m_prior, dm, n);
    HINV_LAUNCH_CHECK();
    prior_apply(1, dm, n, g, n, /*accumulate=*/true);
}

void Problem::linearize(const double* m, const double* u, const double* p) {
    dev_copy(ctx, n, 1, m, n, m_lin.get(), n);
    dev_copy(ctx, ns, 1, u, ns, u_lin.get(), ns);
    dev_copy(ctx, ns, 1, p, ns, p_lin.get(), ns);
    set_state(m_lin.get());
    ha_is_lin = true;
    linearized = true;
    ++lin_version;
}

void Problem::ensure_lin_hierarchy() {
    if (!linearized) fail(HINV_ESTATE, "Hessian action before hinv_linearize");
    if (!ha_is_lin) {
        set_state(m_lin.get());
        ha_is_lin = true;
    }
}

// Right-hand side -[C(u) mhat]_F of the incremental forward problem.
void Problem::inc_forward_rhs(int nc, const double* mhat, int ldm, double* rhs, int ldr) {
    ensure_lin_hierarchy();
    if (S2) {
        S2->sens(nc, mhat, ldm, u_lin.get(), -1.0, rhs, ldr);
        return;
    }
    k_sens<<<grid2(n, nc), kBlock, 0, ctx->stream>>>(N, HA->coefficient(), mhat, ldm, u_lin.get(),
                                                     -1.0, rhs, ldr);
    HINV_LAUNCH_CHECK();
}

// Right-hand side -[B^T B uhat / sigma^2 + C(p) mhat]_F of the incremental
// adjoint problem (Gauss-Newton drops C(p) mhat).
void Problem::inc_adjoint_rhs(int nc, bool gn, const double* mhat, int ldm, const double* uhat,
                              int ldu, double* rhs, int ldr) {
    ensure_lin_hierarchy();
    hipStream_t s = ctx->stream;
    if (S2) {
        // the scale 0 zeroes the column under Gauss-Newton
        S2->sens(nc, mhat, ldm, p_lin.get(), gn ? 0.0 : -1.0, rhs, ldr);
        if (q > 0) {
            double* Bu = obs_scratch(nc);
            observe(uhat, ldu, nc, Bu, q, false);
            S2->observe_adjoint(nc, Bu, q, -1.0 / (sigma * sigma), rhs, ldr);
        }
        return;
    }
    // the scale 0 zeroes the column under Gauss-Newton
    k_sens<<<grid2(n, nc), kBlock, 0, s>>>(N, HA->coefficient(), mhat, ldm, p_lin.get(),
                                           gn ? 0.0 : -1.0, rhs, ldr);
    HINV_LAUNCH_CHECK();
    if (q > 0) {
        double* Bu = obs_scratch(nc);
        observe(uhat, ldu, nc, Bu, q, false);
        k_obs_scatter<<<grid2(n_touch, nc), kBlock, 0, s>>>(n_touch, t_node.get(), t_ptr.get(),
                                                            t_ent.get(), obs_w.get(), Bu, q,
                                                            -1.0 / (sigma * sigma), rhs, ldr);
        HINV_LAUNCH_CHECK();
    }
}

// Hessian action from the incremental states (and R mhat for the full modes).
void Problem::hess_output(int mode, int nc, const double* mhat, int ldm, const double* uh, int ldu,
                          const double* ph, int ldp, double* out, int ldo, const double* rm) {
    const bool gn = mode == HINV_HESS_GN_FULL || mode == HINV_HESS_GN_MISFIT;
    const bool with_prior = mode == HINV_HESS_FULL || mode == HINV_HESS_GN_FULL;
    if (S2) {
        S2->hess_out(nc, gn, u_lin.get(), p_lin.get(), uh, ldu, ph, ldp, mhat, ldm, out, ldo,
                     with_prior ? rm : nullptr, n);
        if (with_prior && !rm) prior_apply(nc, mhat, ldm, out, ldo, true);
        return;
    }
    k_hess_out<<<grid2(n, nc), kBlock, 0, ctx->stream>>>(N, HA->coefficient(), u_lin.get(),
                                                         p_lin.get(), uh, ldu, ph, ldp, mhat, ldm,
                                                         out, ldo, gn ? 1 : 0, with_prior ? rm : nullptr, n);
    HINV_LAUNCH_CHECK();
    if (with_prior && !rm) prior_apply(nc, mhat, ldm, out, ldo, true);
}

hipStream_t Problem::side_stream() {
    if (!side_) {
        HINV_HIP(hipStreamCreateWithFlags(&side_, hipStreamNonBlocking));
        HINV_HIP(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming));
        HINV_HIP(hipEventCreateWithFlags(&ev_join_, hipEventDisableTiming));
    }
    return side_;
}

Problem::~Problem() {
    if (side_) {
        (void)hipStreamSynchronize(side_);
        (void)hipEventDestroy(ev_fork_);
        (void)hipEventDestroy(ev_join_);
        (void)hipStreamDestroy(side_);
    }
}

void Problem::inc_forward(int nc, const double* mhat, int ldm, double* uhat, int ldu, SolveStats* st,
                          double tol) {
    double* rhs = scratch(0, nc);
    inc_forward_rhs(nc, mhat, ldm, rhs, ns);
    // a tighter goal still accepts the problem's tolerance at the rounding floor
    state_solve(nc, rhs, ns, uhat, ldu, tol > 0 ? tol : rtol, st, rtol);
}

void Problem::inc_adjoint(int nc, bool gn, const double* mhat, int ldm, const double* uhat, int ldu,
                          double* phat, int ldp, SolveStats* st) {
    double* rhs = scratch(0, nc);
    inc_adjoint_rhs(nc, gn, mhat, ldm, uhat, ldu, rhs, ns);
    state_solve(nc, rhs, ns, phat, ldp, rtol, st);
}

void Problem::hessian(int mode, int nc, const double* mhat, int ldm, double* out, int ldo,
                      SolveStats* st) {
    const bool gn = mode == HINV_HESS_GN_FULL || mode == HINV_HESS_GN_MISFIT;
    const bool with_prior = mode == HINV_HESS_FULL || mode == HINV_HESS_GN_FULL;
    scratch(0, nc);
    double* uh = scratch(1, nc);
    double* ph = scratch(2, nc);
    // R mhat does not depend on the two solves: it runs on the side stream
    // meanwhile (its own scratch 3-9), joined before the output kernel adds it
    double* rm = nullptr;
    if (with_prior) {
        rm = scratch(9, nc);
        hipStream_t side = side_stream();
        HINV_HIP(hipEventRecord(ev_fork_, ctx->stream));
        HINV_HIP(hipStreamWaitEvent(side, ev_fork_, 0));
        prior_apply(nc, mhat, ldm, rm, n, false, side);
        HINV_HIP(hipEventRecord(ev_join_, side));
    }
    // the P2 state solves in FP64 PCG: no chained tightening
    inc_forward(nc, mhat, ldm, uh, ns, st, S2 ? rtol : chained_first_rtol(precision, nc, rtol));
    inc_adjoint(nc, gn, mhat, ldm, uh, ns, ph, ns, st);
    if (with_prior) HINV_HIP(hipStreamWaitEvent(ctx->stream, ev_join_, 0));
    hess_output(mode, nc, mhat, ldm, uh, ns, ph, ns, out, ldo, rm);
}

void Problem::mass_apply(int nc, const double* x, int ldx, double* y, int ldy) {
    k_prior_apply<<<grid2(n, nc), kBlock, 0, ctx->stream>>>(mass_op(N), x, ldx, y,
                                                            ldy, 0.0);
    HINV_LAUNCH_CHECK();
}

void Problem::mass_solve(int nc, const double* b, int ldb, double* x, int ldx, hipStream_t s, double* ws) {
    // Chebyshev iteration (no inner products) on the Jacobi-scaled consistent
    // mass matrix, whose spectrum lies in [1/2, 2] for P1 triangles.
    if (!s) s = ctx->stream;
    const OpKA<double> M = mass_op(N);
    const double lo = 0.5, hi = 2.0;
    const double theta = 0.5 * (hi + lo), dl = 0.5 * (hi - lo), sigma1 = theta / dl;
    const size_t blk = (size_t)n * nc;
    double* r[2] = {ws ? ws : scratch(5, nc), ws ? ws + 3 * blk : scratch(8, nc)};
    double* d[2] = {ws ? ws + blk : scratch(6, nc), ws ? ws + 2 * blk : scratch(7, nc)};
    if (ldx != n) fail(HINV_EINVAL, "mass_solve needs a packed output");
    if (nc > 65535) fail(HINV_EINVAL, "mass_solve: at most 65535 columns per call");
    const bool small = (long long)ceil_div(N + 1, 32) * ceil_div(N + 1, 32) * nc < 512;
    const int tiles = ceil_div(N + 1, small ? 16 : 32);
    double rho = 1.0 / sigma1;
    for (int launch = 0; launch < kMassCheb / kMassSteps; ++launch) {
        MassSteps cs;
        for (int st = 0; st < kMassSteps; ++st) {
            const double rho_n = 1.0 / (2.0 * sigma1 - rho);
            cs.c1[st] = rho_n * rho;
            cs.c2[st] = 2.0 * rho_n / dl;
            rho = rho_n;
        }
        const int in = launch & 1;
        if (small)
            k_cheb_mass<16><<<dim3(tiles, tiles, nc), 256, 0, s>>>(M, b, ldb, x, r[in], d[in], r[1 - in],
                                                                   d[1 - in], n, cs, launch == 0, 1.0 / theta);
        else
            k_cheb_mass<32><<<dim3(tiles, tiles, nc), 256, 0, s>>>(M, b, ldb, x, r[in], d[in], r[1 - in],
                                                                   d[1 - in], n, cs, launch == 0, 1.0 / theta);
        HINV_LAUNCH_CHECK();
    }
}

void Problem::prior_apply(int nc, const double* x, int ldx, double* y, int ldy, bool accumulate,
                          hipStream_t s, double* ws) {
    if (!s) s = ctx->stream;
    const OpKA<double> K = prior_op(N, prior);
    const size_t blk = (size_t)n * nc;
    double* t1 = ws ? ws : scratch(3, nc);
    double* t2 = ws ? ws + blk : scratch(4, nc);
    k_prior_apply<<<grid2(n, nc), kBlock, 0, s>>>(K, x, ldx, t1, n, 0.0);
    HINV_LAUNCH_CHECK();
    mass_solve(nc, t1, n, t2, n, s, ws ? ws + 2 * blk : nullptr);
    k_prior_apply<<<grid2(n, nc), kBlock, 0, s>>>(K, t2, n, y, ldy, accumulate ? 1.0 : 0.0);
    HINV_LAUNCH_CHECK();
}

void Problem::prior_solve(int nc, const double* x, int ldx, double* y, int ldy, SolveStats* st) {
    double* t1 = scratch(3, nc);
    double* t2 = scratch(4, nc);
    HK->solve(nc, x, ldx, t1, n, precision, rtol, max_iter, st);
    mass_apply(nc, t1, n, t2, n);
    HK->solve(nc, t2, n, y, ldy, precision, rtol, max_iter, st);
}

void Problem::white_noise(uint64_t seed, uint64_t stream, long long first, int ns, double* eta,
                          int ld) {
    const int L = 6 * N * N;
    k_white_noise<<<dim3(ceil_div(L / 4, kBlock), ns), kBlock, 0, ctx->stream>>>(L, seed, stream, first,
                                                                                  eta, ld);
    HINV_LAUNCH_CHECK();
}

void Problem::prior_sample(int ns, const double* eta, int ldeta, double* out, int ldo,
                           bool add_mean, SolveStats* st) {
    double* t = scratch(3, ns);
    k_mass_factor<<<grid2(n, ns), kBlock, 0, ctx->stream>>>(N, eta, ldeta, t, n);
    HINV_LAUNCH_CHECK();
    HK->solve(ns, t, n, out, ldo, precision, rtol, max_iter, st);
    if (add_mean) {
        k_add_scalar<<<grid2(n, ns), kBlock, 0, ctx->stream>>>(n, m_prior, out, ldo);
        HINV_LAUNCH_CHECK();
    }
}

}  // namespace hinv
