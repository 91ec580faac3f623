// Flexible CG with the learned correction, and the harvest of its training
// pairs (see fcg.h).  Vector work runs in kernels; the host makes the scalar
// decisions of the Krylov loop.
#include <algorithm>
#include <cmath>
#include <vector>

#include "fcg.h"

namespace hinv {

namespace {

__device__ inline short bf16_of(double x) {
    unsigned u = __float_as_uint((float)x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// Network input on the full grid (pixel (i, j) = node j (N+1) + i):
// channels (t / s, m, free-node mask), padded with zeros to 16.
__global__ void k_fcg_input(int N, const double* __restrict__ t, double inv_s, const double* __restrict__ m,
                            short* __restrict__ in) {
    const int N1 = N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int j = k / N1;
    const bool fr = j > 0 && j < N;
    short* o = in + (size_t)k * Cnn::kPadIn;
    o[0] = bf16_of(fr ? t[k] * inv_s : 0.0);
    o[1] = bf16_of(m[k]);
    o[2] = bf16_of(fr ? 1.0 : 0.0);
    for (int c = 3; c < Cnn::kPadIn; ++c) o[c] = 0;
}

// c = s y on free nodes, 0 on Dirichlet rows (y: channel 0 of the network output).
__global__ void k_fcg_correction(int N, const float* __restrict__ y, double s, double* __restrict__ cv) {
    const int N1 = N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int j = k / N1;
    cv[k] = (j > 0 && j < N) ? s * (double)y[(size_t)k * Cnn::kPadIn] : 0.0;
}

// y = a x + b y on free nodes, 0 on Dirichlet rows (column blockIdx.y).
__global__ void k_axpby_free(int N, double a, const double* __restrict__ x, int ldx, double b,
                             double* __restrict__ y, int ldy) {
    const int N1 = N + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N1 * N1) return;
    const int j = k / N1;
    const double* xc = x + (size_t)blockIdx.y * ldx;
    double* yc = y + (size_t)blockIdx.y * ldy;
    yc[k] = (j > 0 && j < N) ? a * xc[k] + b * yc[k] : 0.0;
}

// One crop per column (workgroup): rms s of r' over the window, then
// in = (r' / s, m, mask) and target = (e' / s, wE, wN, diagonal of A), planar.
__global__ void k_harvest_crop(int N, int crop, const int* __restrict__ org, const double* __restrict__ rp,
                               const double* __restrict__ ep, int ld, const double* __restrict__ m,
                               const double* __restrict__ wE, const double* __restrict__ wN,
                               const double* __restrict__ dinv, float* __restrict__ in,
                               float* __restrict__ tg) {
    const int N1 = N + 1, c = blockIdx.x;
    const int ox = org[2 * c], oy = org[2 * c + 1];
    const double* r = rp + (size_t)c * ld;
    const double* e = ep + (size_t)c * ld;
    const int np = crop * crop;
    double ss = 0.0;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const double v = r[(oy + p / crop) * N1 + ox + p % crop];
        ss += v * v;
    }
    __shared__ double part[256];
    part[threadIdx.x] = ss;
    __syncthreads();
    __shared__ double inv_s;
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += part[i];
        const double s = sqrt(t / np);
        inv_s = s > 0.0 ? 1.0 / s : 0.0;
    }
    __syncthreads();
    float* o = in + (size_t)c * 3 * np;
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
        const int j = oy + p / crop, k = j * N1 + ox + p % crop;
        const bool fr = j > 0 && j < N;
        o[p] = (float)(r[k] * inv_s);
        o[np + p] = (float)m[k];
        o[2 * np + p] = fr ? 1.f : 0.f;
        float* t = tg + (size_t)c * 4 * np;
        t[p] = (float)(e[k] * inv_s);
        t[np + p] = (float)wE[k];
        t[2 * np + p] = (float)wN[k];
        t[3 * np + p] = dinv[k] > 0.0 ? (float)(1.0 / dinv[k]) : 0.f;
    }
}

uint64_t splitmix(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

}  // namespace

void state_solve_fcg(Problem& P, Cnn* cnn, const double* b, double* x, double rtol, int max_iter,
                     int truncation, FcgStats* out) {
    P.ensure_lin_hierarchy();
    Ctx* c = P.ctx;
    hipStream_t s = c->stream;
    const int N = P.N, n = P.n, mt = truncation;
    Hierarchy& H = *P.HA;
    double* r = P.scratch(0, 1);
    double* z = P.scratch(1, 1);
    double* t = P.scratch(2, 1);
    double* cv = P.scratch(4, 1);
    double* Acv = P.scratch(5, 1);
    // the last mt directions p_j and q_j = A p_j (ring buffer)
    P.ws_fcg.ensure((size_t)2 * mt * n);
    double* Pd = P.ws_fcg.get();
    double* Qd = Pd + (size_t)mt * n;
    std::vector<double> pqs(mt, 0.0);
    const dim3 g1(ceil_div(n, kBlock), 1);
    // x = 0, r = b on free rows
    dev_fill(c, n, 0.0, x);
    k_axpby_free<<<g1, kBlock, 0, s>>>(N, 1.0, b, n, 0.0, r, n);
    HINV_LAUNCH_CHECK();
    const double nb = std::sqrt(dev_dot(c, n, r, r));
    FcgStats st;
    if (nb == 0.0) {
        st.converged = true;
        *out = st;
        return;
    }
    const double npix = (double)n;  // rms over the whole image, as for the training crops
    std::vector<double> hist{nb};
    int it = 0;
    while (it < max_iter) {
        H.precondition(1, r, n, z, n);
        if (cnn) {
            H.apply(1, z, n, t, n);                                        // A z
            k_axpby_free<<<g1, kBlock, 0, s>>>(N, 1.0, r, n, -1.0, t, n);  // t = r - A z
            HINV_LAUNCH_CHECK();
            const double sc = std::sqrt(dev_dot(c, n, t, t) / npix);
            if (sc > 0.0) {
                short* in = cnn->packed_input(N + 1);
                k_fcg_input<<<ceil_div(n, kBlock), kBlock, 0, s>>>(N, t, 1.0 / sc, P.m_lin.get(), in);
                HINV_LAUNCH_CHECK();
                cnn->forward_packed(1, N + 1);
                k_fcg_correction<<<ceil_div(n, kBlock), kBlock, 0, s>>>(N, cnn->packed_output(), sc, cv);
                HINV_LAUNCH_CHECK();
                // energy-optimal step along the correction: the error left by the
                // V-cycle, e' = A^-1 t, is reduced in the A-norm by omega c with
                // omega = c^T t / c^T A c (never increased: omega = 0 at worst)
                H.apply(1, cv, n, Acv, n);
                const double ct = dev_dot(c, n, cv, t), cAc = dev_dot(c, n, cv, Acv);
                if (ct > 0.0 && cAc > 0.0) dev_axpby(c, n, ct / cAc, cv, 1.0, z);
            }
        }
        // p = z - sum_j (z . q_j) / (p_j . q_j) p_j over the kept directions
        double* p = Pd + (size_t)(it % mt) * n;
        double* q = Qd + (size_t)(it % mt) * n;
        const int kept = std::min(it, mt);
        std::vector<double> coef(kept);
        for (int j = 0; j < kept; ++j) {
            const int slot = (it - 1 - j) % mt;
            coef[j] = dev_dot(c, n, z, Qd + (size_t)slot * n) / pqs[slot];
        }
        dev_copy(c, n, 1, z, n, t, n);
        for (int j = 0; j < kept; ++j) dev_axpby(c, n, -coef[j], Pd + (size_t)((it - 1 - j) % mt) * n, 1.0, t);
        dev_copy(c, n, 1, t, n, p, n);  // the slot of p may be one of the kept directions
        H.apply(1, p, n, q, n);
        const double pq = dev_dot(c, n, p, q);
        if (!(pq > 0.0)) break;
        pqs[it % mt] = pq;
        const double alpha = dev_dot(c, n, p, r) / pq;
        dev_axpby(c, n, alpha, p, 1.0, x);
        dev_axpby(c, n, -alpha, q, 1.0, r);
        ++it;
        hist.push_back(std::sqrt(dev_dot(c, n, r, r)));
        if (hist.back() <= rtol * nb) {
            st.converged = true;
            break;
        }
        if (it >= 20 && hist.back() > 0.1 * hist[it - 20]) break;  // stalled
    }
    st.iterations = it;
    if (!st.converged) {
        // multigrid PCG on the remaining residual: A d = r, x += d
        SolveStats ps;
        double* d = P.scratch(3, 1);
        H.solve(1, r, n, d, n, HINV_PREC_FP64, rtol * nb / hist.back(), P.max_iter, &ps);
        dev_axpby(c, n, 1.0, d, 1.0, x);
        st.fallback = 1;
        st.fallback_iterations = ps.iterations;
        st.converged = ps.converged;
    }
    // final residual from scratch
    H.apply(1, x, n, t, n);
    k_axpby_free<<<g1, kBlock, 0, s>>>(N, 1.0, b, n, -1.0, t, n);
    HINV_LAUNCH_CHECK();
    st.relres = std::sqrt(dev_dot(c, n, t, t)) / nb;
    *out = st;
}

void cnn_harvest(Problem& P, int npairs, uint64_t seed, int crop, float* in, float* target, SolveStats* st) {
    P.ensure_lin_hierarchy();
    Ctx* c = P.ctx;
    hipStream_t s = c->stream;
    const int N = P.N, n = P.n, L = 6 * N * N;
    Hierarchy& H = *P.HA;
    constexpr int kRound = 64;
    DBuf<double> eta, rhs, xk, r, z, e;
    DBuf<int> org;
    eta.ensure((size_t)L * kRound);
    for (DBuf<double>* b : {&rhs, &xk, &r, &z, &e}) b->ensure((size_t)n * kRound);
    org.ensure(2 * kRound);
    std::vector<int> horg(2 * kRound);
    for (int base = 0, round = 0; base < npairs; base += kRound, ++round) {
        const int nc = std::min(kRound, npairs - base);
        const int k = round % 8;
        // random directions: the first n white-noise values of each sample
        P.white_noise(seed, 11, base, nc, eta.get(), L);
        P.inc_forward_rhs(nc, eta.get(), L, rhs.get(), n);
        const dim3 g(ceil_div(n, kBlock), nc);
        if (k > 0) {
            SolveStats tmp;
            H.solve(nc, rhs.get(), n, xk.get(), n, HINV_PREC_FP64, 1e-14, k, &tmp);
            H.apply(nc, xk.get(), n, r.get(), n);
            k_axpby_free<<<g, kBlock, 0, s>>>(N, 1.0, rhs.get(), n, -1.0, r.get(), n);  // r = b - A x_k
        } else {
            k_axpby_free<<<g, kBlock, 0, s>>>(N, 1.0, rhs.get(), n, 0.0, r.get(), n);   // r = b
        }
        HINV_LAUNCH_CHECK();
        H.precondition(nc, r.get(), n, z.get(), n);
        H.apply(nc, z.get(), n, xk.get(), n);
        k_axpby_free<<<g, kBlock, 0, s>>>(N, 1.0, r.get(), n, -1.0, xk.get(), n);  // r' = r - A V(r)
        HINV_LAUNCH_CHECK();
        H.solve(nc, xk.get(), n, e.get(), n, P.precision, P.rtol, P.max_iter, st);  // e' = A^-1 r'
        for (int j = 0; j < nc; ++j) {
            const uint64_t h = splitmix(seed ^ splitmix((uint64_t)(base + j) + 0x51ed27ull));
            horg[2 * j] = (int)(h % (uint64_t)(N + 2 - crop));
            horg[2 * j + 1] = (int)((h >> 32) % (uint64_t)(N + 2 - crop));
        }
        HINV_HIP(hipMemcpyAsync(org.get(), horg.data(), sizeof(int) * 2 * nc, hipMemcpyHostToDevice, s));
        const size_t np = (size_t)crop * crop;
        k_harvest_crop<<<nc, 256, 0, s>>>(N, crop, org.get(), xk.get(), e.get(), n, P.m_lin.get(), H.weightsE(),
                                          H.weightsN(), H.inv_diag(), in + (size_t)base * 3 * np,
                                          target + (size_t)base * 4 * np);
        HINV_LAUNCH_CHECK();
        HINV_HIP(hipStreamSynchronize(s));
    }
}

}  // namespace hinv
