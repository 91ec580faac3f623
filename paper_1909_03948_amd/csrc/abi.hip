// extern "C" entry points of libhinv (declared and documented in include/hinv.h).
// Each entry validates its arguments, runs the operation on the context's
// stream and turns internal errors into status codes.
#include <algorithm>
#include <cmath>
#include <map>
#include <new>
#include <vector>

#include "algos.h"
#include "batch.h"
#include "cnn.h"
#include "fcg.h"
#include "noalloc.h"
#include "problem.h"

struct hinv_ctx {
    hinv::Ctx c;
};

struct hinv_problem {
    hinv_ctx* owner;
    std::unique_ptr<hinv::Problem> p;
};

struct hinv_cnn {
    hinv_ctx* owner;
    std::unique_ptr<hinv::Cnn> net;
};

struct hinv_batch {
    hinv_ctx* owner;
    std::vector<hinv_problem*> probs;
    std::unique_ptr<hinv::Batch> b;
    int max_group = 0;  // members of the largest mesh-size group
};

namespace {

thread_local std::string g_noctx_err;

template <class F>
int guarded(hinv::Ctx* c, F f) {
    hinv::CtxScope scope(c);  // buffers made by this call use c's allocator
    try {
        f();
        return HINV_OK;
    } catch (const hinv::Error& e) {
        if (c) c->err = e.msg;
        else g_noctx_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        return HINV_ENOMEM;
    } catch (const std::exception& e) {
        if (c) c->err = e.what();
        return HINV_EHIP;
    }
}

void fill_info(hinv_solve_info* info, const hinv::SolveStats& s) {
    if (!info) return;
    info->status = s.converged ? HINV_OK : HINV_ENOCONV;
    info->solves = s.solves;
    info->iterations = s.iterations;
    info->refinements = s.refinements;
    info->fallbacks = s.fallbacks;
    info->max_relres = s.max_relres;
}

int conv_status(const hinv::SolveStats& s) { return s.converged ? HINV_OK : HINV_ENOCONV; }

#define REQUIRE(cond, msg) \
    do {                   \
        if (!(cond)) hinv::fail(HINV_EINVAL, msg); \
    } while (0)

hinv::Ctx* ctx_of(hinv_problem* p) { return p ? &p->owner->c : nullptr; }

void set_device(hinv::Ctx* c) { HINV_HIP(hipSetDevice(c->device)); }

}  // namespace

extern "C" {

const char* hinv_status_string(int s) {
    switch (s) {
        case HINV_OK: return "ok";
        case HINV_EINVAL: return "invalid argument";
        case HINV_ENOMEM: return "out of device memory";
        case HINV_EHIP: return "HIP runtime error";
        case HINV_ENOCONV: return "iterative solve did not reach its tolerance";
        case HINV_ESTATE: return "call out of order";
        case HINV_ENEGEIG: return "eigenvalue <= -1 passed to the posterior sampler";
        case HINV_EBREAK: return "Cholesky breakdown in PreCholQR";
        default: return "unknown status";
    }
}

int hinv_ctx_create(int device, void* stream, const hinv_allocator* alloc, hinv_ctx** out) {
    if (!out) return HINV_EINVAL;
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->free)) {
        g_noctx_err = "allocator needs both callbacks";
        return HINV_EINVAL;
    }
    hinv_ctx* c = new (std::nothrow) hinv_ctx;
    if (!c) return HINV_ENOMEM;
    const int rc = guarded(nullptr, [&] {
        int ndev = 0;
        HINV_HIP(hipGetDeviceCount(&ndev));
        REQUIRE(device >= 0 && device < ndev, "no such HIP device");
        c->c.device = device;
        c->c.stream = (hipStream_t)stream;
        if (alloc) {
            c->c.alloc = *alloc;
            c->c.has_alloc = true;
        }
        HINV_HIP(hipSetDevice(device));
        // device address of the fixed scratch of hinv_prior_apply_noalloc
        hinv::noalloc_init(device);
    });
    if (rc != HINV_OK) {
        delete c;
        return rc;
    }
    *out = c;
    return HINV_OK;
}

int hinv_ctx_destroy(hinv_ctx* c) {
    if (!c) return HINV_EINVAL;
    delete c;
    return HINV_OK;
}

int hinv_ctx_set_stream(hinv_ctx* c, void* stream) {
    if (!c) return HINV_EINVAL;
    return guarded(&c->c, [&] {
        // buffers in use by work on the old stream are freed on the new one later
        HINV_HIP(hipStreamSynchronize(c->c.stream));
        c->c.stream = (hipStream_t)stream;
    });
}

const char* hinv_last_error(const hinv_ctx* c) {
    if (!c) return g_noctx_err.c_str();
    return c->c.err.c_str();
}

int hinv_tuner_counts(long long* timed, long long* cached) {
    if (!timed || !cached) return HINV_EINVAL;
    long t = 0, c = 0;
    hinv::tuner_counts(&t, &c);
    *timed = t;
    *cached = c;
    return HINV_OK;
}

int hinv_ctx_kernel_timer(hinv_ctx* c, int kclass, int enable, int period) {
    if (!c) return HINV_EINVAL;
    return guarded(&c->c, [&] {
        REQUIRE(kclass >= 0 && kclass < hinv::KernelTimer::kClasses, "bad kernel class");
        REQUIRE(period >= 1, "period must be >= 1");
        auto& k = c->c.timer.cls[kclass];
        if (enable && k.ev.empty()) {
            k.ev.resize(2 * hinv::KernelTimer::kPool);
            for (auto& e : k.ev) HINV_HIP(hipEventCreate(&e));
            k.work.resize(hinv::KernelTimer::kPool);
        }
        k.on = enable != 0;
        k.period = period;
        if (enable) {
            k.used = 0;
            k.launches = 0;
        }
    });
}

int hinv_ctx_kernel_timer_read(hinv_ctx* c, int kclass, int* timed, long* launches_total,
                               double* total_ms, double* total_work) {
    if (!c || !timed || !launches_total || !total_ms || !total_work) return HINV_EINVAL;
    return guarded(&c->c, [&] {
        REQUIRE(kclass >= 0 && kclass < hinv::KernelTimer::kClasses, "bad kernel class");
        auto& k = c->c.timer.cls[kclass];
        HINV_HIP(hipStreamSynchronize(c->c.stream));
        double ms = 0.0, work = 0.0;
        int cnt = 0;
        for (int i = 0; i < k.used; ++i) {
            if (k.work[i] < 0) continue;  // launch of another level: not counted
            float t = 0.f;
            HINV_HIP(hipEventElapsedTime(&t, k.ev[2 * i], k.ev[2 * i + 1]));
            ms += t;
            work += k.work[i];
            ++cnt;
        }
        *timed = cnt;
        *launches_total = k.launches;
        *total_ms = ms;
        *total_work = work;
    });
}

int hinv_problem_create(hinv_ctx* c, const hinv_problem_desc* d, hinv_problem** out) {
    if (!c || !d || !out) return HINV_EINVAL;
    *out = nullptr;
    return guarded(&c->c, [&] {
        REQUIRE(d->N >= 4 && d->N <= 8192 && (d->N & (d->N - 1)) == 0,
                "N must be a power of two in [4, 8192]");
        REQUIRE(d->gamma > 0 && d->delta > 0, "gamma and delta must be positive");
        REQUIRE(std::isnan(d->beta) || d->beta >= 0, "beta must be >= 0 or NaN");
        if (d->theta1 > 0.0) {
            REQUIRE(d->theta2 > 0.0 && std::isfinite(d->theta1) && std::isfinite(d->theta2) &&
                        std::isfinite(d->alpha),
                    "Theta needs theta1, theta2 > 0 and a finite alpha");
            // the smoother's spectral bound needs K_Theta's couplings <= 0:
            // 0 <= t12 <= min(t11, t22) (the mesh diagonal along Theta's
            // principal direction)
            const double sa = std::sin(d->alpha), ca = std::cos(d->alpha);
            const double t11 = d->theta1 * sa * sa + d->theta2 * ca * ca;
            const double t12 = (d->theta1 - d->theta2) * sa * ca;
            const double t22 = d->theta1 * ca * ca + d->theta2 * sa * sa;
            const double eps = 1e-12 * (t11 + t22);
            REQUIRE(t12 >= -eps && t12 <= std::min(t11, t22) + eps,
                    "Theta must satisfy 0 <= Theta_12 <= min(Theta_11, Theta_22) on this mesh");
        }
        REQUIRE(d->state_degree >= 0 && d->state_degree <= 2, "state_degree must be 0, 1 or 2");
        REQUIRE(d->q >= 0, "q must be >= 0");
        REQUIRE(d->q == 0 || d->obs_xy, "obs_xy is required when q > 0");
        REQUIRE(d->sigma > 0, "sigma must be positive");
        REQUIRE(d->precision >= HINV_PREC_FP64 && d->precision <= HINV_PREC_AUTO, "bad precision");
        REQUIRE(d->rtol > 0 && d->rtol < 1, "rtol must be in (0, 1)");
        for (int o = 0; o < d->q; ++o) {
            const double x = d->obs_xy[2 * o], y = d->obs_xy[2 * o + 1];
            REQUIRE(x >= 0 && x <= 1 && y >= 0 && y <= 1, "observation point outside [0,1]^2");
        }
        set_device(&c->c);
        auto hp = std::make_unique<hinv_problem>();
        hp->owner = c;
        hp->p = std::make_unique<hinv::Problem>(&c->c, *d);
        *out = hp.release();
    });
}

int hinv_problem_destroy(hinv_problem* p) {
    if (!p) return HINV_EINVAL;
    delete p;
    return HINV_OK;
}

int hinv_problem_size(const hinv_problem* p, int* n) {
    if (!p || !n) return HINV_EINVAL;
    *n = p->p->n;
    return HINV_OK;
}

int hinv_problem_state_size(const hinv_problem* p, int* ns) {
    if (!p || !ns) return HINV_EINVAL;
    *ns = p->p->ns;
    return HINV_OK;
}

int hinv_set_data(hinv_problem* p, const double* d_obs, double sigma) {
    if (!p) return HINV_EINVAL;
    return guarded(ctx_of(p), [&] {
        REQUIRE(sigma > 0 || std::isnan(sigma), "sigma must be positive (or NaN to keep it)");
        p->p->set_data(d_obs, std::isnan(sigma) ? -1.0 : sigma);
    });
}

int hinv_set_solver(hinv_problem* p, int precision, double rtol, int max_iter) {
    if (!p) return HINV_EINVAL;
    return guarded(ctx_of(p), [&] {
        REQUIRE(precision >= HINV_PREC_FP64 && precision <= HINV_PREC_AUTO, "bad precision");
        REQUIRE(rtol > 0 && rtol < 1, "rtol must be in (0, 1)");
        p->p->precision = precision;
        p->p->rtol = rtol;
        p->p->max_iter = max_iter > 0 ? max_iter : 200;
    });
}

int hinv_forward(hinv_problem* p, const double* m, double* u, hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        REQUIRE(m && u, "null vector");
        p->p->forward(m, u, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

int hinv_cost(hinv_problem* p, const double* m, const double* u, double* misfit, double* reg) {
    if (!p) return HINV_EINVAL;
    return guarded(ctx_of(p), [&] {
        REQUIRE(m && u && misfit && reg, "null argument");
        p->p->cost(m, u, misfit, reg);
    });
}

int hinv_observe(hinv_problem* p, const double* u, double* Bu) {
    if (!p) return HINV_EINVAL;
    return guarded(ctx_of(p), [&] {
        REQUIRE(u && (Bu || p->p->q == 0), "null argument");
        p->p->observe(u, p->p->ns, 1, Bu, p->p->q, false);
    });
}

int hinv_gradient(hinv_problem* p, const double* m, const double* u, double* adj, double* g,
                  hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        REQUIRE(m && u && adj && g, "null vector");
        p->p->gradient(m, u, adj, g, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

int hinv_linearize(hinv_problem* p, const double* m, const double* u, const double* adj) {
    if (!p) return HINV_EINVAL;
    return guarded(ctx_of(p), [&] {
        REQUIRE(m && u && adj, "null vector");
        p->p->linearize(m, u, adj);
    });
}

int hinv_inc_forward(hinv_problem* p, int nrhs, const double* mhat, int ldm, double* uhat, int ldu,
                     hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        const int n = p->p->n, ns = p->p->ns;
        REQUIRE(nrhs >= 0 && ldm >= n && ldu >= ns, "bad size or leading dimension");
        REQUIRE(nrhs == 0 || (mhat && uhat), "null vector");
        if (nrhs) p->p->inc_forward(nrhs, mhat, ldm, uhat, ldu, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

int hinv_inc_adjoint(hinv_problem* p, int nrhs, int gauss_newton, const double* mhat, int ldm,
                     const double* uhat, int ldu, double* phat, int ldp, hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        const int n = p->p->n, ns = p->p->ns;
        REQUIRE(nrhs >= 0 && ldm >= n && ldu >= ns && ldp >= ns, "bad size or leading dimension");
        REQUIRE(nrhs == 0 || (mhat && uhat && phat), "null vector");
        if (nrhs) p->p->inc_adjoint(nrhs, gauss_newton != 0, mhat, ldm, uhat, ldu, phat, ldp, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

int hinv_hessian_apply(hinv_problem* p, int mode, int nrhs, const double* mhat, int ldm,
                       double* out, int ldo, hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        const int n = p->p->n;
        REQUIRE(mode >= HINV_HESS_FULL && mode <= HINV_HESS_GN_MISFIT, "bad Hessian mode");
        REQUIRE(nrhs >= 0 && ldm >= n && ldo >= n, "bad size or leading dimension");
        REQUIRE(nrhs == 0 || (mhat && out), "null vector");
        if (nrhs) p->p->hessian(mode, nrhs, mhat, ldm, out, ldo, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

int hinv_prior_apply(hinv_problem* p, int nrhs, const double* x, int ldx, double* y, int ldy) {
    if (!p) return HINV_EINVAL;
    return guarded(ctx_of(p), [&] {
        const int n = p->p->n;
        REQUIRE(nrhs >= 0 && ldx >= n && ldy >= n, "bad size or leading dimension");
        REQUIRE(nrhs == 0 || (x && y), "null vector");
        if (nrhs) p->p->prior_apply(nrhs, x, ldx, y, ldy);
    });
}

int hinv_prior_apply_noalloc(hinv_problem* p, int nrhs, const double* x, int ldx, double* y, int ldy) {
    if (!p) return HINV_EINVAL;
    return guarded(ctx_of(p), [&] {
        const int n = p->p->n;
        REQUIRE(nrhs >= 0 && ldx >= n && ldy >= n, "bad size or leading dimension");
        REQUIRE(nrhs == 0 || (x && y), "null vector");
        const size_t need = (size_t)6 * n * nrhs;
        if (need > hinv::kNoAllocScratchDoubles)
            hinv::fail(HINV_EINVAL, "hinv_prior_apply_noalloc: 6 n nrhs = " + std::to_string(need) +
                                        " doubles exceed the fixed scratch of " +
                                        std::to_string(hinv::kNoAllocScratchDoubles));
        if (nrhs)
            p->p->prior_apply(nrhs, x, ldx, y, ldy, false, nullptr,
                              hinv::noalloc_scratch(ctx_of(p)->device));
    });
}

int hinv_prior_solve(hinv_problem* p, int nrhs, const double* x, int ldx, double* y, int ldy,
                     hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        const int n = p->p->n;
        REQUIRE(nrhs >= 0 && ldx >= n && ldy >= n, "bad size or leading dimension");
        REQUIRE(nrhs == 0 || (x && y), "null vector");
        if (nrhs) p->p->prior_solve(nrhs, x, ldx, y, ldy, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

int hinv_prior_sample(hinv_problem* p, int ns, const double* eta, int ldeta, double* out, int ldo,
                      hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        const int n = p->p->n, N = p->p->N;
        REQUIRE(ns >= 0 && ldeta >= 6 * N * N && ldo >= n, "bad size or leading dimension");
        REQUIRE(ns == 0 || (eta && out), "null vector");
        if (ns) p->p->prior_sample(ns, eta, ldeta, out, ldo, true, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

int hinv_white_noise(hinv_problem* p, uint64_t seed, uint64_t stream, int64_t first, int ns,
                     double* eta, int ld) {
    if (!p) return HINV_EINVAL;
    return guarded(ctx_of(p), [&] {
        const int N = p->p->N;
        REQUIRE(ns >= 0 && first >= 0 && ld >= 6 * N * N, "bad size or leading dimension");
        REQUIRE(ns == 0 || eta, "null output");
        if (ns) p->p->white_noise(seed, stream, first, ns, eta, ld);
    });
}

int hinv_map_newton(hinv_problem* p, const double* m0, double* m_map, const hinv_newton_opts* opts,
                    hinv_newton_info* info) {
    if (!p) return HINV_EINVAL;
    int status = HINV_OK;
    int rc = guarded(ctx_of(p), [&] {
        REQUIRE(m_map, "null output");
        hinv_newton_opts o;
        o.rel_tol = 1e-6;
        o.abs_tol = 0.0;
        o.max_iter = 50;
        o.max_backtrack = 10;
        o.c_armijo = 1e-4;
        o.max_cg = 500;
        o.gn_iters = 5;
        if (opts) o = *opts;
        REQUIRE(o.max_iter >= 0 && o.max_iter <= HINV_NEWTON_MAXREC, "max_iter out of range");
        REQUIRE(o.max_backtrack >= 0 && o.max_cg >= 1 && o.gn_iters >= 0, "bad Newton options");
        hinv_newton_info tmp;
        status = hinv::map_newton(*p->p, m0, m_map, o, info ? info : &tmp);
    });
    return rc != HINV_OK ? rc : status;
}

int hinv_lowrank_eig(hinv_problem* p, int mode, int tprod, int s, const double* omega, int ldo,
                     int k, double* lambda_host, double* V, int ldv, hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int status = HINV_OK;
    int rc = guarded(ctx_of(p), [&] {
        const int n = p->p->n;
        REQUIRE(mode == HINV_HESS_MISFIT || mode == HINV_HESS_GN_MISFIT, "mode must be a misfit mode");
        REQUIRE(tprod == HINV_TPROD_FP64 || tprod == HINV_TPROD_BF16, "bad block-product precision");
        REQUIRE(s >= 1 && s <= 512 && s <= n, "probe count s must be in [1, min(512, n)]");
        REQUIRE(k >= 1 && k <= s, "k must be in [1, s]");
        REQUIRE(ldo >= n && ldv >= n, "bad leading dimension");
        REQUIRE(omega && lambda_host && V, "null argument");
        status = hinv::lowrank_eig(*p->p, mode, tprod, s, omega, ldo, k, lambda_host, V, ldv, &st);
    });
    fill_info(info, st);
    if (rc != HINV_OK) return rc;
    if (status != HINV_OK) return status;
    return conv_status(st);
}

int hinv_lowrank_eig_single(hinv_problem* p, int mode, int s, const double* omega, int ldo, int k,
                            double* lambda_host, double* V, int ldv, hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int status = HINV_OK;
    int rc = guarded(ctx_of(p), [&] {
        const int n = p->p->n;
        REQUIRE(mode == HINV_HESS_MISFIT || mode == HINV_HESS_GN_MISFIT, "mode must be a misfit mode");
        REQUIRE(s >= 1 && s <= 512 && s <= n, "probe count s must be in [1, min(512, n)]");
        REQUIRE(k >= 1 && k <= s, "k must be in [1, s]");
        REQUIRE(ldo >= n && ldv >= n, "bad leading dimension");
        REQUIRE(omega && lambda_host && V, "null argument");
        status = hinv::lowrank_eig_single(*p->p, mode, s, omega, ldo, k, lambda_host, V, ldv, &st);
    });
    fill_info(info, st);
    if (rc != HINV_OK) return rc;
    if (status != HINV_OK) return status;
    return conv_status(st);
}

int hinv_prior_variance(hinv_problem* p, int s, const double* omega, int ldo, double* diag, double* mu_host,
                        hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int status = HINV_OK;
    int rc = guarded(ctx_of(p), [&] {
        const int n = p->p->n;
        REQUIRE(s >= 1 && s <= 512 && s <= n, "probe count s must be in [1, min(512, n)]");
        REQUIRE(ldo >= n, "bad leading dimension");
        REQUIRE(omega && diag, "null argument");
        status = hinv::prior_variance(*p->p, s, omega, ldo, diag, mu_host, &st);
    });
    fill_info(info, st);
    if (rc != HINV_OK) return rc;
    if (status != HINV_OK) return status;
    return conv_status(st);
}

int hinv_posterior_variance(hinv_problem* p, const double* prior_diag, int k, const double* lambda_host,
                            const double* V, int ldv, double* diag) {
    if (!p) return HINV_EINVAL;
    return guarded(ctx_of(p), [&] {
        const int n = p->p->n;
        REQUIRE(k >= 0 && (k == 0 || ldv >= n), "bad size or leading dimension");
        REQUIRE(prior_diag && diag && (k == 0 || (lambda_host && V)), "null argument");
        for (int i = 0; i < k; ++i)
            if (!(lambda_host[i] > -1.0)) hinv::fail(HINV_ENEGEIG, "eigenvalue <= -1");
        hinv::posterior_variance(*p->p, prior_diag, k, lambda_host, V, ldv, diag);
    });
}

int hinv_posterior_sample(hinv_problem* p, const double* m_map, int k, const double* lambda_host,
                          const double* V, int ldv, int ns, const double* eta, int ldeta,
                          double* out, int ldo, hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        const int n = p->p->n, N = p->p->N;
        REQUIRE(k >= 0 && ns >= 0 && ldv >= n && ldo >= n && ldeta >= 6 * N * N, "bad size");
        REQUIRE(m_map && (k == 0 || (lambda_host && V)) && (ns == 0 || (eta && out)), "null argument");
        for (int i = 0; i < k; ++i)
            if (!(lambda_host[i] > -1.0)) hinv::fail(HINV_ENEGEIG, "eigenvalue <= -1");
        if (ns) hinv::posterior_sample(*p->p, m_map, k, lambda_host, V, ldv, ns, eta, ldeta, out, ldo, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

int hinv_posterior_sample_seeded(hinv_problem* p, const double* m_map, int k, const double* lambda_host,
                                 const double* V, int ldv, uint64_t seed, uint64_t stream, int64_t first, int ns,
                                 double* out, int ldo, hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        const int n = p->p->n;
        REQUIRE(k >= 0 && ns >= 0 && first >= 0 && ldv >= n && ldo >= n, "bad size");
        REQUIRE(m_map && (k == 0 || (lambda_host && V)) && (ns == 0 || out), "null argument");
        for (int i = 0; i < k; ++i)
            if (!(lambda_host[i] > -1.0)) hinv::fail(HINV_ENEGEIG, "eigenvalue <= -1");
        if (ns)
            hinv::posterior_sample_seeded(*p->p, m_map, k, lambda_host, V, ldv, seed, stream, first, ns, out, ldo,
                                          &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

// ------------------------------------------------------------- batches ---
int hinv_batch_create(hinv_ctx* c, int nprob, hinv_problem* const* probs, hinv_batch** out) {
    if (!c || !out) return HINV_EINVAL;
    *out = nullptr;
    return guarded(&c->c, [&] {
        REQUIRE(nprob >= 1 && nprob <= 4096, "nprob must be in [1, 4096]");
        REQUIRE(probs, "null problem list");
        std::vector<hinv::Problem*> ps;
        std::map<int, int> count;
        for (int i = 0; i < nprob; ++i) {
            REQUIRE(probs[i] && probs[i]->owner == c, "every problem must belong to this context");
            for (int j = 0; j < i; ++j) REQUIRE(probs[j] != probs[i], "a problem appears twice");
            REQUIRE(probs[i]->p->deg == 1, "batches take P1-state problems only");
            ps.push_back(probs[i]->p.get());
            ++count[probs[i]->p->N];
        }
        set_device(&c->c);
        auto hb = std::make_unique<hinv_batch>();
        hb->owner = c;
        hb->probs.assign(probs, probs + nprob);
        for (auto& kv : count) hb->max_group = std::max(hb->max_group, kv.second);
        hb->b = std::make_unique<hinv::Batch>(&c->c, nprob, ps.data());
        *out = hb.release();
    });
}

int hinv_batch_destroy(hinv_batch* b) {
    if (!b) return HINV_EINVAL;
    delete b;
    return HINV_OK;
}

int hinv_batch_hessian_apply(hinv_batch* b, int mode, int nrhs, const double* const* mhat,
                             double* const* out, hinv_solve_info* info) {
    if (!b) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(&b->owner->c, [&] {
        REQUIRE(mode >= HINV_HESS_FULL && mode <= HINV_HESS_GN_MISFIT, "bad Hessian mode");
        REQUIRE(nrhs >= 0, "nrhs must be >= 0");
        REQUIRE((long long)nrhs * b->max_group <= 4096,
                "nrhs times the largest mesh-size group must not exceed 4096 columns");
        if (nrhs == 0) return;
        REQUIRE(mhat && out, "null pointer list");
        for (size_t i = 0; i < b->probs.size(); ++i) REQUIRE(mhat[i] && out[i], "null vector");
        b->b->hessian(mode, nrhs, mhat, out, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

int hinv_batch_lowrank_eig(hinv_batch* b, int mode, int tprod, int s, const double* const* omega,
                           int k, double* lambda_host, double* const* V, hinv_solve_info* info) {
    if (!b) return HINV_EINVAL;
    hinv::SolveStats st;
    int status = HINV_OK;
    int rc = guarded(&b->owner->c, [&] {
        REQUIRE(mode == HINV_HESS_MISFIT || mode == HINV_HESS_GN_MISFIT, "mode must be a misfit mode");
        REQUIRE(tprod == HINV_TPROD_FP64 || tprod == HINV_TPROD_BF16, "bad block-product precision");
        int nmin = 1 << 30;
        for (auto* p : b->probs) nmin = std::min(nmin, p->p->n);
        REQUIRE(s >= 1 && s <= 512 && s <= nmin, "probe count s must be in [1, min(512, n_i)]");
        REQUIRE((long long)s * b->max_group <= 4096,
                "s times the largest mesh-size group must not exceed 4096 columns");
        REQUIRE(k >= 1 && k <= s, "k must be in [1, s]");
        REQUIRE(omega && lambda_host && V, "null argument");
        for (size_t i = 0; i < b->probs.size(); ++i) REQUIRE(omega[i] && V[i], "null vector");
        status = b->b->lowrank_eig(mode, tprod, s, omega, k, lambda_host, V, &st);
    });
    fill_info(info, st);
    if (rc != HINV_OK) return rc;
    if (status != HINV_OK) return status;
    return conv_status(st);
}

// ------------------------------------------------- state-operator solves ---
int hinv_state_apply(hinv_problem* p, int nrhs, const double* x, int ldx, double* y, int ldy) {
    if (!p) return HINV_EINVAL;
    return guarded(ctx_of(p), [&] {
        const int ns = p->p->ns;
        REQUIRE(nrhs >= 0 && ldx >= ns && ldy >= ns, "bad size or leading dimension");
        REQUIRE(nrhs == 0 || (x && y), "null vector");
        REQUIRE(p->p->linearized, "state operator used before hinv_linearize");
        if (!nrhs) return;
        p->p->ensure_lin_hierarchy();
        p->p->state_apply(nrhs, x, ldx, y, ldy);
    });
}

int hinv_state_solve(hinv_problem* p, int nrhs, const double* b, int ldb, double* x, int ldx,
                     hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        const int ns = p->p->ns;
        REQUIRE(nrhs >= 0 && ldb >= ns && ldx >= ns, "bad size or leading dimension");
        REQUIRE(nrhs == 0 || (b && x), "null vector");
        REQUIRE(p->p->linearized, "state operator used before hinv_linearize");
        if (!nrhs) return;
        hinv::Problem& P = *p->p;
        P.ensure_lin_hierarchy();
        P.state_solve(nrhs, b, ldb, x, ldx, P.rtol, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

int hinv_state_solve_fcg(hinv_problem* p, hinv_cnn* net, const double* b, double* x, double rtol,
                         int max_iter, int truncation, hinv_fcg_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::FcgStats st;
    int rc = guarded(ctx_of(p), [&] {
        REQUIRE(b && x, "null vector");
        REQUIRE(rtol > 0 && rtol < 1, "rtol must be in (0, 1)");
        REQUIRE(max_iter >= 1, "max_iter must be >= 1");
        REQUIRE(truncation >= 1 && truncation <= 32, "truncation must be in [1, 32]");
        REQUIRE(!net || net->owner == p->owner, "network and problem must share the context");
        REQUIRE(p->p->linearized, "state operator used before hinv_linearize");
        REQUIRE(p->p->deg == 1, "flexible CG takes P1-state problems only");
        hinv::state_solve_fcg(*p->p, net ? net->net.get() : nullptr, b, x, rtol, max_iter, truncation, &st);
    });
    if (info) {
        info->status = st.converged ? HINV_OK : HINV_ENOCONV;
        info->iterations = st.iterations;
        info->fallback = st.fallback;
        info->fallback_iterations = st.fallback_iterations;
        info->relres = st.relres;
    }
    if (rc != HINV_OK) return rc;
    return st.converged ? HINV_OK : HINV_ENOCONV;
}

// ------------------------------------------------------------- network ---
int hinv_cnn_create(hinv_ctx* c, hinv_cnn** out) {
    if (!c || !out) return HINV_EINVAL;
    *out = nullptr;
    return guarded(&c->c, [&] {
        set_device(&c->c);
        auto h = std::make_unique<hinv_cnn>();
        h->owner = c;
        h->net = std::make_unique<hinv::Cnn>(&c->c);
        *out = h.release();
    });
}

int hinv_cnn_destroy(hinv_cnn* net) {
    if (!net) return HINV_EINVAL;
    delete net;
    return HINV_OK;
}

int hinv_cnn_param_count(void) { return hinv::Cnn::nparams(); }

int hinv_cnn_set_params(hinv_cnn* net, const float* host, int count) {
    if (!net) return HINV_EINVAL;
    return guarded(&net->owner->c, [&] {
        REQUIRE(host && count == hinv::Cnn::nparams(), "parameter count mismatch");
        net->net->set_params(host);
    });
}

int hinv_cnn_get_params(hinv_cnn* net, float* host, int count) {
    if (!net) return HINV_EINVAL;
    return guarded(&net->owner->c, [&] {
        REQUIRE(host && count == hinv::Cnn::nparams(), "parameter count mismatch");
        net->net->get_params(host);
    });
}

int hinv_cnn_forward(hinv_cnn* net, int B, int S, const float* in, float* out) {
    if (!net) return HINV_EINVAL;
    return guarded(&net->owner->c, [&] {
        REQUIRE(B >= 1 && S >= 1 && S <= 8193 && (long long)B * S * S <= (1LL << 28), "bad image batch size");
        REQUIRE(in && out, "null image");
        net->net->forward(B, S, in, out);
    });
}

int hinv_cnn_gradient(hinv_cnn* net, int B, int S, const float* in, const float* target, int tchan,
                      double* loss, float* grad_host) {
    if (!net) return HINV_EINVAL;
    return guarded(&net->owner->c, [&] {
        REQUIRE(B >= 1 && S >= 1 && S <= 8193 && (long long)B * S * S <= (1LL << 26), "bad image batch size");
        REQUIRE(tchan == 1 || tchan == 4, "target channels must be 1 or 4");
        REQUIRE(in && target && loss, "null argument");
        *loss = net->net->gradient(B, S, in, target, tchan, grad_host);
    });
}

int hinv_cnn_train_step(hinv_cnn* net, int B, int S, const float* in, const float* target, int tchan,
                        float lr, double* loss) {
    if (!net) return HINV_EINVAL;
    return guarded(&net->owner->c, [&] {
        REQUIRE(B >= 1 && S >= 1 && S <= 8193 && (long long)B * S * S <= (1LL << 26), "bad image batch size");
        REQUIRE(tchan == 1 || tchan == 4, "target channels must be 1 or 4");
        REQUIRE(in && target && loss, "null argument");
        REQUIRE(lr > 0 && std::isfinite(lr), "learning rate must be positive");
        *loss = net->net->train_step(B, S, in, target, tchan, lr);
    });
}

int hinv_cnn_harvest(hinv_problem* p, int npairs, uint64_t seed, int crop, float* in, float* target,
                     hinv_solve_info* info) {
    if (!p) return HINV_EINVAL;
    hinv::SolveStats st;
    int rc = guarded(ctx_of(p), [&] {
        REQUIRE(npairs >= 0, "npairs must be >= 0");
        REQUIRE(crop >= 3 && crop <= p->p->N + 1, "crop must be in [3, N + 1]");
        REQUIRE(npairs == 0 || (in && target), "null output");
        REQUIRE(p->p->linearized, "harvest before hinv_linearize");
        REQUIRE(p->p->deg == 1, "the pair harvest takes P1-state problems only");
        if (npairs) hinv::cnn_harvest(*p->p, npairs, seed, crop, in, target, &st);
    });
    fill_info(info, st);
    return rc != HINV_OK ? rc : conv_status(st);
}

}  // extern "C"
