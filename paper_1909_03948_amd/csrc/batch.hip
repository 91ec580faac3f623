// Batches of independent inversions of uneven mesh sizes (see batch.h).
#include <algorithm>
#include <map>

#include "algos.h"
#include "batch.h"
#include "dense.h"

namespace hinv {

Batch::Batch(Ctx* ctx, int nprob, Problem* const* probs) {
    if (nprob <= 0) fail(HINV_EINVAL, "a batch needs at least one problem");
    std::map<int, std::vector<int>> by_N;
    precision_ = probs[0]->precision;
    rtol_ = probs[0]->rtol;
    max_iter_ = probs[0]->max_iter;
    for (int i = 0; i < nprob; ++i) {
        Problem* p = probs[i];
        if (!p) fail(HINV_EINVAL, "null problem in batch");
        if (p->ctx != ctx) fail(HINV_EINVAL, "every problem of a batch must use the batch's context");
        P_.push_back(p);
        by_N[p->N].push_back(i);
        rtol_ = std::min(rtol_, p->rtol);
        max_iter_ = std::max(max_iter_, p->max_iter);
    }
    // largest meshes first: their solves dominate, the small groups follow
    for (auto it = by_N.rbegin(); it != by_N.rend(); ++it) {
        auto g = std::make_unique<Group>();
        g->N = it->first;
        g->n = (g->N + 1) * (g->N + 1);
        g->mem = it->second;
        g->ver.assign(g->mem.size(), -1);
        const int ni = (int)g->mem.size();
        std::vector<PriorParams> pps(ni);
        for (int j = 0; j < ni; ++j) {
            const Problem* p = P_[g->mem[j]];
            pps[j] = p->prior;
        }
        g->HA = std::make_unique<Hierarchy>(ctx, kOpState, g->N, pps[0], ni);
        g->HK = std::make_unique<Hierarchy>(ctx, kOpPrior, g->N, pps[0], ni, pps.data());
        G_.push_back(std::move(g));
    }
}

// Brings the stacked state coefficients up to each member's linearization point.
void Batch::sync(Group& g) {
    for (size_t j = 0; j < g.mem.size(); ++j) {
        Problem* p = P_[g.mem[j]];
        if (!p->linearized) fail(HINV_ESTATE, "batched Hessian action before hinv_linearize of every problem");
        if (g.ver[j] != p->lin_version) {
            g.HA->set_state_coefficient(p->m_lin.get(), (int)j);
            g.ver[j] = p->lin_version;
        }
    }
}

void Batch::ensure(Group& g, int nrhs) {
    if (nrhs <= g.cap) return;
    const size_t len = (size_t)g.n * g.mem.size() * nrhs;
    g.a.ensure(len);
    g.b.ensure(len);
    g.c.ensure(len);
    g.cap = nrhs;
}

void Batch::group_hessian(Group& g, int mode, int nrhs, const std::vector<const double*>& mh,
                          const std::vector<double*>& out, SolveStats* st) {
    const bool gn = mode == HINV_HESS_GN_FULL || mode == HINV_HESS_GN_MISFIT;
    const int ni = (int)g.mem.size(), n = g.n, nc = ni * nrhs;
    sync(g);
    ensure(g, nrhs);
    auto blk = [&](const DBuf<double>& b, int j) { return b.get() + (size_t)j * nrhs * n; };
    // incremental forward: one solve for the columns of every member
    for (int j = 0; j < ni; ++j) P_[g.mem[j]]->inc_forward_rhs(nrhs, mh[j], n, blk(g.a, j), n);
    g.HA->solve(nc, g.a.get(), n, g.b.get(), n, precision_, chained_first_rtol(precision_, nc, rtol_), max_iter_,
                st, rtol_);
    // incremental adjoint
    for (int j = 0; j < ni; ++j)
        P_[g.mem[j]]->inc_adjoint_rhs(nrhs, gn, mh[j], n, blk(g.b, j), n, blk(g.a, j), n);
    g.HA->solve(nc, g.a.get(), n, g.c.get(), n, precision_, rtol_, max_iter_, st);
    for (int j = 0; j < ni; ++j)
        P_[g.mem[j]]->hess_output(mode, nrhs, mh[j], n, blk(g.b, j), n, blk(g.c, j), n, out[j], n);
}

void Batch::hessian(int mode, int nrhs, const double* const* mhat, double* const* out,
                    SolveStats* st) {
    if (nrhs <= 0) return;
    for (auto& gp : G_) {
        Group& g = *gp;
        std::vector<const double*> mh;
        std::vector<double*> o;
        for (int i : g.mem) {
            mh.push_back(mhat[i]);
            o.push_back(out[i]);
        }
        group_hessian(g, mode, nrhs, mh, o, st);
    }
}

int Batch::lowrank_eig(int mode, int tprod, int s, const double* const* omega, int k,
                       double* lambda_host, double* const* V, SolveStats* st) {
    size_t most = 0;  // members of the largest group
    for (auto& gp : G_) most = std::max(most, gp->mem.size());
    const size_t ss = (size_t)s * s;
    small_.ensure(most * (4 * ss + s));
    double* G = small_.get();
    double* Ri = G + most * ss;
    double* T = Ri + most * ss;
    double* S = T + most * ss;
    double* lam = S + most * ss;
    DenseWork& dw = dw_;
    int status = HINV_OK;
    for (auto& gp : G_) {
        Group& g = *gp;
        const int ni = (int)g.mem.size(), n = g.n, nc = ni * s;
        // three stacked blocks of s columns per member: W, Y, Zb; the Hessian
        // action uses g.a/g.b/g.c internally, so these live apart
        g.blocks.ensure((size_t)3 * n * nc);
        double* W = g.blocks.get();
        double* Y = W + (size_t)n * nc;
        double* Zb = Y + (size_t)n * nc;
        auto at = [&](double* base, int j) { return base + (size_t)j * s * n; };
        std::vector<const double*> om, wq;
        std::vector<double*> wout, zout;
        for (int j = 0; j < ni; ++j) {
            om.push_back(omega[g.mem[j]]);
            wout.push_back(at(W, j));
            wq.push_back(at(W, j));
            zout.push_back(at(Zb, j));
        }
        // pass 1: Ybar = A Omega, Y = R^-1 Ybar = K_A^-1 M K_A^-1 Ybar (M is the
        // same for every member of a mesh size: one launch over the block)
        group_hessian(g, mode, s, om, wout, st);
        g.HK->solve(nc, W, n, Y, n, precision_, rtol_, max_iter_, st);
        P_[g.mem[0]]->mass_apply(nc, Y, n, Zb, n);
        g.HK->solve(nc, Zb, n, Y, n, precision_, rtol_, max_iter_, st);
        // PreCholQR of every member: Q into W
        std::vector<Problem*> mp(ni);
        std::vector<double*> vout(ni), lout(ni);
        for (int j = 0; j < ni; ++j) {
            mp[j] = &*P_[g.mem[j]];
            vout[j] = V[g.mem[j]];
            lout[j] = lambda_host + (size_t)g.mem[j] * k;
        }
        status = precholqr(mp.data(), ni, dw, s, Y, Zb, W, G, Ri);
        if (status != HINV_OK) return status;
        // pass 2: A Q for every member, then the Rayleigh-Ritz step of every member
        group_hessian(g, mode, s, wq, zout, st);
        rayleigh_ritz(mp.data(), ni, dw, s, k, tprod, W, Zb, T, S, lam, vout.data(), n, lout.data());
    }
    return status;
}

}  // namespace hinv
