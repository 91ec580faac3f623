// Many independent inversions of uneven mesh sizes advanced together.
//
// The instances are grouped by mesh size.  Each group owns a state hierarchy
// and a prior hierarchy that stack its instances (own coefficients, own prior
// parameters), so every solve of a Hessian action or of R^-1 runs once per
// group with the columns of all its instances in one multi-right-hand-side
// PCG.  The per-instance work around the solves (right-hand sides, outputs,
// the dense stages of the double pass) is launched instance by instance.
#pragma once

#include <vector>

#include "problem.h"

namespace hinv {

class Batch {
  public:
    Batch(Ctx* ctx, int nprob, Problem* const* probs);

    int size() const { return (int)P_.size(); }

    // out[i] (n_i x nrhs, ld n_i) = H_i mhat[i] for every instance i.
    void hessian(int mode, int nrhs, const double* const* mhat, double* const* out, SolveStats* st);

    // Double pass (Alg. 2 + Alg. 4) for every instance: omega[i] is n_i x s,
    // V[i] receives n_i x k (ld n_i), lambda_host[i k + j] the eigenvalues.
    int lowrank_eig(int mode, int tprod, int s, const double* const* omega, int k,
                    double* lambda_host, double* const* V, SolveStats* st);

  private:
    struct Group {
        int N = 0, n = 0;
        std::vector<int> mem;  // problem indices, in stacking order
        std::vector<long long> ver;  // linearization applied per member (-1: none)
        std::unique_ptr<Hierarchy> HA, HK;
        DBuf<double> a, b, c;  // stacked n x (members x cap) work blocks
        DBuf<double> blocks;   // the double pass's three stacked n x (members x s) blocks
        int cap = 0;
    };
    void sync(Group& g);
    void ensure(Group& g, int nrhs);
    // stacked Hessian action of group g: in/out column blocks of member j at
    // mh[j] / out[j] (ld n)
    void group_hessian(Group& g, int mode, int nrhs, const std::vector<const double*>& mh,
                       const std::vector<double*>& out, SolveStats* st);

    DBuf<double> small_;  // s x s matrices of the double pass, every member of a group
    DenseWork dw_;
    std::vector<Problem*> P_;
    std::vector<std::unique_ptr<Group>> G_;
    int precision_, max_iter_;
    double rtol_;
};

}  // namespace hinv
