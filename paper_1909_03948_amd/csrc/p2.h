// Quadratic (P2) state for the Poisson problem.  The paper's experiment
// (Sec. 5.1) pairs a P2 state with a P1 parameter; the coefficient
// c_T = exp(mean of m over the triangle) is the same per-triangle array as for
// the P1 state.
//
// Degrees of freedom are the vertices and edge midpoints, i.e. the nodes of
// the (2N+1) x (2N+1) grid of spacing h/2, numbered J (2N+1) + I; rows J = 0
// and J = 2N are the Dirichlet rows.  A triangle's six local dofs are ordered
// (a, r, b, mid(a,r), mid(r,b), mid(a,b)) with (a, r, b) as for P1.
//
// Solves: FP64 PCG preconditioned by a two-level cycle: degree-2
// Chebyshev-Jacobi smoothing on P2 around one V-cycle of the P1 hierarchy of
// the same coefficient, which is the exact Galerkin coarse operator
// (P^T A_2 P = A_1 for the embedding P of P1 functions into P2).
#pragma once

#include "solver.h"

namespace hinv {

// Unit-coefficient element stiffness of the lower (s = 0) and upper (s = 1)
// triangle of a cell, in local dof order.
struct P2Elem {
    double K[2][6][6];
};

class P2Space {
  public:
    P2Space(Ctx* ctx, int N);
    int N, side, ns;

    // per-triangle coefficient (owned by the P1 state hierarchy) and the
    // inverse diagonal of A_2 built from it
    void set_coefficient(const double* cT);
    const double* coefficient() const { return cT_; }

    // y = scale A_2 x on the free rows, 0 on the Dirichlet rows (x complete,
    // its Dirichlet values take part).  ldx = 0: one x for every column.
    void apply(int nc, const double* x, int ldx, double* y, int ldy, double scale);
    // y = scale K[s] w, s_T = (c_T / 3) sum_{v in T} mhat_v (w shared by the columns).
    void sens(int nc, const double* mhat, int ldm, const double* w, double scale, double* y, int ldy);
    // -A_FD u_D for u_D = 1 on the top row: the forward right-hand side
    void forward_rhs(double* rhs);
    void set_top(double* u);
    // A_FF x = b per column, to |b - A x| <= rtol |b| (b's Dirichlet rows ignored)
    void solve(int nc, const double* b, int ldb, double* x, int ldx, Hierarchy& coarse, double rtol,
               int max_iter, SolveStats* st);
    // g_v = sum_{T ni v} (c_T / 3) u_T^T K_T p_T (data part of the gradient)
    void grad(const double* u, const double* p, double* g);
    // Hessian output without the prior term (gn drops the terms with p);
    // add: added column by column when not null
    void hess_out(int nc, bool gn, const double* u, const double* p, const double* uh, int ldu,
                  const double* ph, int ldp, const double* mh, int ldm, double* out, int ldo,
                  const double* add, int ldadd);

    // observation operator: 6 (dof, weight) pairs per point, transpose in CSR
    void set_observations(int q, const double* xy_dev);
    void observe(int nc, const double* u, int ldu, const double* d, double* out, int ldo);
    void observe_adjoint(int nc, const double* v, int ldv, double scale, double* y, int ldy);

    const P2Elem& element() const { return el_; }
    double smoother_max() const { return lmax_; }

  private:
    Ctx* ctx_;
    P2Elem el_;
    double lmax_;  // upper bound of the spectrum of D^-1 A_2 (element-wise)
    const double* cT_ = nullptr;
    DBuf<double> dinv_;
    int q_ = 0, n_touch_ = 0;
    DBuf<int> obs_node_, t_node_, t_ptr_, t_ent_;
    DBuf<double> obs_w_;
    // solver workspaces (ns x cap columns each) and per-column scalars
    int cap_ = 0;
    DBuf<double> r_, z_, p_, q_v_, t1_, t2_, t3_, part_, scal_;
    DBuf<double> rc_, ec_;  // P1 restriction / coarse correction
    DBuf<int> act_;
    void ensure(int nc);
    void precondition(int nc, const double* r, int ldr, double* z, int ldz, Hierarchy& coarse);
    void dots(int nc, const double* a, int lda, const double* b, int ldb, double* out);
};

// The element matrices from the basis gradients at the edge midpoints (the
// three-point rule is exact for the quadratic integrand).
P2Elem p2_element();

}  // namespace hinv
