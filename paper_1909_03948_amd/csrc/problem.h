// The inverse-problem object behind hinv_problem: mesh-sized device data, the
// two multigrid hierarchies (state operator A(m), prior operator K_A) and the
// operations of the method.
#pragma once

#include <memory>

#include "p2.h"
#include "solver.h"

namespace hinv {

class Problem {
  public:
    Problem(Ctx* ctx, const hinv_problem_desc& d);
    ~Problem();
    Problem(const Problem&) = delete;
    Problem& operator=(const Problem&) = delete;

    Ctx* ctx;
    int N, n, q;
    double gamma, delta, beta, m_prior, sigma;
    PriorParams prior;  // gamma, delta, beta and the tensor Theta of K_A
    int precision;
    double rtol;
    int max_iter;

    std::unique_ptr<Hierarchy> HA;  // state operator A(m) (the P1 state, or the coarse space of P2)
    std::unique_ptr<Hierarchy> HK;  // prior operator K_A
    int deg = 1;                    // state degree (1: P1, 2: P2 on the (2N+1)^2 nodes)
    int ns = 0;                     // entries of a state vector
    std::unique_ptr<P2Space> S2;    // the P2 state space (deg == 2)

    // observation operator: 3 (node, weight) pairs per point; transpose in CSR
    DBuf<double> obs_xy, obs_w, d;
    DBuf<int> obs_node, t_node, t_ptr, t_ent;
    int n_touch = 0;

    // linearization point
    DBuf<double> m_lin, u_lin, p_lin;
    bool linearized = false;
    bool ha_is_lin = false;
    long long lin_version = 0;  // counts linearizations (batches track it)

    void set_data(const double* d_host, double sig);

    // --- operations (device pointers, FP64) ---
    void forward(const double* m, double* u, SolveStats* st);
    void observe(const double* u, int ldu, int nc, double* out, int ldo, bool minus_data);
    void cost(const double* m, const double* u, double* misfit, double* reg);
    void gradient(const double* m, const double* u, double* p, double* g, SolveStats* st);
    void linearize(const double* m, const double* u, const double* p);
    // tol <= 0: the problem's tolerance
    void inc_forward(int nc, const double* mhat, int ldm, double* uhat, int ldu, SolveStats* st,
                     double tol = 0.0);
    void inc_adjoint(int nc, bool gn, const double* mhat, int ldm, const double* uhat, int ldu,
                     double* phat, int ldp, SolveStats* st);
    void hessian(int mode, int nc, const double* mhat, int ldm, double* out, int ldo,
                 SolveStats* st);
    // the three stages of a Hessian action around the two solves
    void inc_forward_rhs(int nc, const double* mhat, int ldm, double* rhs, int ldr);
    void inc_adjoint_rhs(int nc, bool gn, const double* mhat, int ldm, const double* uhat, int ldu,
                         double* rhs, int ldr);
    // rm: R mhat already computed (full modes), added instead of computed here
    void hess_output(int mode, int nc, const double* mhat, int ldm, const double* uh, int ldu,
                     const double* ph, int ldp, double* out, int ldo, const double* rm = nullptr);
    // s: the stream to run on (the context's stream when null); ws: when not
    // null, 6 n nc doubles of workspace used instead of the problem's scratch
    void prior_apply(int nc, const double* x, int ldx, double* y, int ldy, bool accumulate = false,
                     hipStream_t s = nullptr, double* ws = nullptr);
    void prior_solve(int nc, const double* x, int ldx, double* y, int ldy, SolveStats* st);
    void mass_apply(int nc, const double* x, int ldx, double* y, int ldy);
    // ws: when not null, 4 n nc doubles of workspace instead of the problem's scratch
    void mass_solve(int nc, const double* x, int ldx, double* y, int ldy, hipStream_t s = nullptr,
                    double* ws = nullptr);
    void prior_sample(int ns, const double* eta, int ldeta, double* out, int ldo, bool add_mean,
                      SolveStats* st);
    void white_noise(uint64_t seed, uint64_t stream, long long first, int ns, double* eta, int ld);

    // scratch of n x cap columns
    double* scratch(int which, int nc);
    double* obs_scratch(int nc);

    // A(m_lin) rebuilt in HA if a solve at another parameter replaced it
    void ensure_lin_hierarchy();
    // the state operator at parameter m (P1 hierarchy, and the P2 diagonal)
    void set_state(const double* m);
    // state solve / apply in the problem's state space (P1 or P2)
    void state_solve(int nc, const double* b, int ldb, double* x, int ldx, double tol, SolveStats* st,
                     double accept = 0.0);
    void state_apply(int nc, const double* x, int ldx, double* y, int ldy);

    // Workspaces of the algorithm drivers (Newton-CG, eigensolvers, samples,
    // variance, flexible CG): grown to the largest call, kept until the
    // problem is destroyed, so repeated calls of one shape allocate nothing.
    DBuf<double> ws_newton, ws_scal, ws_big, ws_small, ws_fcg, ws_eta;
    DenseWork dw;

  private:
    static constexpr int kScratch = 10;
    // second stream (default priority) on which a full Hessian action computes
    // R mhat while the two solves run on the context's stream
    hipStream_t side_ = nullptr;
    hipEvent_t ev_fork_ = nullptr, ev_join_ = nullptr;
    hipStream_t side_stream();
    int cap_ = 0;
    DBuf<double> w_[kScratch];
    int qcap_ = 0;
    DBuf<double> wq_;
    DBuf<double> red_;
};

// ---- device vector helpers (FP64, single stream) ---------------------------
double dev_dot(Ctx* ctx, int n, const double* a, const double* b);
void dev_dot_to(Ctx* ctx, int n, const double* a, const double* b, double* out);  // a^T b into device *out
void dev_dots(Ctx* ctx, int n, int nc, const double* a, int lda, const double* b, int ldb,
              double* host_out);
void dev_axpby(Ctx* ctx, int n, double a, const double* x, double b, double* y);  // y = a x + b y
void dev_copy(Ctx* ctx, int n, int nc, const double* x, int ldx, double* y, int ldy);
void dev_fill(Ctx* ctx, int n, double v, double* y);

}  // namespace hinv
