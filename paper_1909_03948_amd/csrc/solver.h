// Geometric-multigrid preconditioned CG on the structured mesh, batched over
// right-hand sides, in FP64 or as FP32 PCG inside FP64 iterative refinement.
#pragma once

#include <algorithm>
#include <cstdlib>
#include <functional>

#include <memory>

#include "common.h"
#include "grid.h"

namespace hinv {

enum OpKind { kOpState = 0, kOpPrior = 1 };

// One multigrid level.  For the state operator it holds the triangle
// coefficients and the five-point weights in FP64 and FP32; the prior
// operator needs nothing but N.
struct Level {
    int N = 0, n = 0;
    DBuf<double> cT, wE64, wN64, dinv64;
    DBuf<float> wE32, wN32, dinv32;
};

// Launch shapes tuned by timing and taken from the persistent cache, process-wide.
void tuner_counts(long* timed, long* cached);

struct SolveStats {
    int solves = 0, iterations = 0, refinements = 0, fallbacks = 0;
    double max_relres = 0.0;
    bool converged = true;
    void add(const SolveStats& o) {
        solves += o.solves;
        iterations += o.iterations;
        refinements += o.refinements;
        fallbacks += o.fallbacks;
        if (o.max_relres != o.max_relres || o.max_relres > max_relres) max_relres = o.max_relres;  // NaN stays
        converged = converged && o.converged;
    }
};

// Per-precision scratch of the batched PCG (column-major, ld = level size).
template <typename T>
struct PcgWork {
    int cap = 0;  // columns
    DBuf<T> x, r, z, p, p2, q;
    std::vector<std::unique_ptr<DBuf<T>>> lb, lx, lt;  // per level b, x, t
};

struct ColState {
    double bb;   // |b|^2 of the inner problem
    double rz, pq, rr, tol2, alpha, beta;
    double rz_new;  // r^T z of the current iteration, summed once by the PCG apply kernel
    double obb;  // |b|^2 of the outer (FP64) problem
    double its;  // PCG iterations this column has taken in the current inner solve
};

// A hierarchy may stack ninst instances of one mesh size (their own state
// coefficients, or their own prior parameters): a call with nc columns then
// gives nc / ninst consecutive columns to each instance, in instance order.
class Hierarchy {
  public:
    Hierarchy(Ctx* ctx, OpKind kind, int N, PriorParams pp, int ninst = 1,
              const PriorParams* inst_pp = nullptr);
    ~Hierarchy();
    // State operator: builds all levels of instance inst from the FP64
    // parameter field m (device).
    void set_state_coefficient(const double* m, int inst = 0);
    // Solves A x = b for nc columns.  b and x: device FP64, column-major.
    // Only the free rows of b are read; x is zero on Dirichlet rows.
    // accept > rtol: rtol is a goal; once an FP64 pass no longer lowers the
    // residuals of the remaining columns (their FP64 rounding floor) and all
    // of them are at or below accept, the solve ends as converged.
    void solve(int nc, const double* b, int ldb, double* x, int ldx, int precision, double rtol,
               int max_iter, SolveStats* st, double accept = 0.0);
    // y = A x (FP64, masked to free rows).
    void apply(int nc, const double* x, int ldx, double* y, int ldy);
    // z = one V-cycle (FP64) applied to r, zero on Dirichlet rows.
    void precondition(int nc, const double* r, int ldr, double* z, int ldz);
    // Level-0 triangle coefficients c_T (state operator only).
    const double* coefficient(int inst = 0) const {
        return lev_[0]->cT.get() + (size_t)inst * 2 * N_ * N_;
    }
    const double* weightsE(int inst = 0) const { return lev_[0]->wE64.get() + (size_t)inst * n_; }
    const double* weightsN(int inst = 0) const { return lev_[0]->wN64.get() + (size_t)inst * n_; }
    const double* inv_diag(int inst = 0) const { return lev_[0]->dinv64.get() + (size_t)inst * n_; }
    bool ready() const { return ready_; }
    int N() const { return N_; }
    int n() const { return n_; }
    int ninst() const { return ninst_; }
    double inner_tol32 = 1e-5;  // FP32 inner relative tolerance of the refinement loop (its lower bound)

  private:
    // Runs the PCG iterations of the current inner solve.  tail, when given,
    // is enqueued before every completion check (the refinement step, gated
    // on the device to the columns whose PCG has finished); returns true when
    // the last check found every column finished, its read-back (column states
    // and outer flags in the host block) then follows the tail.
    template <typename T>
    bool pcg(int nc, int max_iter, int* iters, const std::function<void()>* tail = nullptr);
    template <typename T>
    void pcg_iteration(int nc, int cur, int first);
    template <typename T>
    hipGraphExec_t pcg_graph(int nc, int reps);
    template <typename T>
    hipGraphExec_t prologue_graph(int nc, int reps);
    template <typename T>
    hipGraphExec_t capture(int nc, bool prologue, int reps);
    void drop_graphs();
    template <typename T>
    void vcycle(int nc, int check);
    template <typename T, typename TI>
    void vcycle_impl(int nc, int check);
    struct PcgRed pcg_red(int nc) const;
    template <typename T>
    PcgWork<T>& work();
    void ensure_cols(int nc);
    void set_columns(int nc);
    // Launch shape of the batched kernels: V-cycle tiles (small: 8 / 16 nodes
    // per coarse / fine side, else 16 / 32), columns per V-cycle workgroup
    // (the coefficient tile is staged once for them) and node blocks per
    // workgroup of the PCG vector kernels.  Chosen by timing on the first call of each
    // (column count, precision); HINV_AUTOTUNE=0 uses the fixed rule instead.
    struct LaunchShape {
        bool small;         // small tiles on every level
        int small_max = 0;  // otherwise small tiles on the levels with N_l <= small_max
        int per;
        int cb;  // columns per workgroup of the V-cycle kernels
        // nodes per workgroup of the PCG vector kernels; 0: 256 per.  A
        // balanced chunk spreads a column over a whole number of workgroups
        // per compute unit instead of whole 256-node blocks.
        int chunk = 0;
    };
    bool small_tiles(int l) const { return shape_.small || lev_[l]->N <= shape_.small_max; }
    // Cycles with small tiles everywhere (few columns: the coarse launches are
    // latency bound) run two coarse levels a launch; one instance only
    // (HINV_NO_PAIRS: one level a launch throughout).
    bool pair_levels() const { return shape_.small && ninst_ == 1 && !no_pairs_; }
    bool no_pairs_ = std::getenv("HINV_NO_PAIRS") != nullptr;
    int cus_ = 0;  // compute units of the device
    bool finest_wide(int nc) const;
    LaunchShape default_shape(int nc) const;
    int min_per() const;
    template <typename T>
    void tune_shape(int nc);
    void build_coarse(int inst);
    // calls fn with the operator of level l in precision T (all instances)
    template <typename T, class F>
    void with_op(int l, F fn);

    Ctx* ctx_;
    OpKind kind_;
    int N_, n_;
    PriorParams pp_;
    bool ready_ = false;
    int ninst_ = 1;
    int cpi_ = 1;  // columns per instance of the current call
    LaunchShape shape_{true, 1, 1};  // launch shape of the current call
    std::vector<std::pair<long long, LaunchShape>> tuned_;  // (nc * 2 + fp32, shape)
    std::vector<std::pair<long long, int>> last_iters_;    // (nc * 2 + fp32, PCG iterations)
    std::vector<PriorParams> inst_pp_;
    std::vector<char> inst_ready_;
    DBuf<KARow<double>> karow64_;  // stacked prior rows: [level][instance][9]
    DBuf<KARow<float>> karow32_;
    std::vector<std::unique_ptr<Level>> lev_;
    DBuf<double> cinv64_;
    DBuf<float> cinv32_;
    int nc_coarse_ = 0;
    // Largest true-residual reduction of one FP32 refinement pass (after the
    // first) in the last FP32 solve: the inner PCG is not run much below it.
    double rho32_ = 0.0;
    // refinement state
    int cap_ = 0;
    DBuf<double> x64_, r64_;
    DBuf<double> partial_;
    DBuf<double> pcg_part_;  // partial sums of r^T z, p^T q, r^T r per workgroup and column
    int red_stride_ = 0;
    // Column states and flags in one device block [st[cap] | act[cap] | oact[cap]
    // | tdone[cap]] (inner and outer activity, refinement step taken this
    // pass), so that one copy reads back what a completion check needs; the
    // pinned host block mirrors its layout.
    template <typename T>
    struct View {
        T* p = nullptr;
        T* get() const { return p; }
    };
    DBuf<char> sblk_;
    View<ColState> st_;
    View<int> act_, oact_, tdone_;
    DBuf<double> colnorm_;  // per column |r| used to scale the inner right-hand side
    char* hblk_ = nullptr;   // pinned, room for 4096 columns
    ColState* host_st() const { return reinterpret_cast<ColState*>(hblk_); }
    int* host_act() const { return reinterpret_cast<int*>(hblk_ + sizeof(ColState) * cap_); }
    int* host_oact() const { return host_act() + cap_; }
    // reads back the column states and the first nflags flag arrays (act, then
    // oact) of nc columns in one copy; no synchronization
    void read_state(hipStream_t s, int nc, int nflags);
    hipStream_t gs_ = nullptr;             // private stream for graph capture
    hipStream_t launch_stream_ = nullptr;  // stream the PCG kernels go to (capture or caller)
    // FP64 / FP32 graphs of 2 reps iterations, reps = 1 .. kMaxReps: a run of
    // iterations is one graph launch (each launch costs ~8 us of idle GPU)
    static constexpr int kMaxReps = 6;
    hipGraphExec_t gexec_[2][kMaxReps] = {};
    int gexec_nc_[2][kMaxReps] = {};
    // FP64 / FP32 prologue graphs (V-cycle, first iteration) followed by
    // 2 reps iterations, reps = 0 .. kMaxReps
    hipGraphExec_t gpro_[2][kMaxReps + 1] = {};
    int gpro_nc_[2][kMaxReps + 1] = {};
    long solves_ = 0;  // inner solves so far (every 16th runs its prologue eagerly while timing)
    PcgWork<double> w64_;
    PcgWork<float> w32_;
};

}  // namespace hinv
