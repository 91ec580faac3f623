// State-operator solves at the linearization point: multigrid PCG, flexible
// CG with the learned correction, and the harvest of its training pairs.
#pragma once

#include "cnn.h"
#include "problem.h"

namespace hinv {

struct FcgStats {
    int iterations = 0;           // flexible-CG iterations
    int fallback = 0;             // 1 when it stalled and multigrid PCG finished the solve
    int fallback_iterations = 0;  // PCG iterations of the fallback
    double relres = 0.0;          // final |b - A x| / |b|
    bool converged = false;
};

// Flexible CG (Notay's FCG keeping the last `truncation` directions) on
// A(m_lin) x = b, one right-hand side, FP64.  Preconditioner: one V-cycle
// z = V(r); with a network, plus its correction of the V-cycle's residual,
// c = s y((r - A z) / s), s = rms of that residual, at the energy-optimal step
// z += omega c, omega = c^T (r - A z) / c^T A c when positive.  A stall (less than a 10x
// residual drop over 20 iterations) hands the rest of the solve to multigrid PCG.
void state_solve_fcg(Problem& P, Cnn* cnn, const double* b, double* x, double rtol, int max_iter,
                     int truncation, FcgStats* st);

// Training pairs from the incremental forward solves at the linearization
// point: for random directions mhat, b = -C(u) mhat, x_k = k multigrid-PCG
// iterations on A x = b (k = 0..7 cycling over the rounds), r = b - A x_k,
// r' = r - A V(r) (the residual the V-cycle leaves), e' = A^-1 r'.  Each pair
// is cut to a crop x crop window at a seeded position and scaled by the rms s
// of r' there: in = (r' / s, m_lin, free-node mask), target = (e' / s, and the
// stencil of A there: east and north edge weights, diagonal).
void cnn_harvest(Problem& P, int npairs, uint64_t seed, int crop, float* in, float* target,
                 SolveStats* st);

}  // namespace hinv
