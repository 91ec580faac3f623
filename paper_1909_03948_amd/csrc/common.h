// Internal definitions shared by the libhinv translation units.
//
// Mesh conventions (identical to the public header): N x N cells on the unit
// square, node k(i,j) = j (N+1) + i, cell (i,j) split by the diagonal from
// (i,j) to (i+1,j+1) into the lower triangle (a,r,b) = ((i,j),(i+1,j),(i+1,j+1))
// and the upper triangle ((i,j),(i,j+1),(i+1,j+1)); r is the right-angle
// vertex; triangle index t = 2 (j N + i) + s.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hinv.h"

namespace hinv {

// ---------------------------------------------------------------- errors ---
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error{code, msg}; }

#define HINV_HIP(expr)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            ::hinv::fail(e_ == hipErrorOutOfMemory ? HINV_ENOMEM : HINV_EHIP,               \
                         std::string(#expr) + ": " + hipGetErrorString(e_));               \
    } while (0)

#define HINV_LAUNCH_CHECK() HINV_HIP(hipGetLastError())

// -------------------------------------------------------- device buffers ---
struct Ctx;

// The context whose entry point is running on this thread: device buffers
// created meanwhile take their memory from its allocator.
inline thread_local Ctx* tl_ctx = nullptr;
struct CtxScope {
    Ctx* prev;
    explicit CtxScope(Ctx* c) : prev(tl_ctx) { tl_ctx = c; }
    ~CtxScope() { tl_ctx = prev; }
    CtxScope(const CtxScope&) = delete;
    CtxScope& operator=(const CtxScope&) = delete;
};

// Device memory of `owner` (its allocator callback, else hipMalloc; owner may
// be null: hipMalloc), and its stream-ordered return (defined below Ctx).
void* dev_alloc(Ctx* owner, size_t bytes);
void dev_free(Ctx* owner, void* p, size_t bytes);

template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    Ctx* owner = nullptr;  // context whose allocator provided p
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) dev_free(owner, p, n * sizeof(T));
        p = nullptr;
        n = 0;
        owner = nullptr;
    }
    // (Re)allocates to hold at least cnt elements; contents are not kept.
    void ensure(size_t cnt) {
        if (cnt <= n && p) return;
        release();
        if (cnt == 0) return;
        owner = tl_ctx;
        p = static_cast<T*>(dev_alloc(owner, cnt * sizeof(T)));
        n = cnt;
    }
    T* get() const { return p; }
};

// Sampled kernel timing: while a class is enabled, every `period`-th eagerly
// launched kernel of it (every one while `force` is set: the solver forces
// two warm iterations of every 16th solve) carries an event pair in its own
// dispatch (hipExtLaunchKernelGGL), so the pair brackets the kernel's
// execution alone, and the algorithmic bytes (or flops) of that launch are
// recorded with it.
struct KernelTimer {
    static constexpr int kClasses = 12;
    static constexpr int kPool = 2048;  // event pairs per class
    struct Class {
        bool on = false;
        int period = 16;
        long launches = 0;
        std::vector<hipEvent_t> ev;  // 2 * kPool, created on enable
        std::vector<double> work;    // per recorded pair
        int used = 0;
    } cls[kClasses];
    bool paused = false;  // set while a graph is being captured
    bool force = false;   // sample every launch (not every period-th)
    bool any_on() const {
        for (const auto& k : cls)
            if (k.on) return true;
        return false;
    }
    // Returns the event-pair slot this launch carries, or -1.
    int sample(int c, double work) {
        if (c < 0 || paused) return -1;
        Class& k = cls[c];
        if (!k.on) return -1;
        const long idx = k.launches++;
        if ((!force && idx % k.period) || k.used >= kPool) return -1;
        const int slot = k.used++;
        k.work[slot] = work;
        return slot;
    }
    // Launches that ran inside a graph replay: counted, not timed.
    void count_only(int c, long n) {
        if (c >= 0 && cls[c].on) cls[c].launches += n;
    }
    ~KernelTimer() {
        for (auto& k : cls)
            for (auto e : k.ev) (void)hipEventDestroy(e);
    }
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // caller-supplied device allocator (declared before every buffer of the
    // context, so it outlives them); has_alloc = false: hipMalloc / hipFree
    hinv_allocator alloc{};
    bool has_alloc = false;
    long long allocations = 0;  // device allocations made for this context
    DBuf<double> red;  // reduction scratch of the vector helpers
    double* host_red = nullptr;  // pinned landing buffer of their results (kHostRed doubles)
    static constexpr int kHostRed = 4096;
    KernelTimer timer;
    Ctx() = default;
    Ctx(const Ctx&) = delete;
    Ctx& operator=(const Ctx&) = delete;
    ~Ctx() {
        if (host_red) (void)hipHostFree(host_red);
    }
};

inline void* dev_alloc(Ctx* owner, size_t bytes) {
    void* p = nullptr;
    if (owner && owner->has_alloc) {
        p = owner->alloc.alloc(bytes, owner->stream, owner->alloc.user);
        if (!p) fail(HINV_ENOMEM, "allocator callback returned no memory for " + std::to_string(bytes) + " bytes");
    } else {
        HINV_HIP(hipMalloc(&p, bytes));
    }
    if (owner) ++owner->allocations;
    return p;
}

inline void dev_free(Ctx* owner, void* p, size_t bytes) {
    if (owner && owner->has_alloc) {
        // stream-ordered: work already queued on the stream may still use p
        owner->alloc.free(p, bytes, owner->stream, owner->alloc.user);
        return;
    }
    // library-owned memory: let the context's stream finish with it first (a
    // full Hessian action's internal stream joins that stream before returning)
    (void)hipStreamSynchronize(owner ? owner->stream : nullptr);
    (void)hipFree(p);
}

// Scratch for split-K partial products and the small dense factorizations.
struct DenseWork {
    DBuf<double> part;
    DBuf<double> shift;  // per-matrix diagonal shifts
    DBuf<double> tmp;    // block products of the blocked triangular inverse
    DBuf<double> rot;    // recorded Jacobi rotations (large s)
    DBuf<int> flag;
};

// Kernel classes of the timer (values of HINV_KCLASS_* in the public header).
// The bandwidth-bound classes are timed apart for launches of one to seven
// columns (single right-hand sides: latency-bound at every mesh size here)
// and of eight or more (batched: bandwidth-bound).
enum KClass {
    kKDown = 0, kKUp = 1, kKBottom = 2, kKPcgApply = 3, kKPcgUpdate = 4, kKGram = 5,
    kKDownB = 6, kKUpB = 7, kKPcgApplyB = 8, kKPcgUpdateB = 9
};

// Launch of a timed class (-1: untimed): a sampled launch carries the class's
// next event pair in its dispatch.
template <typename F, typename... Args>
inline void timed_launch_shm(Ctx* ctx, int cls, double work, F kernel, dim3 grid, dim3 block, size_t shm,
                             hipStream_t s, Args... args) {
    const int slot = ctx->timer.sample(cls, work);
    if (slot >= 0) {
        auto& k = ctx->timer.cls[cls];
        hipExtLaunchKernelGGL(kernel, grid, block, shm, s, k.ev[2 * slot], k.ev[2 * slot + 1], 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
    }
}
template <typename F, typename... Args>
inline void timed_launch(Ctx* ctx, int cls, double work, F kernel, dim3 grid, dim3 block,
                         hipStream_t s, Args... args) {
    timed_launch_shm(ctx, cls, work, kernel, grid, block, 0, s, args...);
}

// ------------------------------------------------------------ constants ---
constexpr int kBlock = 256;   // threads per workgroup for grid kernels
constexpr int kCoarseMaxN = 8;  // coarsest multigrid level has N_c <= 8
constexpr int kMaxVecPartials = 520;  // partial sums per column of the PCG vector kernels
constexpr int kAutoBatch = 8;   // HINV_PREC_AUTO switches to FP32 refinement from this many columns

// A Hessian action chains two solves: the incremental adjoint's right-hand
// side carries u-hat, so the first solve's error reaches the output through
// the observation and W_uu terms.  Solved by FP32 refinement, the first solve
// runs to a tenth of the tolerance: at 1025^2 nodes and 1e-10 the action's
// relative error was 1.3e-8 with both solves at 1e-10 and 8.8e-10 with the
// first at 1e-11 (tightening the second instead changed nothing), while FP64
// PCG, which overshoots the tolerance by up to one iteration's reduction,
// gave 3.8e-10 without it.  The problem's tolerance stays the acceptance
// bar: a column whose FP64 residual cannot go lower (its rounding floor, seen
// near 3e-11 for some R-orthonormal directions at that size) ends there.
inline double chained_first_rtol(int precision, int nc, double rtol) {
    const bool ir = precision == HINV_PREC_FP32_IR || (precision == HINV_PREC_AUTO && nc >= kAutoBatch);
    return ir ? 0.1 * rtol : rtol;
}

// Timer class of a launch of `nc` columns (the batched class from kAutoBatch up).
inline int kclass_for(int base, int nc) {
    if (nc < kAutoBatch) return base;
    switch (base) {
        case kKDown: return kKDownB;
        case kKUp: return kKUpB;
        case kKPcgApply: return kKPcgApplyB;
        case kKPcgUpdate: return kKPcgUpdateB;
        default: return base;
    }
}

// Chebyshev smoother: degree 2, targets the interval [0.5, 2] of the
// Jacobi-scaled operator (2 bounds the spectrum by Gershgorin for both the
// five-point state operator and the prior operator K_A).
constexpr double kChebLo = 0.5, kChebHi = 2.0;

__host__ __device__ inline int knode(int i, int j, int N) { return j * (N + 1) + i; }

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Prior operator K_A = gamma K_Theta + delta M + beta M_boundary on a level
// with N cells; Theta = [[t11, t12], [t12, t22]] (identity by default).  All
// coefficients are constants of the mesh.
struct PriorParams {
    double gamma, delta, beta;
    double t11 = 1.0, t12 = 0.0, t22 = 1.0;
};

}  // namespace hinv
