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
template <typename T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        // work queued on any stream may still use the buffer
        if (p) (void)hipDeviceSynchronize();
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    // (Re)allocates to hold at least cnt elements; contents are not kept.
    void ensure(size_t cnt) {
        if (cnt <= n && p) return;
        release();
        if (cnt == 0) return;
        HINV_HIP(hipMalloc(&p, cnt * sizeof(T)));
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
inline void timed_launch(Ctx* ctx, int cls, double work, F kernel, dim3 grid, dim3 block,
                         hipStream_t s, Args... args) {
    const int slot = ctx->timer.sample(cls, work);
    if (slot >= 0) {
        auto& k = ctx->timer.cls[cls];
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, k.ev[2 * slot], k.ev[2 * slot + 1], 0, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
    }
}

// ------------------------------------------------------------ constants ---
constexpr int kBlock = 256;   // threads per workgroup for grid kernels
constexpr int kCoarseMaxN = 8;  // coarsest multigrid level has N_c <= 8
constexpr int kMaxVecPartials = 520;  // partial sums per column of the PCG vector kernels
constexpr int kAutoBatch = 8;   // HINV_PREC_AUTO switches to FP32 refinement from this many columns

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

// Prior operator K_A = gamma K + delta M + beta M_boundary on a level with N
// cells (isotropic Theta = I).  All coefficients are constants of the mesh.
struct PriorParams {
    double gamma, delta, beta;
};

}  // namespace hinv
