// Internal definitions shared by the libhinv translation units.
//
// Mesh conventions (identical to the public header): N x N cells on the unit
// square, node k(i,j) = j (N+1) + i, cell (i,j) split by the diagonal from
// (i,j) to (i+1,j+1) into the lower triangle (a,r,b) = ((i,j),(i+1,j),(i+1,j+1))
// and the upper triangle ((i,j),(i,j+1),(i+1,j+1)); r is the right-angle
// vertex; triangle index t = 2 (j N + i) + s.
#pragma once

#include <hip/hip_runtime.h>

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

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    DBuf<double> red;  // reduction scratch of the vector helpers
};

// ------------------------------------------------------------ constants ---
constexpr int kBlock = 256;   // threads per workgroup for grid kernels
constexpr int kCoarseMaxN = 8;  // coarsest multigrid level has N_c <= 8
constexpr int kAutoBatch = 8;   // HINV_PREC_AUTO switches to FP32 refinement from this many columns

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
