// Fused multigrid V-cycle and PCG kernels (included by solver.hip only).
//
// V-cycle, per level above the bottom (N_l > kBottomN), two LDS-tiled kernels:
//   k_down: x2 = S(b) (two Chebyshev steps from zero), r = b - A x2, b_coarse = P^T r
//   k_up:   x = x2 + P x_coarse, then two Chebyshev steps on A x = b
// and one kernel for all levels with N_l <= kBottomN (one workgroup per column,
// every vector in LDS in FP32, the coarsest level solved with its dense inverse).
// PCG reductions finish in the producing kernel: the last workgroup of a column
// to arrive sums the per-workgroup partials in a fixed order.
#pragma once

#include "grid.h"
#include "solver.h"

namespace hinv {

// Workgroup barrier for data exchanged through LDS.  __syncthreads() also
// orders global memory, so every wave first waits for all of its outstanding
// global loads; no kernel here exchanges data through global memory within a
// launch (each reads buffers that only earlier launches write), so with this
// barrier loads issued before it stay in flight across it and their latency
// overlaps the staging and reductions that follow.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Tile sides: large tiles (less halo work) for batches, small tiles (more
// workgroups) when few columns make the V-cycle latency bound.
constexpr int kTCBig = 16, kTFBig = 32;      // coarse / fine nodes per tile side
constexpr int kTCSmall = 8, kTFSmall = 16;
constexpr int kTCWide = 9, kTFWide = 18;     // finest level of small-tile cycles with many workgroups
constexpr int kTPair = 4;      // k_down2: level-C tile side
constexpr int kPairMaxN = 256;  // k_down2 pairs levels whose finer one has N_l <= this
constexpr int kTFChain = 16;   // k_up_chain: level-0 tile side
constexpr int kChainLen = 4;   // k_up_chain: levels a launch (measured: 4 > 2 at N = 1024)
constexpr int kSmallTileCols = 8;            // batches below this use the small tiles
constexpr int kBottomN = 32;   // levels with N_l <= kBottomN run in the bottom kernel
constexpr int kBottomLevels = 4;  // at most (N_l = 64, 32, 16, 8 when kBottomN = 64)

// Chebyshev degree-2 coefficients passed to the smoothing kernels.
struct ChebCoef {
    double inv_theta, theta, cA, cB, c1;  // pre: x = cA d0 + cB D^-1 r1; post: (1 + c1) d0 + cB D^-1 r1
};

// In-kernel reductions: every workgroup writes one partial sum per column to
// part[col * stride + blk]; a later kernel (after the kernel boundary, so no
// fences are needed) sums them in a fixed order.
// First phase: this thread's strided share of the partials (loads only, so
// that a kernel can issue them together with its other loads).
// In two steps, so that a kernel can issue other loads in between:
// partial_first loads this thread's first partial (usually its only one),
// partial_rest adds the further ones.
__device__ inline double partial_first(const double* part, int col, int stride, int nblk) {
    const int t = threadIdx.x;
    return t < nblk ? part[(size_t)col * stride + t] : 0.0;
}
__device__ inline double partial_rest(double s, const double* part, int col, int stride, int nblk) {
    const double* p = part + (size_t)col * stride;
    for (int b = threadIdx.x + blockDim.x; b < nblk; b += blockDim.x) s += p[b];
    return s;
}
// The whole share of nblk >= 1 partials with the first kShareLoads per thread
// loaded without branches (clamped index, dropped afterwards), so that they
// are in flight together with the caller's other loads (a loop waits for
// each load it accumulates); more partials than kShareLoads per thread
// follow in a loop.  Summed in index order, as partial_rest does.
constexpr int kShareLoads = 3;
__device__ inline double partial_share(const double* part, int col, int stride, int nblk) {
    const double* p = part + (size_t)col * stride;
    const int t = threadIdx.x, nt = blockDim.x;
    double v[kShareLoads];
#pragma unroll
    for (int k = 0; k < kShareLoads; ++k) v[k] = p[min(t + k * nt, nblk - 1)];
    double s = t < nblk ? v[0] : 0.0;
#pragma unroll
    for (int k = 1; k < kShareLoads; ++k)
        if (t + k * nt < nblk) s += v[k];
    for (int b = t + kShareLoads * nt; b < nblk; b += nt) s += p[b];
    return s;
}

// Index i clamped into the mesh [0, N]: tile loads read a valid node for
// every slot and drop the off-mesh ones afterwards.  Used on tiles of at
// most kFlatLoads elements a thread (the few-column cycles, latency bound);
// larger tiles keep branched loads and fewer registers.
__device__ inline int clamp_node(int i, int N) { return min(max(i, 0), N); }
template <int E>
constexpr bool kFlatLoads = E <= 3;

// Waves of the workgroup as a uniform value (read once, outside the
// single-thread code that sums the per-wave slots).
__device__ inline int group_waves() { return __builtin_amdgcn_readfirstlane((int)(blockDim.x >> 6)); }

// Second phase: the workgroup total of the shares, returned to every thread.
__device__ inline double share_total(double s) {
    __shared__ double ps[16];
    __shared__ double tot;
    const int nw = group_waves();
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) ps[threadIdx.x >> 6] = s;
    lds_barrier();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += ps[w];
        tot = t;
    }
    lds_barrier();
    return tot;
}

__device__ inline double partial_total(const double* part, int col, int stride, int nblk) {
    return share_total(partial_share(part, col, stride, nblk));
}

// Partial-sum buffers of the PCG inner products ([ncols][stride] each).
struct PcgRed {
    double* rz;
    double* pq;
    double* rr;
    int stride;
    int nrz;  // number of partials of r^T z (workgroups of the last V-cycle kernel)
    int nvec; // number of partials of p^T q and r^T r (workgroups of the PCG vector kernels)
    int per;  // node blocks of 256 per workgroup: sets the PCG vector kernels' threads
    int chunk;  // consecutive nodes per workgroup in the PCG vector kernels (<= kVecNodes threads)
};

// Threads per workgroup of the PCG vector kernels: 256 per node block up to
// 1024, so a workgroup covers its 256 per nodes in at most kVecNodes passes.
__host__ __device__ inline int vec_threads(int per) { return per >= 4 ? 1024 : 256 * per; }
constexpr int kVecNodes = 4;

// Workgroup sum with its own LDS slot; result valid in thread 0.
__device__ inline double group_sum(double v) {
    __shared__ double part[16];
    const int nw = group_waves();
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    lds_barrier();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < nw; ++w) r += part[w];
    return r;
}

// Convergence test at the start of a V-cycle: r^T r of the PCG update that
// precedes it is summed from its partials (share: this thread's part of
// them, loaded ahead by the caller); a column at its tolerance stops (every
// workgroup reaches the same decision; workgroup 0 records it).
__device__ inline bool column_done_share(double share, const PcgRed& red, int col, ColState* st, int* act,
                                         bool lead) {
    const double rr = share_total(share);
    const ColState& c = st[col];
    const bool done = rr <= c.tol2 * c.bb;
    if (lead && threadIdx.x == 0) {
        st[col].rr = rr;
        if (done) act[col] = 0;
    }
    return done;
}

// XCD-aware tile order.  The hardware hands consecutive workgroups to the
// eight XCDs in turn, so in the plain order the tiles next to a tile (which
// read its halo rows) run on other XCDs and fetch those rows into their own
// L2 again.  Here the j-th workgroup of XCD x (dispatch index h = 8 j + x)
// takes logical tile x P + j with P = floor(T / 8) of the T workgroups: each
// XCD sweeps a contiguous run of tiles in row-major order (x fastest, then y,
// then the column block), so left/right and most upper/lower halos come from
// its own L2.  The last T - 8 P workgroups keep the plain order.  A
// bijection of [0, T); returns the logical (x, y, z) of this workgroup.
__device__ inline int3 xcd_tile() {
    const int X = gridDim.x, Y = gridDim.y;
    const int T = X * Y * gridDim.z;
    const int h = blockIdx.x + X * (blockIdx.y + Y * blockIdx.z);
    const int P = T >> 3;
    const int L = h < 8 * P ? (h & 7) * P + (h >> 3) : h;
    const int z = L / (X * Y), r = L - z * X * Y;
    return make_int3(r % X, r / X, z);
}

// --------------------------------------------------------------- k_down ---
// Grid: (tiles over coarse x, tiles over coarse y, column blocks).  Coarse
// tile [I0, I0+kTC) x [J0, J0+kTC) needs the fine residual on
// [2 I0 - 1, 2 I1 + 1], hence x2 one node further out and b two nodes further
// out.  The operator rows of the tile are staged once per problem instance;
// the workgroup then sweeps cb consecutive columns.
// b may be of a wider type TB than the level's vectors (the finest level of a
// V-cycle in FP32 preconditioning an FP64 PCG reads the FP64 residual).
template <typename T, class Op, int kTC, typename TB = T, int WPE = 1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_down(Op op_, const TB* __restrict__ b, T* __restrict__ x,
                                              int ld, T* __restrict__ bc, int ldc, int dirichlet,
                                              int* __restrict__ act, ChebCoef cc, PcgRed red,
                                              ColState* __restrict__ st, int check, int nc, int cb) {
    constexpr int TW = 2 * kTC + 5, NN = TW * TW;
    // the prior operator (7 points, constant coefficients) on large tiles
    // reads its class table: a third of the LDS, more workgroups per compute
    // unit, for the batched solves that are bound by LDS traffic (measured:
    // a 220-column prior solve at N = 1024 9% faster; on the small tiles of
    // single-column cycles the staged rows stay faster, except on tiles of
    // interior nodes only, which apply row 0 of the table throughout (HYB)
    constexpr bool NE = kNorthEast<Op>;
    constexpr bool KA = NE && kTC == kTCBig;
    constexpr bool HYB = NE && !KA;
    __shared__ T sb[NN], sx[NN], sr[NN];
    __shared__ T tc[NE && !KA ? NN : 1], te[KA ? 1 : NN], tn[KA ? 1 : NN], tdv[KA ? 1 : NN], tg[NE && !KA ? NN : 1];
    __shared__ KARow<T> krows[KA ? 9 : 1];
    const TileStencil<T> ts{tc, te, tn, tg, tdv};
    const int N = op_.N, N1 = N + 1, Nc = N / 2, Nc1 = Nc + 1;
    const int3 tb = xcd_tile();
    const int I0 = tb.x * kTC, J0 = tb.y * kTC;
    const int I1 = min(I0 + kTC - 1, Nc), J1 = min(J0 + kTC - 1, Nc);
    const int ox = 2 * I0 - 3, oy = 2 * J0 - 3;  // global coordinates of local (0, 0)
    const TileKA<T, TW> tk{krows, ox, oy, N, ox >= 1 && oy >= 1 && ox + TW - 1 <= N - 1 && oy + TW - 1 <= N - 1};
    const bool inner = HYB && tk.interior;  // uniform in the workgroup
    KARow<T> r0{};  // inner tiles: row 0 of the instance's class table (uniform: scalar registers)
    auto tapply = [&](int l, const T* v) -> T {
        if constexpr (KA) return tk.apply(l, v);
        else if constexpr (HYB) return inner ? row_apply(r0, TW, l, v) : tile_apply<NE>(ts, TW, l, v);
        else return tile_apply<NE>(ts, TW, l, v);
    };
    auto tdinv = [&](int l) -> T {
        if constexpr (KA) return tk.dinv(l);
        else if constexpr (HYB) return inner ? r0.dinv : tdv[l];
        else return tdv[l];
    };
    const T inv_theta = (T)cc.inv_theta, cA = (T)cc.cA, cB = (T)cc.cB;
    const int own_i1 = min(2 * I1 + 1, N), own_j1 = min(2 * J1 + 1, N);
    constexpr int E = (NN + 255) / 256;  // tile elements per thread
    const void* staged = nullptr;  // the staged rows belong to this instance
    const int c_end = min(nc, (tb.z + 1) * cb);
    for (int col = tb.z * cb; col < c_end; ++col) {
        // with the convergence test on, the lead workgroup clears act[col]
        // (column_done_share below) while other workgroups of this launch read it:
        // one decision for the whole workgroup, or its waves could see
        // different values and meet different barriers (without the test no
        // kernel of the launch writes act)
        if (act && !(check ? __syncthreads_or(act[col]) : act[col])) continue;
        const auto& op = op_.at(col);  // operator of the instance owning this column
        const TB* bcol = b + (size_t)col * ld;
        T* xcol = x + (size_t)col * ld;
        // loads first: b, the convergence test's partials, then the operator
        // rows, so that their latencies overlap.  On small tiles of the prior
        // operator b is read at a clamped node without a branch (a load
        // converted inside its branch waits there for its data) and the
        // off-mesh entries are dropped at the LDS store.  Large tiles (many
        // workgroups a compute unit) keep the branch and their registers, and
        // so does the state operator, whose row loads from global memory
        // cover the latency of b (measured: the branch-free form no faster)
        constexpr bool kFlat = kFlatLoads<E> && NE;
        T vb[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = threadIdx.x + 256 * e;
            const int i = ox + t % TW, j = oy + t / TW;
            if constexpr (kFlat)
                vb[e] = (T)bcol[clamp_node(j, N) * N1 + clamp_node(i, N)];
            else
                vb[e] = (t < NN && i >= 0 && i <= N && j >= 0 && j <= N) ? (T)bcol[j * N1 + i] : (T)0;
        }
        const double rr_share = check ? partial_share(red.rr, col, red.stride, red.nvec) : 0.0;
        lds_barrier();  // the previous column's LDS reads are done
        if (instance_key(op) != staged) {
            if constexpr (KA) {
                if (threadIdx.x < 9) krows[threadIdx.x] = op.rows[threadIdx.x];
            } else if constexpr (HYB) {
                if (inner)
                    r0 = op.rows[0];
                else
                    stage_stencil<TW, 256>(op, ts, ox, oy);
            } else {
                stage_stencil<TW, 256>(op, ts, ox, oy);
            }
            staged = instance_key(op);
        }
        if (check && column_done_share(rr_share, red, col, st, act, tb.x == 0 && tb.y == 0)) continue;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = threadIdx.x + 256 * e;
            const int i = ox + t % TW, j = oy + t / TW;
            if (t < NN) sb[t] = !kFlat || (i >= 0 && i <= N && j >= 0 && j <= N) ? vb[e] : (T)0;
        }
        lds_barrier();
        // d0 = D^-1 b / theta on the whole tile (zero off the free nodes)
        for (int t = threadIdx.x; t < NN; t += blockDim.x) sr[t] = tdinv(t) * sb[t] * inv_theta;
        lds_barrier();
        // x2 = cA d0 + cB D^-1 (b - A d0) on local [1, TW-1)^2; owned nodes to global
        {
            constexpr int W = TW - 2;
            for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
                const int il = 1 + t % W, jl = 1 + t / W, l = jl * TW + il;
                const T v = cA * sr[l] + cB * tdinv(l) * (sb[l] - tapply(l, sr));
                sx[l] = v;
                const int i = ox + il, j = oy + jl;
                if (i >= 2 * I0 && i <= own_i1 && j >= 2 * J0 && j <= own_j1) xcol[j * N1 + i] = v;
            }
        }
        lds_barrier();
        // residual b - A x2 on the free nodes of local [2, TW-2)^2
        {
            constexpr int W = TW - 4;
            for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
                const int l = (2 + t / W) * TW + 2 + t % W;
                const T v = sb[l] - tapply(l, sx);
                sr[l] = tdinv(l) != (T)0 ? v : (T)0;
            }
        }
        lds_barrier();
        // restriction P^T onto the coarse tile
        T* bccol = bc + (size_t)col * ldc;
        const int cw = I1 - I0 + 1, ch = J1 - J0 + 1;
        auto res = [&](int i, int j) { return sr[(j - oy) * TW + (i - ox)]; };
        for (int t = threadIdx.x; t < cw * ch; t += blockDim.x) {
            const int I = I0 + t % cw, J = J0 + t / cw;
            T v = 0;
            if (!(dirichlet && (J == 0 || J == Nc))) {
                const int i = 2 * I, j = 2 * J;
                T sm = 0;
                if (i > 0) sm += res(i - 1, j);
                if (i < N) sm += res(i + 1, j);
                if (j > 0) sm += res(i, j - 1);
                if (j < N) sm += res(i, j + 1);
                if (i < N && j < N) sm += res(i + 1, j + 1);
                if (i > 0 && j > 0) sm += res(i - 1, j - 1);
                v = res(i, j) + (T)0.5 * sm;
            }
            bccol[J * Nc1 + I] = v;
        }
    }
}

// ----------------------------------------------------------------- k_up ---
// Grid: (tiles over fine x, tiles over fine y, column blocks).  Fine tile O of
// kTF x kTF nodes; x = x2 + P x_coarse is formed two nodes around O (x2 is
// read from its own buffer: neighbouring workgroups write the output), b and
// the first Chebyshev correction d0 one node around O.  Optionally writes the
// workgroup's part of sum_k rv_k x_k (the PCG inner product r^T z).
// b and rv may be of a wider type TB and the output x of a wider type TX than
// the level's vectors (see k_down).
template <typename T, class Op, int kTF, typename TB = T, typename TX = T, int WPE = 1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE))) void k_up(Op op_, const TB* __restrict__ b, const T* __restrict__ x2,
                                            TX* __restrict__ x, int ld, const T* __restrict__ xc,
                                            int ldc, int dirichlet,
                                            const int* __restrict__ act, ChebCoef cc,
                                            const TB* __restrict__ rv, PcgRed red, int nc, int cb) {
    constexpr int TW = kTF + 4, NN = TW * TW;
    constexpr bool NE = kNorthEast<Op>;
    constexpr bool KA = NE && kTF == kTFBig;  // class table for the prior operator (see k_down)
    constexpr bool HYB = NE && !KA;           // row 0 on interior small tiles (see k_down)
    __shared__ T sx[NN], sd[NN], sb[NN];
    __shared__ T tc[NE && !KA ? NN : 1], te[KA ? 1 : NN], tn[KA ? 1 : NN], tdv[KA ? 1 : NN], tg[NE && !KA ? NN : 1];
    __shared__ KARow<T> krows[KA ? 9 : 1];
    const TileStencil<T> ts{tc, te, tn, tg, tdv};
    const int N = op_.N, N1 = N + 1, Nc1 = N / 2 + 1;
    const int3 tb = xcd_tile();
    const int i0 = tb.x * kTF, j0 = tb.y * kTF;
    const int i1 = min(i0 + kTF - 1, N), j1 = min(j0 + kTF - 1, N);
    const int ox = i0 - 2, oy = j0 - 2;
    const TileKA<T, TW> tk{krows, ox, oy, N, ox >= 1 && oy >= 1 && ox + TW - 1 <= N - 1 && oy + TW - 1 <= N - 1};
    const bool inner = HYB && tk.interior;  // uniform in the workgroup
    KARow<T> r0{};  // inner tiles: row 0 of the instance's class table (uniform: scalar registers)
    auto tapply = [&](int l, const T* v) -> T {
        if constexpr (KA) return tk.apply(l, v);
        else if constexpr (HYB) return inner ? row_apply(r0, TW, l, v) : tile_apply<NE>(ts, TW, l, v);
        else return tile_apply<NE>(ts, TW, l, v);
    };
    auto tdinv = [&](int l) -> T {
        if constexpr (KA) return tk.dinv(l);
        else if constexpr (HYB) return inner ? r0.dinv : tdv[l];
        else return tdv[l];
    };
    auto tcen = [&](int l) -> T {
        if constexpr (KA) return tk.center(l);
        else if constexpr (HYB) return inner ? r0.c : tile_center<NE>(ts, TW, l);
        else return tile_center<NE>(ts, TW, l);
    };
    const T inv_theta = (T)cc.inv_theta, theta = (T)cc.theta, cB = (T)cc.cB, c1 = (T)cc.c1;
    constexpr int E = (NN + 255) / 256;  // tile elements per thread
    const void* staged = nullptr;
    const int c_end = min(nc, (tb.z + 1) * cb);
    for (int col = tb.z * cb; col < c_end; ++col) {
        if (act && !act[col]) continue;
        const auto& op = op_.at(col);  // operator of the instance owning this column
        const TB* bcol = b + (size_t)col * ld;
        const T* x2col = x2 + (size_t)col * ld;
        TX* xcol = x + (size_t)col * ld;
        const T* ccol = xc + (size_t)col * ldc;
        // loads first (b, x2 and the two coarse values of the prolongation,
        // then the operator rows) so that their latencies overlap.  P x_c at
        // (i, j): the coarse node (i/2, j/2) when both are even, else the mean
        // of the two coarse ends of the fine edge through (i, j).
        TB vb[E];  // small tiles: read at a clamped node without a branch (see k_down)
        T vx[E], pc0[E], pc1[E];
        bool even[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = threadIdx.x + 256 * e;
            const int i = ox + t % TW, j = oy + t / TW;
            const bool in = t < NN && i >= 0 && i <= N && j >= 0 && j <= N;
            const bool fr = in && !(dirichlet && (j == 0 || j == N));
            const int I = i >> 1, J = j >> 1;
            const int a0 = J * Nc1 + I, a1 = (J + (j & 1)) * Nc1 + I + (i & 1);
            if constexpr (kFlatLoads<E>)
                vb[e] = bcol[clamp_node(j, N) * N1 + clamp_node(i, N)];  // dropped at its store when !in
            else
                vb[e] = in ? bcol[j * N1 + i] : (TB)0;
            vx[e] = fr ? x2col[j * N1 + i] : (T)0;
            pc0[e] = fr ? ccol[a0] : (T)0;
            pc1[e] = fr ? ccol[a1] : (T)0;
            even[e] = !((i | j) & 1);
        }
        // small tiles (one output node a thread, the few-column cycles): rv at
        // the thread's output node is loaded with the tile; large tiles read it
        // at use (prefetching four values costs them occupancy)
        const int w = i1 - i0 + 1, h = j1 - j0 + 1;
        constexpr bool kPre = kTF * kTF <= 256;
        TB rv0 = 0;
        if constexpr (kPre) {
            const int t = threadIdx.x;
            if (rv && t < w * h) rv0 = rv[(size_t)col * ld + (j0 + t / w) * N1 + (i0 + t % w)];
        }
        lds_barrier();  // the previous column's LDS reads are done
        if (instance_key(op) != staged) {
            if constexpr (KA) {
                if (threadIdx.x < 9) krows[threadIdx.x] = op.rows[threadIdx.x];
            } else if constexpr (HYB) {
                if (inner)
                    r0 = op.rows[0];
                else
                    stage_stencil<TW, 256>(op, ts, ox, oy);
            } else {
                stage_stencil<TW, 256>(op, ts, ox, oy);
            }
            staged = instance_key(op);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = threadIdx.x + 256 * e;
            if (t < NN) {
                const int i = ox + t % TW, j = oy + t / TW;
                sx[t] = vx[e] + (even[e] ? pc0[e] : (T)0.5 * (pc0[e] + pc1[e]));
                sb[t] = (i >= 0 && i <= N && j >= 0 && j <= N) ? (T)vb[e] : (T)0;
            }
        }
        lds_barrier();
        // d0 = D^-1 (b - A x) / theta on local [1, TW-1)^2 (zero off the free nodes)
        {
            constexpr int W = TW - 2;
            for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
                const int l = (1 + t / W) * TW + 1 + t % W;
                sd[l] = tdinv(l) * (sb[l] - tapply(l, sx)) * inv_theta;
            }
        }
        lds_barrier();
        // x += (1 + c1) d0 + cB D^-1 r1 on O with r1 = r0 - A d0 = theta D d0 - A d0
        double dot = 0.0;
        for (int t = threadIdx.x; t < w * h; t += blockDim.x) {
            const int i = i0 + t % w, j = j0 + t / w;
            const int l = (j - oy) * TW + (i - ox), k = j * N1 + i;
            const T dk = sd[l];
            const T r1 = theta * dk * tcen(l) - tapply(l, sd);
            const T v = sx[l] + ((T)1 + c1) * dk + cB * tdinv(l) * r1;
            xcol[k] = (TX)v;
            if (rv) dot += (double)v * (double)(kPre ? rv0 : rv[(size_t)col * ld + k]);
        }
        if (rv) {
            const double sm = group_sum(dot);
            if (threadIdx.x == 0) red.rz[(size_t)col * red.stride + tb.y * gridDim.x + tb.x] = sm;
        }
    }
}

// ------------------------------------------------- two levels a launch ---
// Few columns make the coarse levels latency bound: a launch there costs
// ~4.5 us however small its level.  k_down2 does the down steps of two
// consecutive levels F (N) and M (N/2) in one launch, k_up_chain the up
// steps of up to kChainMax levels: each workgroup recomputes the coarser
// values its tile needs on a larger tile (redundant work on the halo instead
// of more launches).  The arithmetic per node is that of k_down / k_up, so
// the cycle's result is the same bit for bit.

// Grid: (tiles over level-C x, tiles over level-C y, column blocks), C = N/4.
// Level-C tile [K0, K0+kT) x [L0, L0+kT) needs b_M on level-M nodes
// [2 K0 - 3, 2 K1 + 3] (the k_down tile of width MW = 2 kT + 5), which in
// turn needs b_F on the level-F tile of width FW = 2 MW + 5.  Writes x2_F and
// x2_M, and b_M (read again by the up step of level M) on the nodes the tile
// owns, and b_C on the level-C tile.
template <typename T, class Op, int kT, int NT>
__global__ __launch_bounds__(NT) void k_down2(Op opF_, Op opM_, const T* __restrict__ bF, T* __restrict__ xF,
                                               int ldF, T* __restrict__ bM, T* __restrict__ xM, int ldM,
                                               T* __restrict__ bC, int ldC, int dirichlet,
                                               const int* __restrict__ act, ChebCoef cc, int nc, int cb) {
    constexpr int MW = 2 * kT + 5, FW = 2 * MW + 5, NM = MW * MW, NF = FW * FW;
    constexpr bool NE = kNorthEast<Op>;
    __shared__ T fb[NF], fx[NF], fr[NF];
    __shared__ T fc[NE ? NF : 1], fe[NF], fn[NF], fdv[NF], fg[NE ? NF : 1];
    __shared__ T mb[NM], mx[NM], mr[NM];
    __shared__ T mc[NE ? NM : 1], me[NM], mn[NM], mdv[NM], mg[NE ? NM : 1];
    const TileStencil<T> tsF{fc, fe, fn, fg, fdv}, tsM{mc, me, mn, mg, mdv};
    const int Nf = opF_.N, Nf1 = Nf + 1, Nm = Nf / 2, Nm1 = Nm + 1, Nc = Nm / 2, Nc1 = Nc + 1;
    const int3 tb = xcd_tile();
    const int K0 = tb.x * kT, L0 = tb.y * kT;
    const int K1 = min(K0 + kT - 1, Nc), L1 = min(L0 + kT - 1, Nc);
    const int mox = 2 * K0 - 3, moy = 2 * L0 - 3;  // level-M coordinates of local (0, 0)
    const int fox = 2 * mox - 3, foy = 2 * moy - 3;  // level-F coordinates of local (0, 0)
    // owned nodes: level M [2 K0, 2 K1 + 1], level F [2 i0, 2 i1 + 1] of those
    const int mi0 = 2 * K0, mj0 = 2 * L0, mi1 = min(2 * K1 + 1, Nm), mj1 = min(2 * L1 + 1, Nm);
    const int fi0 = 2 * mi0, fj0 = 2 * mj0, fi1 = min(2 * mi1 + 1, Nf), fj1 = min(2 * mj1 + 1, Nf);
    const T inv_theta = (T)cc.inv_theta, cA = (T)cc.cA, cB = (T)cc.cB;
    constexpr int E = (NF + NT - 1) / NT;
    const void* staged = nullptr;
    const int c_end = min(nc, (tb.z + 1) * cb);
    for (int col = tb.z * cb; col < c_end; ++col) {
        // no kernel of the launch writes act (the convergence test runs on the finest level)
        if (act && !act[col]) continue;
        const auto& opF = opF_.at(col);
        const auto& opM = opM_.at(col);
        const T* bcol = bF + (size_t)col * ldF;
        T vb[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = threadIdx.x + NT * e;
            const int i = fox + t % FW, j = foy + t / FW;
            vb[e] = (t < NF && i >= 0 && i <= Nf && j >= 0 && j <= Nf) ? bcol[j * Nf1 + i] : (T)0;
        }
        lds_barrier();  // the previous column's LDS reads are done
        if (instance_key(opF) != staged) {
            stage_stencil<FW, NT>(opF, tsF, fox, foy);
            stage_stencil<MW, NT>(opM, tsM, mox, moy);
            staged = instance_key(opF);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int t = threadIdx.x + NT * e;
            if (t < NF) fb[t] = vb[e];
        }
        lds_barrier();
        // level F: d0 = D^-1 b / theta; x2 = cA d0 + cB D^-1 (b - A d0) on
        // local [1, FW-1)^2 (owned nodes to global); residual on [2, FW-2)^2
        for (int t = threadIdx.x; t < NF; t += blockDim.x) fr[t] = fdv[t] * fb[t] * inv_theta;
        lds_barrier();
        {
            T* xcol = xF + (size_t)col * ldF;
            constexpr int W = FW - 2;
            for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
                const int il = 1 + t % W, jl = 1 + t / W, l = jl * FW + il;
                const T v = cA * fr[l] + cB * fdv[l] * (fb[l] - tile_apply<NE>(tsF, FW, l, fr));
                fx[l] = v;
                const int i = fox + il, j = foy + jl;
                if (i >= fi0 && i <= fi1 && j >= fj0 && j <= fj1) xcol[j * Nf1 + i] = v;
            }
        }
        lds_barrier();
        {
            constexpr int W = FW - 4;
            for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
                const int l = (2 + t / W) * FW + 2 + t % W;
                const T v = fb[l] - tile_apply<NE>(tsF, FW, l, fx);
                fr[l] = fdv[l] != (T)0 ? v : (T)0;
            }
        }
        lds_barrier();
        // P^T onto the whole level-M tile: b_M, zero off the mesh and on
        // Dirichlet rows; owned nodes to global
        {
            T* bcol2 = bM + (size_t)col * ldM;
            auto res = [&](int i, int j) { return fr[(j - foy) * FW + (i - fox)]; };
            for (int t = threadIdx.x; t < NM; t += blockDim.x) {
                const int I = mox + t % MW, J = moy + t / MW;
                T v = 0;
                if (I >= 0 && I <= Nm && J >= 0 && J <= Nm && !(dirichlet && (J == 0 || J == Nm))) {
                    const int i = 2 * I, j = 2 * J;
                    T sm = 0;
                    if (i > 0) sm += res(i - 1, j);
                    if (i < Nf) sm += res(i + 1, j);
                    if (j > 0) sm += res(i, j - 1);
                    if (j < Nf) sm += res(i, j + 1);
                    if (i < Nf && j < Nf) sm += res(i + 1, j + 1);
                    if (i > 0 && j > 0) sm += res(i - 1, j - 1);
                    v = res(i, j) + (T)0.5 * sm;
                }
                if (I >= mi0 && I <= mi1 && J >= mj0 && J <= mj1) bcol2[J * Nm1 + I] = v;
                mb[t] = v;
            }
        }
        lds_barrier();
        // level M: the same three steps on the level-M tile
        for (int t = threadIdx.x; t < NM; t += blockDim.x) mr[t] = mdv[t] * mb[t] * inv_theta;
        lds_barrier();
        {
            T* xcol = xM + (size_t)col * ldM;
            constexpr int W = MW - 2;
            for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
                const int il = 1 + t % W, jl = 1 + t / W, l = jl * MW + il;
                const T v = cA * mr[l] + cB * mdv[l] * (mb[l] - tile_apply<NE>(tsM, MW, l, mr));
                mx[l] = v;
                const int I = mox + il, J = moy + jl;
                if (I >= mi0 && I <= mi1 && J >= mj0 && J <= mj1) xcol[J * Nm1 + I] = v;
            }
        }
        lds_barrier();
        {
            constexpr int W = MW - 4;
            for (int t = threadIdx.x; t < W * W; t += blockDim.x) {
                const int l = (2 + t / W) * MW + 2 + t % W;
                const T v = mb[l] - tile_apply<NE>(tsM, MW, l, mx);
                mr[l] = mdv[l] != (T)0 ? v : (T)0;
            }
        }
        lds_barrier();
        // P^T onto the level-C tile
        T* bccol = bC + (size_t)col * ldC;
        const int cw = K1 - K0 + 1, ch = L1 - L0 + 1;
        auto res = [&](int I, int J) { return mr[(J - moy) * MW + (I - mox)]; };
        for (int t = threadIdx.x; t < cw * ch; t += blockDim.x) {
            const int K = K0 + t % cw, L = L0 + t / cw;
            T v = 0;
            if (!(dirichlet && (L == 0 || L == Nc))) {
                const int I = 2 * K, J = 2 * L;
                T sm = 0;
                if (I > 0) sm += res(I - 1, J);
                if (I < Nm) sm += res(I + 1, J);
                if (J > 0) sm += res(I, J - 1);
                if (J < Nm) sm += res(I, J + 1);
                if (I < Nm && J < Nm) sm += res(I + 1, J + 1);
                if (I > 0 && J > 0) sm += res(I - 1, J - 1);
                v = res(I, J) + (T)0.5 * sm;
            }
            bccol[L * Nc1 + K] = v;
        }
    }
}

// Up steps of NL consecutive levels 0 (finest of the chain) .. NL-1 in one
// launch.  Grid: (tiles over level-0 x, tiles over level-0 y, column blocks).
// Level 0 is the k_up tile: the output tile O of kTF x kTF nodes at local
// [2, kTF+2) of a tile of width W_0 = kTF + 4 whose every node forms
// x2 + P x_1.  The level-(k+1) values that prolongation reads are the nodes
// [floor(o_k / 2), ceil((o_k + W_k - 1) / 2)] (o_k: the tile's origin), at
// most (W_k + 1) / 2 + 1 of them per side; they are the output region of the
// level-(k+1) up step on a tile two nodes wider on each side, so
// o_{k+1} = floor(o_k / 2) - 2 and W_{k+1} = (W_k + 1) / 2 + 5.  The widths
// settle at 11, so the redundant work per level stays bounded (kTF = 16:
// 20, 15, 13, 12, 11, ...); each level still adds its passes to the
// workgroup's latency.  Every input (b and x2 of each level,
// the level-NL correction x_C, the operator rows) is loaded at the start; the
// levels then run coarse to fine in LDS.  Writes x of level 0 on O only (the
// coarser x are used by nothing else).
template <int kTF>
constexpr int chain_width(int k) {
    int w = kTF + 4;
    for (int i = 0; i < k; ++i) w = (w + 1) / 2 + 5;
    return w;
}
template <int kTF>
constexpr int chain_offset(int k) {
    int s = 0;
    for (int i = 0; i < k; ++i) s += chain_width<kTF>(i) * chain_width<kTF>(i);
    return s;
}
constexpr int kChainMax = kChainLen;  // levels a chain may hold

template <typename T, class Op>
struct ChainArgs {
    Op op[kChainMax];
    const T* b[kChainMax];
    const T* x2[kChainMax];
    int ld[kChainMax];
    T* x;         // level-0 output
    const T* xc;  // level-NL correction (from the level below the chain)
    int ldc;
};

// Row of node (i, j) in the tile-stencil form (zero off the mesh), same
// arithmetic as stage_stencil.
template <typename T>
struct TileRow {
    T c, e, n, g, dv;
};
// The loads are issued without a branch, at the node clamped into the mesh
// (chain_load zeroes the row off the mesh): a load inside a branch makes the
// wave wait for it, and with it for every load issued before.
template <typename T>
__device__ inline TileRow<T> tile_row(const OpA<T>& op, int i, int j) {
    const int N = op.N, N1 = N + 1, k = clamp_node(j, N) * N1 + clamp_node(i, N);
    return TileRow<T>{(T)0, -op.wE[k], -op.wN[k], (T)0, op.dinv[k]};  // diagonal: tile_center
}
template <typename T, class OpK>
__device__ inline TileRow<T> tile_row(const OpK& op, int i, int j) {
    const int N = op.N;
    const KARow<T>& r = op.rows[ka_class(clamp_node(i, N), clamp_node(j, N), N)];
    return TileRow<T>{r.c, r.e, r.n, r.ne, r.dinv};
}

// Level k of the chain (then k - 1, ..., 0): x2 + P x_{k+1} (except on the
// coarsest level, whose P x_C came with the loads), d0, then x in place
// (level 0: to global on O).
template <typename T, class Op, int kTF, int NL, int k>
__device__ inline void chain_step(const ChainArgs<T, Op>& a, const int* ox, const int* oy, T* sx, T* sd,
                                  const T* sb, const TileStencil<T>& ts, int dirichlet, const ChebCoef& cc,
                                  int i0, int i1, int j0, int j1, int col) {
    constexpr int W = chain_width<kTF>(k), off = chain_offset<kTF>(k), NN = W * W;
    constexpr bool NE = kNorthEast<Op>;
    const TileStencil<T> st{NE ? ts.c + off : ts.c, ts.e + off, ts.n + off, NE ? ts.g + off : ts.g, ts.dv + off};
    T* x = sx + off;
    T* d = sd + off;
    const T* b = sb + off;
    const T inv_theta = (T)cc.inv_theta, theta = (T)cc.theta, cB = (T)cc.cB, c1 = (T)cc.c1;
    if constexpr (k < NL - 1) {
        constexpr int W1 = chain_width<kTF>(k + 1), off1 = chain_offset<kTF>(k + 1);
        const T* x1 = sx + off1;
        const int N = a.op[k].N, ox1 = ox[k + 1], oy1 = oy[k + 1];
        for (int t = threadIdx.x; t < NN; t += blockDim.x) {
            const int i = ox[k] + t % W, j = oy[k] + t / W;
            if (i >= 0 && i <= N && j >= 0 && j <= N && !(dirichlet && (j == 0 || j == N))) {
                const int I = i >> 1, J = j >> 1;
                const T p0 = x1[(J - oy1) * W1 + (I - ox1)];
                x[t] += ((i | j) & 1) ? (T)0.5 * (p0 + x1[(J + (j & 1) - oy1) * W1 + (I + (i & 1) - ox1)]) : p0;
            }
        }
        lds_barrier();
    }
    {
        constexpr int Wi = W - 2;
        for (int t = threadIdx.x; t < Wi * Wi; t += blockDim.x) {
            const int l = (1 + t / Wi) * W + 1 + t % Wi;
            d[l] = st.dv[l] * (b[l] - tile_apply<NE>(st, W, l, x)) * inv_theta;
        }
    }
    lds_barrier();
    if constexpr (k > 0) {
        // x on [2, W-2)^2 in place of x2 + P x (each node reads only its own entry)
        constexpr int Wi = W - 4;
        for (int t = threadIdx.x; t < Wi * Wi; t += blockDim.x) {
            const int l = (2 + t / Wi) * W + 2 + t % Wi;
            const T dk = d[l];
            const T r1 = theta * dk * tile_center<NE>(st, W, l) - tile_apply<NE>(st, W, l, d);
            x[l] = x[l] + ((T)1 + c1) * dk + cB * st.dv[l] * r1;
        }
        lds_barrier();
        chain_step<T, Op, kTF, NL, k - 1>(a, ox, oy, sx, sd, sb, ts, dirichlet, cc, i0, i1, j0, j1, col);
    } else {
        const int N1 = a.op[0].N + 1;
        T* xcol = a.x + (size_t)col * a.ld[0];
        const int w = i1 - i0 + 1, h = j1 - j0 + 1;
        for (int t = threadIdx.x; t < w * h; t += blockDim.x) {
            const int i = i0 + t % w, j = j0 + t / w;
            const int l = (j - oy[0]) * W + (i - ox[0]);
            const T dk = d[l];
            const T r1 = theta * dk * tile_center<NE>(st, W, l) - tile_apply<NE>(st, W, l, d);
            xcol[j * N1 + i] = x[l] + ((T)1 + c1) * dk + cB * st.dv[l] * r1;
        }
    }
}

// Loads of level k of the chain (then k + 1, ...), kept in registers until
// every level's loads are issued, then stored to LDS: b, x2 (plus P x_C on
// the coarsest level) and, when stage is set, the operator rows.
template <typename T, class Op, int kTF, int NL, int NT, int k>
__device__ inline void chain_load(const ChainArgs<T, Op>& a, const int* ox, const int* oy, int dirichlet, int col,
                                  bool stage, T* sx, T* sb, const TileStencil<T>& ts) {
    constexpr int W = chain_width<kTF>(k), off = chain_offset<kTF>(k), NN = W * W, E = (NN + NT - 1) / NT;
    constexpr bool NE = kNorthEast<Op>;
    const Op& op = a.op[k];
    const int N = op.N;
    // every load at a node clamped into the mesh, without a branch (a load
    // inside a branch waits there, and with it every load issued before it);
    // off-mesh and off-tile slots are dropped at the LDS stores
    T vb[E], vx[E], pc0[E], pc1[E];
    TileRow<T> vr[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = threadIdx.x + NT * e;
        const int i = ox[k] + t % W, j = oy[k] + t / W;
        const size_t g = (size_t)col * a.ld[k] + (size_t)clamp_node(j, N) * (N + 1) + clamp_node(i, N);
        vb[e] = a.b[k][g];
        vx[e] = a.x2[k][g];
        if constexpr (k == NL - 1) {
            // P x_C operands: the coarse node (i/2, j/2) and the far coarse
            // end of the fine edge through (i, j)
            const int Nc = N / 2, ic = clamp_node(i, N), jc = clamp_node(j, N), I = ic >> 1, J = jc >> 1;
            const T* xcc = a.xc + (size_t)col * a.ldc;
            pc0[e] = xcc[J * (Nc + 1) + I];
            pc1[e] = xcc[min(J + (jc & 1), Nc) * (Nc + 1) + min(I + (ic & 1), Nc)];
        }
        // rows loaded whether or not this column stages them (few-column
        // cycles: the next columns of a workgroup find them in cache)
        vr[e] = tile_row<T>(op.at(col), i, j);
    }
    if constexpr (k + 1 < NL) chain_load<T, Op, kTF, NL, NT, k + 1>(a, ox, oy, dirichlet, col, stage, sx, sb, ts);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = threadIdx.x + NT * e;
        if (t < NN) {
            const int i = ox[k] + t % W, j = oy[k] + t / W;
            const bool in = i >= 0 && i <= N && j >= 0 && j <= N;
            const bool fr = in && !(dirichlet && (j == 0 || j == N));
            T v = fr ? vx[e] : (T)0;
            // x2 + P x_C on the coarsest level of the chain: the coarse node
            // when i and j are even, else the mean of the edge's two ends
            if constexpr (k == NL - 1)
                if (fr) v += ((i | j) & 1) ? (T)0.5 * (pc0[e] + pc1[e]) : pc0[e];
            sb[off + t] = in ? vb[e] : (T)0;
            sx[off + t] = v;
            if (stage) {
                const TileRow<T> r = in ? vr[e] : TileRow<T>{};
                if constexpr (NE) ts.c[off + t] = r.c;
                ts.e[off + t] = r.e;
                ts.n[off + t] = r.n;
                if constexpr (NE) ts.g[off + t] = r.g;
                ts.dv[off + t] = r.dv;
            }
        }
    }
}

template <typename T, class Op, int kTF, int NL, int NT>
__global__ __launch_bounds__(NT) void k_up_chain(ChainArgs<T, Op> a, int dirichlet, const int* __restrict__ act,
                                                 ChebCoef cc, int nc, int cb) {
    static_assert(kTF % 2 == 0 && NL >= 2 && NL <= kChainMax, "chain shape");
    constexpr int NA = chain_offset<kTF>(NL);  // nodes of all the chain's tiles
    constexpr bool NE = kNorthEast<Op>;
    __shared__ T sx[NA], sd[NA], sb[NA];
    __shared__ T tc[NE ? NA : 1], te[NA], tn[NA], tdv[NA], tg[NE ? NA : 1];
    const TileStencil<T> ts{tc, te, tn, tg, tdv};
    const int3 tb = xcd_tile();
    const int i0 = tb.x * kTF, j0 = tb.y * kTF;
    const int i1 = min(i0 + kTF - 1, a.op[0].N), j1 = min(j0 + kTF - 1, a.op[0].N);
    int ox[NL], oy[NL];
    ox[0] = i0 - 2;
    oy[0] = j0 - 2;
#pragma unroll
    for (int k = 1; k < NL; ++k) {
        ox[k] = (ox[k - 1] >> 1) - 2;  // floor(o / 2) - 2
        oy[k] = (oy[k - 1] >> 1) - 2;
    }
    const void* staged = nullptr;
    const int c_end = min(nc, (tb.z + 1) * cb);
    for (int col = tb.z * cb; col < c_end; ++col) {
        // no kernel of the launch writes act (the convergence test runs on the finest level)
        if (act && !act[col]) continue;
        const void* key = instance_key(a.op[0].at(col));
        lds_barrier();  // the previous column's LDS reads are done
        chain_load<T, Op, kTF, NL, NT, 0>(a, ox, oy, dirichlet, col, key != staged, sx, sb, ts);
        staged = key;
        lds_barrier();
        chain_step<T, Op, kTF, NL, NL - 1>(a, ox, oy, sx, sd, sb, ts, dirichlet, cc, i0, i1, j0, j1, col);
    }
}

// -------------------------------------------------------------- bottom ---
// All levels with N_l <= kBottomN (up to four: 64, 32, 16, 8) for one column in
// one workgroup of 1024 threads.  The bottom computes in FP32 whatever the
// solve's precision: it is the coarse correction of a preconditioner, so its
// rounding changes the preconditioner slightly but no result (the PCG and the
// refinement test residuals of the solve's own precision), and FP32 halves the
// LDS a level takes, so that the level-64 sweeps run here instead of in two
// more launches per V-cycle.  b and x are global level-Lb vectors of the
// solve's precision TV.
struct BottomArgs {
    int nlev;                           // levels handled here (the last is the coarsest)
    int N[kBottomLevels];
    const float* wE[kBottomLevels];     // state operator coefficients (unused for the prior)
    const float* wN[kBottomLevels];
    const float* dinv[kBottomLevels];
    const float* cinv;                  // dense inverse of the coarsest level
    int nc;                             // its size
    KARow<float> ka[kBottomLevels][9];  // prior operator rows of each level
    // stacked instances (cpi = 0: one instance): column c belongs to instance
    // c / cpi, whose state coefficients of level l start cs[l] elements further,
    // whose coarse inverse starts cinv_stride further and whose prior rows of
    // level l are karows[l][9 inst .. 9 inst + 8]
    int cpi;
    long long cs[kBottomLevels];
    long long cinv_stride;
    const KARow<float>* karows[kBottomLevels];
};

// Bottom levels in LDS with a ring of zeros around each level (padded width
// P_l = N_l + 3): the stencil applies without boundary branches (an absent
// neighbour has a zero coupling and a zero value), and Dirichlet rows are
// masked by their zero inverse diagonal.  Sizes for a top level of at most
// TOP (a power of two, at least 8).
template <int TOP>
constexpr int bottom_padded() {
    int s = 0;
    for (int n = TOP; n >= 8; n /= 2) s += (n + 3) * (n + 3);
    return s;
}
template <int TOP>
constexpr int bottom_nodes() {
    int s = 0;
    for (int n = TOP; n >= 8; n /= 2) s += (n + 1) * (n + 1);
    return s;
}
// node slots of a thread on level l (a level of N has (N + 1)^2 nodes)
template <int TOP>
constexpr int bottom_slots(int l) {
    return l < kBottomLevels && (TOP >> l) >= 8 ? (((TOP >> l) + 1) * ((TOP >> l) + 1) + 1023) / 1024 : 0;
}

// q / d for 0 <= q < 2^22 and d >= 1 by a float reciprocal: (q + 1/2) / d lies
// at least 1 / (2 d) from an integer and the float product errs by less than
// 2^-23 (q / d) < 1 / (2 d), so the truncation is exact (integer division is a
// long instruction sequence on the vector ALU).
__device__ inline int small_div(int q, float inv_d) { return (int)(((float)q + 0.5f) * inv_d); }

// x_top = V-cycle(b_top) for every column (blockIdx.x = column).  When rv is
// given (the bottom is the whole hierarchy), sum_k rv_k x_k is written as the
// single partial of r^T z.  Thread t holds the nodes q = t + 1024 s of each
// level (padded position and (i, j) per slot).
template <typename TV, int KIND, int TOP>
__global__ __launch_bounds__(1024) void k_bottom(BottomArgs a, const TV* __restrict__ bg, TV* __restrict__ xg,
                                                 int ld, int* __restrict__ act, ChebCoef cc,
                                                 const TV* __restrict__ rv, PcgRed red,
                                                 ColState* __restrict__ st, int check) {
    constexpr bool PRIOR = KIND == kOpPrior;
    constexpr int PN = bottom_padded<TOP>(), NT = 1024, LV = kBottomLevels, MS = bottom_slots<TOP>(0);
    const int col = blockIdx.x;
    if (act && !act[col]) return;
    // the convergence test's partials load together with the level data
    // below; the test itself follows the loads
    const double rr_share = check ? partial_share(red.rr, col, red.stride, red.nvec) : 0.0;
    __shared__ float sb[PN], sx[PN], sw[PN];  // right-hand side, iterate, work vector
    __shared__ float te[PRIOR ? 1 : PN], tn[PRIOR ? 1 : PN], tdv[PRIOR ? 1 : PN];  // -wE, -wN, 1/diag
    __shared__ KARow<float> rows[PRIOR ? LV * 9 : 1];
    const int inst = a.cpi ? col / a.cpi : 0;
    const int nlev = a.nlev, L = nlev - 1;  // L: the coarsest level, solved with its dense inverse
    int Nl[LV], Pl[LV], po[LV], uo[LV + 1];
    float inv_n1[LV];
    {
        int p = 0, u = 0;
#pragma unroll
        for (int l = 0; l < LV; ++l) {
            const int n = l < nlev ? a.N[l] : 0;
            Nl[l] = n;
            Pl[l] = n + 3;
            po[l] = p;
            uo[l] = u;
            inv_n1[l] = 1.0f / (float)(n + 1);
            if (l < nlev) {
                p += (n + 3) * (n + 3);
                u += (n + 1) * (n + 1);
            }
        }
        uo[LV] = u;
    }
    const int n0 = uo[1];
    // ---- loads: b, the state coefficients (unpadded concatenation of the
    // levels), this thread's part of the dense coarse inverse
    constexpr int EB = (bottom_nodes<TOP>() + NT - 1) / NT, S = 12, kCU = 8;
    float vb[EB], vE[EB], vN[EB], vD[EB];
    int vp[EB], vl[EB], vij[EB];
#pragma unroll
    for (int e = 0; e < EB; ++e) {
        const int t = threadIdx.x + NT * e;
        const int l = (t >= uo[1]) + (t >= uo[2]) + (t >= uo[3]);
        const bool in = t < uo[LV];
        const int q = t - (l == 0 ? 0 : (l == 1 ? uo[1] : (l == 2 ? uo[2] : uo[3])));
        const int N1 = (l == 0 ? Nl[0] : (l == 1 ? Nl[1] : (l == 2 ? Nl[2] : Nl[3]))) + 1;
        const int j = small_div(q, l == 0 ? inv_n1[0] : (l == 1 ? inv_n1[1] : (l == 2 ? inv_n1[2] : inv_n1[3])));
        const int P = N1 + 2, i = q - j * N1;
        vl[e] = l;
        vij[e] = i | (j << 16);
        vp[e] = in ? (l == 0 ? po[0] : (l == 1 ? po[1] : (l == 2 ? po[2] : po[3]))) + (j + 1) * P + i + 1 : -1;
        vb[e] = t < n0 ? (float)bg[(size_t)col * ld + t] : 0.0f;
        vE[e] = vN[e] = vD[e] = 0.0f;
        if constexpr (!PRIOR) {
            const long long cs = l == 0 ? a.cs[0] : (l == 1 ? a.cs[1] : (l == 2 ? a.cs[2] : a.cs[3]));
            const long long at = (a.cpi ? inst * cs : 0) + q;
            const float* pE = l == 0 ? a.wE[0] : (l == 1 ? a.wE[1] : (l == 2 ? a.wE[2] : a.wE[3]));
            const float* pN = l == 0 ? a.wN[0] : (l == 1 ? a.wN[1] : (l == 2 ? a.wN[2] : a.wN[3]));
            const float* pD = l == 0 ? a.dinv[0] : (l == 1 ? a.dinv[1] : (l == 2 ? a.dinv[2] : a.dinv[3]));
            vE[e] = in ? pE[at] : 0.0f;
            vN[e] = in ? pN[at] : 0.0f;
            vD[e] = in ? pD[at] : 0.0f;
        }
    }
    const float* ci = a.cinv + (a.cpi ? inst * a.cinv_stride : 0);
    const int cr = threadIdx.x / S, cpart = threadIdx.x % S;
    float cv[kCU];
#pragma unroll
    for (int u = 0; u < kCU; ++u) {
        const int c = cpart + u * S;
        cv[u] = (cr < a.nc && c < a.nc) ? ci[cr * a.nc + c] : 0.0f;
    }
    if (check && column_done_share(rr_share, red, col, st, act, true)) return;
    // ---- per-thread slots: padded position (-1 past the level) and (i, j)
    int sp[LV][MS], sij[LV][MS];
#pragma unroll
    for (int l = 0; l < LV; ++l)
#pragma unroll
        for (int s = 0; s < MS; ++s) {
            if (s >= bottom_slots<TOP>(l)) break;
            const int q = threadIdx.x + NT * s;
            const int N1 = Nl[l] + 1;
            const bool in = l < nlev && q < N1 * N1;
            const int jq = small_div(q, inv_n1[l]);
            const int i = in ? q - jq * N1 : 0, j = in ? jq : 0;
            sp[l][s] = in ? po[l] + (j + 1) * Pl[l] + i + 1 : -1;
            sij[l][s] = i | (j << 16);
        }
    // ---- LDS: zeros everywhere (the rings stay zero), then the interiors
    if constexpr (PRIOR)
        for (int t = threadIdx.x; t < nlev * 9; t += NT)
            rows[t] = a.cpi ? a.karows[t / 9][9 * inst + t % 9] : a.ka[t / 9][t % 9];
    for (int q = threadIdx.x; q < PN; q += NT) {
        sb[q] = sx[q] = sw[q] = 0.0f;
        if constexpr (!PRIOR) te[q] = tn[q] = tdv[q] = 0.0f;
    }
    lds_barrier();
    const float inv_theta = (float)cc.inv_theta, theta = (float)cc.theta, cA = (float)cc.cA, cB = (float)cc.cB,
                c1 = (float)cc.c1;
#pragma unroll
    for (int e = 0; e < EB; ++e) {
        const int p = vp[e];
        if (p < 0) continue;
        if constexpr (!PRIOR) {
            te[p] = -vE[e];
            tn[p] = -vN[e];
            tdv[p] = vD[e];
        } else {
            const int l = vl[e];
            const int N = l == 0 ? Nl[0] : (l == 1 ? Nl[1] : (l == 2 ? Nl[2] : Nl[3]));
            vD[e] = rows[9 * l + ka_class(vij[e] & 0xffff, vij[e] >> 16, N)].dinv;
        }
        if (threadIdx.x + NT * e < n0) {
            sb[p] = vb[e];
            sw[p] = vD[e] * vb[e] * inv_theta;  // d0 of the first smoothing step
        }
    }
    lds_barrier();
    // (A x)_p at padded position p of level l (node ij), with the diagonal and
    // 1/diagonal of the row
    auto apply = [&](int l, int p, int ij, const float* x, float& diag, float& dv) -> float {
        const int P = Pl[l];
        if constexpr (!PRIOR) {
            const float e0 = te[p], e1 = te[p - 1], m0 = tn[p], m1 = tn[p - P];
            diag = -(e0 + e1 + m0 + m1);
            dv = tdv[p];
            return diag * x[p] + e0 * x[p + 1] + e1 * x[p - 1] + m0 * x[p + P] + m1 * x[p - P];
        } else {
            const KARow<float>& r = rows[9 * l + ka_class(ij & 0xffff, ij >> 16, Nl[l])];
            diag = r.c;
            dv = r.dinv;
            return r.c * x[p] + r.e * x[p + 1] + r.w * x[p - 1] + r.n * x[p + P] + r.s * x[p - P] +
                   r.ne * x[p + P + 1] + r.sw * x[p - P - 1];
        }
    };
    auto inv_diag = [&](int l, int p, int ij) -> float {
        if constexpr (!PRIOR)
            return tdv[p];
        else
            return rows[9 * l + ka_class(ij & 0xffff, ij >> 16, Nl[l])].dinv;
    };
    // ---- down
#pragma unroll
    for (int l = 0; l < LV - 1; ++l) {
        if (l >= L) break;
        const int P = Pl[l];
        // x2 = cA d0 + cB D^-1 (b - A d0), d0 in sw
#pragma unroll
        for (int s = 0; s < bottom_slots<TOP>(l); ++s) {
            const int p = sp[l][s];
            if (p < 0) continue;
            float dg, dv;
            const float ad = apply(l, p, sij[l][s], sw, dg, dv);
            sx[p] = cA * sw[p] + cB * dv * (sb[p] - ad);
        }
        lds_barrier();
        // residual b - A x2 on the free nodes, into sw
#pragma unroll
        for (int s = 0; s < bottom_slots<TOP>(l); ++s) {
            const int p = sp[l][s];
            if (p < 0) continue;
            float dg, dv;
            const float v = sb[p] - apply(l, p, sij[l][s], sx, dg, dv);
            sw[p] = dv != 0.0f ? v : 0.0f;
        }
        lds_barrier();
        // restriction P^T to level l + 1, and its first smoothing correction d0
#pragma unroll
        for (int s = 0; s < bottom_slots<TOP>(l + 1); ++s) {
            const int pc = sp[l + 1][s];
            if (pc < 0) continue;
            const int I = sij[l + 1][s] & 0xffff, J = sij[l + 1][s] >> 16;
            const int f = po[l] + (2 * J + 1) * P + 2 * I + 1;
            const float dvc = inv_diag(l + 1, pc, sij[l + 1][s]);
            float v = 0.0f;
            if (dvc != 0.0f)
                v = sw[f] + 0.5f * (sw[f - 1] + sw[f + 1] + sw[f - P] + sw[f + P] + sw[f + P + 1] + sw[f - P - 1]);
            sb[pc] = v;
            sw[pc] = dvc * v * inv_theta;
        }
        lds_barrier();
    }
    // ---- coarsest: dense inverse, S threads per row (entries prefetched in cv)
    {
        const int N1 = (L == 0 ? Nl[0] : (L == 1 ? Nl[1] : (L == 2 ? Nl[2] : Nl[3]))) + 1;
        const int P = N1 + 2, o = L == 0 ? po[0] : (L == 1 ? po[1] : (L == 2 ? po[2] : po[3]));
        // the work vector is free here (the dense solve reads b only; the ring
        // entries it overwrites meet zero couplings only): 12 * 81 <= PN
        float* tmp = sw;
        const float inv_c = 1.0f / (float)N1;
        if (cr < a.nc) {
            float s = 0.0f;
            // entry c = cpart + u S at (c mod N1, c / N1), stepped without dividing
            int jc = small_div(cpart, inv_c), ic = cpart - jc * N1;
#pragma unroll
            for (int u = 0; u < kCU; ++u) {
                const int c = cpart + u * S;
                if (c < a.nc) s += cv[u] * sb[o + (jc + 1) * P + ic + 1];
                ic += S;
                while (ic >= N1) {
                    ic -= N1;
                    ++jc;
                }
            }
            tmp[threadIdx.x] = s;
        }
        lds_barrier();
        for (int r = threadIdx.x; r < a.nc; r += NT) {
            float s = 0.0f;
            for (int part = 0; part < S; ++part) s += tmp[r * S + part];
            const int jr = small_div(r, inv_c);
            sx[o + (jr + 1) * P + r - jr * N1 + 1] = s;
        }
        lds_barrier();
    }
    // ---- up
#pragma unroll
    for (int l = LV - 2; l >= 0; --l) {
        if (l >= L) continue;
        const int Pc = Pl[l + 1];
        // x += P x_coarse on the free nodes
#pragma unroll
        for (int s = 0; s < bottom_slots<TOP>(l); ++s) {
            const int p = sp[l][s];
            if (p < 0) continue;
            const int ij = sij[l][s], i = ij & 0xffff, j = ij >> 16;
            if (inv_diag(l, p, ij) == 0.0f) continue;
            const int I = i >> 1, J = j >> 1;
            const int ca0 = po[l + 1] + (J + 1) * Pc + I + 1;
            const int ca1 = po[l + 1] + (J + 1 + (j & 1)) * Pc + I + 1 + (i & 1);
            sx[p] += ((i | j) & 1) ? 0.5f * (sx[ca0] + sx[ca1]) : sx[ca0];
        }
        lds_barrier();
        // d0 = D^-1 (b - A x) / theta
#pragma unroll
        for (int s = 0; s < bottom_slots<TOP>(l); ++s) {
            const int p = sp[l][s];
            if (p < 0) continue;
            float dg, dv;
            const float ax = apply(l, p, sij[l][s], sx, dg, dv);
            sw[p] = dv * (sb[p] - ax) * inv_theta;
        }
        lds_barrier();
        // x += (1 + c1) d0 + cB D^-1 r1 with r1 = theta D d0 - A d0
#pragma unroll
        for (int s = 0; s < bottom_slots<TOP>(l); ++s) {
            const int p = sp[l][s];
            if (p < 0) continue;
            float dg, dv;
            const float ad = apply(l, p, sij[l][s], sw, dg, dv);
            const float dk = sw[p];
            const float r1 = theta * dk * dg - ad;
            sx[p] += (1.0f + c1) * dk + cB * dv * r1;
        }
        lds_barrier();
    }
    double dot = 0.0;
#pragma unroll
    for (int s = 0; s < bottom_slots<TOP>(0); ++s) {
        const int q = threadIdx.x + NT * s;
        const int p = sp[0][s];
        if (p >= 0) {
            const TV v = (TV)sx[p];
            xg[(size_t)col * ld + q] = v;
            if (rv) dot += (double)v * (double)rv[(size_t)col * ld + q];
        }
    }
    if (rv) {
        const double sm = group_sum(dot);
        if (threadIdx.x == 0) red.rz[(size_t)col * red.stride] = sm;
    }
}

// ------------------------------------------------------------------ PCG ---
// Workgroup blockIdx.x covers nodes [chunk x, chunk (x + 1)) of column
// blockIdx.y with vec_threads(per) threads, at most kVecNodes nodes a thread.

// p_new = z + beta p_old with beta = (r^T z) / rz_old (p_new = z on the first
// iteration, FIRST), q = A p_new = A z + beta A p_old, partials of p_new^T q.
// The loads of the r^T z partials and of the thread's nodes (z and p_old at
// the stencil points, the operator rows) are issued before any of them is
// used, so their latencies overlap: all at once where the registers allow,
// else node by node with apply_window() nodes in flight (FP64 rows would spill).
// Node k = j (N + 1) + i is split by a double reciprocal: (k + 1/2) / (N + 1)
// lies at least 1 / (2 (N + 1)) from an integer and the product errs by far
// less, so the truncation is exact.  Workgroup 0 records r^T z for the update
// kernel, which then reads one value instead of the partials.
// The operator form the apply kernel combines with: the state operator as it
// is, the prior operators through their rows staged in LDS.
template <class OpT>
struct ApplyForm {
    using type = OpT;
    static constexpr bool kTable = false;
};
template <typename T>
struct ApplyForm<OpKA<T>> {
    using type = OpKALds<T>;
    static constexpr bool kTable = true;
};
template <typename T>
struct ApplyForm<OpKARef<T>> {
    using type = OpKALds<T>;
    static constexpr bool kTable = true;
};

template <class OpT>
constexpr int apply_window() {
    constexpr size_t b = sizeof(typename OpT::Row) + 2 * sizeof(typename OpT::Nb);  // loaded bytes per node
    return b <= 96 ? kVecNodes : (b <= 128 ? 3 : 2);
}

template <typename T, class Op, bool FIRST>
__global__ __launch_bounds__(1024) void k_pcg_apply(Op op_, const T* __restrict__ z, const T* __restrict__ p_old,
                                                    T* __restrict__ p_new, T* __restrict__ q, int ld,
                                                    const int* __restrict__ act, ColState* __restrict__ st,
                                                    PcgRed red) {
    // node blocks in XCD-aware order: the rows above and below a block's
    // nodes belong to blocks on the same XCD
    const int3 tb = xcd_tile();
    const int col = tb.y, bx = tb.x;
    const auto& op = op_.at(col);  // operator of the instance owning this column
    if (!act[col]) return;
    const int N = op.N, N1 = N + 1, n = N1 * N1;
    const bool need_rz = !FIRST || bx == 0;  // uniform in the workgroup
    double srz = need_rz ? partial_first(red.rz, col, red.stride, red.nrz) : 0.0;
    const double rz_old = FIRST ? 1.0 : st[col].rz;
    const T* zc = z + (size_t)col * ld;
    const T* pc = p_old + (size_t)col * ld;
    const int k0 = bx * red.chunk, k1 = min(n, k0 + red.chunk);
    const double inv_n1 = 1.0 / N1;
    using Form = ApplyForm<std::decay_t<decltype(op)>>;
    using OpT = typename Form::type;
    __shared__ KARow<T> krows[Form::kTable ? 9 : 1];
    OpT sop;
    if constexpr (Form::kTable)
        sop = OpT{N, krows};
    else
        sop = op;
    typename OpT::Row rw[kVecNodes];
    typename OpT::Nb vz[kVecNodes], vp[kVecNodes];
    T zk[kVecNodes], pk[kVecNodes], az[kVecNodes], ap[kVecNodes];
    auto node = [&](int e, int& i, int& j) {
        const int k = k0 + e * (int)blockDim.x + (int)threadIdx.x;
        j = (int)(((double)k + 0.5) * inv_n1);
        i = k - j * N1;
        return k;
    };
    auto load = [&](int e) {
        int i, j;
        const int k = node(e, i, j);
        if (k < k1) {
            rw[e] = sop.row(i, j, k);
            vz[e] = sop.gather(i, j, k, zc);
            if constexpr (!FIRST) vp[e] = sop.gather(i, j, k, pc);
        }
    };
    auto combine = [&](int e) {
        int i, j;
        const int k = node(e, i, j);
        zk[e] = pk[e] = az[e] = ap[e] = 0;
        if (k < k1) {
            const bool fr = sop.is_free(i, j);
            zk[e] = vz[e].c;
            if (fr) az[e] = sop.combine(i, j, rw[e], vz[e]);
            if constexpr (!FIRST) {
                pk[e] = vp[e].c;
                if (fr) ap[e] = sop.combine(i, j, rw[e], vp[e]);
            }
        }
    };
    constexpr int W = apply_window<OpT>();
#pragma unroll
    for (int e = 0; e < W; ++e) load(e);
    if constexpr (Form::kTable) {
        // rows staged after the node loads are issued (waiting for them then
        // waits for nothing those loads would not)
        if (threadIdx.x < 9) krows[threadIdx.x] = ka_row(op, threadIdx.x);
        lds_barrier();
    }
#pragma unroll
    for (int e = W; e < kVecNodes; ++e) {
        combine(e - W);
        __builtin_amdgcn_sched_barrier(0);  // keeps the window: no later load moves above
        load(e);
    }
    if (need_rz) srz = partial_rest(srz, red.rz, col, red.stride, red.nrz);
#pragma unroll
    for (int e = kVecNodes - W; e < kVecNodes; ++e) combine(e);
    T beta = 0;
    if (need_rz) {
        const double rz = share_total(srz);
        if (!FIRST) beta = (T)(rz / rz_old);
        if (bx == 0 && threadIdx.x == 0) st[col].rz_new = rz;
    }
    double dot = 0.0;
#pragma unroll
    for (int e = 0; e < kVecNodes; ++e) {
        const int k = k0 + e * (int)blockDim.x + (int)threadIdx.x;
        if (k < k1) {
            const T pn = FIRST ? zk[e] : zk[e] + beta * pk[e];
            const T v = FIRST ? az[e] : az[e] + beta * ap[e];
            p_new[(size_t)col * ld + k] = pn;
            q[(size_t)col * ld + k] = v;
            dot += (double)pn * (double)v;
        }
    }
    const double sm = group_sum(dot);
    if (threadIdx.x == 0) red.pq[(size_t)col * red.stride + bx] = sm;
}

// alpha = (r^T z) / (p^T q); x += alpha p, r -= alpha q; partials of r^T r.
// Workgroup 0 records rz (the next beta's denominator) and alpha; a column
// with p^T q <= 0 (breakdown) stops.
// Eight waves a SIMD: two 1024-thread workgroups a compute unit, so the ~500
// workgroups of a one-column update at N = 1024 run in one round instead of
// two (the FP64 form then spills four registers; measured 2% faster solves).
template <typename T>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_pcg_update(T* __restrict__ x, T* __restrict__ r,
                                                     const T* __restrict__ p, const T* __restrict__ q,
                                                     int ld, int n, int* __restrict__ act,
                                                     ColState* __restrict__ st, PcgRed red) {
    const int col = blockIdx.y;
    // workgroup 0 clears act[col] on breakdown while the others read it: one
    // decision per workgroup (see k_down)
    if (!__syncthreads_or(act[col])) return;
    double spq = partial_first(red.pq, col, red.stride, red.nvec);
    const double rz = st[col].rz_new;
    const int k0 = blockIdx.x * red.chunk, k1 = min(n, k0 + red.chunk);
    T xk[kVecNodes], rk[kVecNodes], pk[kVecNodes], qk[kVecNodes];
#pragma unroll
    for (int e = 0; e < kVecNodes; ++e) {
        const int k = k0 + e * blockDim.x + threadIdx.x;
        const size_t o = (size_t)col * ld + k;
        xk[e] = rk[e] = pk[e] = qk[e] = 0;
        if (k < k1) {
            xk[e] = x[o];
            rk[e] = r[o];
            pk[e] = p[o];
            qk[e] = q[o];
        }
    }
    spq = partial_rest(spq, red.pq, col, red.stride, red.nvec);
    const double pq = share_total(spq);
    const double alpha = pq > 0.0 ? rz / pq : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ColState& c = st[col];
        c.rz = rz;
        c.pq = pq;
        c.alpha = alpha;
        c.its += 1.0;
        if (!(pq > 0.0)) act[col] = 0;
    }
    double rr = 0.0;
    const T a = (T)alpha;
#pragma unroll
    for (int e = 0; e < kVecNodes; ++e) {
        const int k = k0 + e * blockDim.x + threadIdx.x;
        if (k < k1) {
            const size_t o = (size_t)col * ld + k;
            x[o] = xk[e] + a * pk[e];
            const T rv = rk[e] - a * qk[e];
            r[o] = rv;
            rr += (double)rv * (double)rv;
        }
    }
    const double s = group_sum(rr);
    if (threadIdx.x == 0) red.rr[(size_t)col * red.stride + blockIdx.x] = s;
}

}  // namespace hinv
