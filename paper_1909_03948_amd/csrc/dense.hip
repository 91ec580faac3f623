// Dense kernels: matrix-core tall-skinny products and s x s factorizations
// (s = k + oversampling <= 512), one workgroup per matrix in LDS while it
// fits, blocked or in global memory beyond.
//
// Matrix-core operand layouts (wave64), checked on the device:
//   f64 16x16x4:   A (16 x 4): lane l holds A[l % 16][l / 16]
//                  B (4 x 16): lane l holds B[l / 16][l % 16]
//                  D (16 x 16): lane l, item v holds D[4 v + l / 16][l % 16]
//   bf16 16x16x32 (gfx950): A: lane l holds A[l % 16][8 (l / 16) + e], e = 0..7
//                  B: lane l holds B[8 (l / 16) + e][l % 16]
//                  D: lane l, item v holds D[4 (l / 16) + v][l % 16]
#include <algorithm>
#include <vector>

#include "dense.h"

namespace hinv {

namespace {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));
typedef short s8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

__device__ inline short to_bf16(double x) {
    // round-to-nearest-even of the float value
    const float f = (float)x;
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

// Block products: a workgroup of kBlkWaves waves owns a 128 x 128 block of the
// output; wave w computes its rows [16 w, 16 w + 16) against all 128 columns
// (kBlkTiles matrix-core tiles sharing one operand), so each column of X and
// Y is read by ceil(s / 128) workgroups instead of ceil(s / 16).
constexpr int kBlkWaves = 8, kBlkTiles = 8, kBlk = 128;

// Split-K Gram C = X^T Y: grid.x = output block, grid.y = K chunk (a multiple
// of kGramKC rows).  The block's 128 columns of Y are staged in LDS kGramKC
// rows at a time (double-buffered: the next stage is loaded into registers
// while the matrix cores work on the current one), so the eight waves share
// one read of Y; each wave loads its 16 columns of X for the stage's eight K
// steps at once.  Products are accumulated in K order.
constexpr int kGramKC = 32;   // K rows per LDS stage

// XCD-aware order of the workgroups of a (per x chunks) grid: the hardware
// hands consecutive workgroups to the eight XCDs in turn, so with the plain
// order the `per` output blocks of one K chunk (which read the same rows of
// X and Y) land on different XCDs and each XCD's L2 fetches those rows again.
// Workgroup h is mapped to block b and chunk c such that the blocks of chunk
// c run on one XCD one after another (h = 8 j + x: XCD x, its j-th
// workgroup); the chunks beyond the last multiple of 8 keep the plain order.
// A bijection of [0, per * chunks) onto the (block, chunk) pairs, whatever
// the grid's shape (h is the dispatch order, x fastest).
__device__ inline void xcd_block_chunk(int per, int chunks, int& b, int& c) {
    const int h = blockIdx.x + gridDim.x * blockIdx.y;
    const int full = chunks & ~7;
    if (h < full * per) {
        const int x = h & 7, j = h >> 3;
        b = j % per;
        c = (j / per) * 8 + x;
    } else {
        const int t = h - full * per;
        b = t % per;
        c = full + t / per;
    }
}
constexpr int kGramLd = 144;  // LDS row stride (doubles): rows k and k + 1 fall in different bank halves
__global__ __launch_bounds__(512) void k_gram_f64(int n, int s1, int s2, int chunk,
                                                  const double* __restrict__ X, int ldx,
                                                  const double* __restrict__ Y, int ldy,
                                                  double* __restrict__ part) {
    __shared__ double ys[2][kGramKC * kGramLd];
    const int blocks_i = (s1 + kBlk - 1) / kBlk;
    int blk, split;
    xcd_block_chunk(gridDim.x, gridDim.y, blk, split);
    const int bi = blk % blocks_i, bj = blk / blocks_i;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = bi * kBlk + wave * 16 + (lane & 15);
    const bool rows_on = bi * kBlk + wave * 16 < s1;  // this wave has output rows (all waves stage Y)
    const int kr = lane >> 4;
    const int k_begin = split * chunk;
    const int k_end = min(n, k_begin + chunk);
    const double* xc = X + (size_t)(i < s1 ? i : 0) * ldx;
    // staging: thread t loads rows 8 (t mod 4) .. + 8 of block column t / 4
    const int jj = threadIdx.x >> 2, r8 = (threadIdx.x & 3) * 8;
    const bool jok = bj * kBlk + jj < s2;
    const double* ycol = Y + (size_t)(jok ? bj * kBlk + jj : 0) * ldy;
    double stg[8];
    auto load_stage = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + r8 + e;
            stg[e] = (jok && k < k_end) ? ycol[k] : 0.0;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 8; ++e) ys[buf][(r8 + e) * kGramLd + jj] = stg[e];
    };
    d4_t acc[kBlkTiles];
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t) acc[t] = d4_t{0.0, 0.0, 0.0, 0.0};
    load_stage(k_begin);
    store_stage(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = k_begin; k0 < k_end; k0 += kGramKC) {
        const bool more = k0 + kGramKC < k_end;
        if (more) load_stage(k0 + kGramKC);
        if (rows_on) {
            double a[kGramKC / 4];
#pragma unroll
            for (int u = 0; u < kGramKC / 4; ++u) {
                const int k = k0 + 4 * u + kr;
                a[u] = (i < s1 && k < k_end) ? xc[k] : 0.0;
            }
            const double* yb = ys[buf] + kr * kGramLd + (lane & 15);
#pragma unroll
            for (int u = 0; u < kGramKC / 4; ++u)
#pragma unroll
                for (int t = 0; t < kBlkTiles; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], yb[4 * u * kGramLd + t * 16], acc[t], 0, 0, 0);
        }
        // the other buffer was last read before the previous barrier
        if (more) store_stage(1 - buf);
        __syncthreads();
        buf = 1 - buf;
    }
    if (!rows_on) return;
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t)
        for (int v = 0; v < 4; ++v) {
            const int gi = bi * kBlk + wave * 16 + 4 * v + (lane >> 4);
            const int gj = bj * kBlk + t * 16 + (lane & 15);
            if (gi < s1 && gj < s2) part[((size_t)split * s2 + gj) * s1 + gi] = acc[t][v];
        }
}

__global__ __launch_bounds__(512) void k_gram_bf16(int n, int s1, int s2, int chunk,
                                                   const double* __restrict__ X, int ldx,
                                                   const double* __restrict__ Y, int ldy,
                                                   double* __restrict__ part) {
    const int blocks_i = (s1 + kBlk - 1) / kBlk;
    int blk, split;
    xcd_block_chunk(gridDim.x, gridDim.y, blk, split);
    const int bi = blk % blocks_i, bj = blk / blocks_i;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = bi * kBlk + wave * 16 + (lane & 15);
    if (bi * kBlk + wave * 16 >= s1) return;  // no rows for this wave (no barrier below)
    const int kq = (lane >> 4) * 8;  // gfx950 16x16x32 BF16: 8 consecutive K per lane
    const int k_begin = split * chunk;
    const int k_end = min(n, k_begin + chunk);
    const double* xc = X + (size_t)(i < s1 ? i : 0) * ldx;
    const double* yc[kBlkTiles];
    bool jv[kBlkTiles];
    f4_t acc[kBlkTiles];
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t) {
        const int j = bj * kBlk + t * 16 + (lane & 15);
        jv[t] = j < s2;
        yc[t] = Y + (size_t)(jv[t] ? j : 0) * ldy;
        acc[t] = f4_t{0.f, 0.f, 0.f, 0.f};
    }
    for (int k0 = k_begin; k0 < k_end; k0 += 32) {
        s8_t a;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + kq + e;
            a[e] = to_bf16((i < s1 && k < k_end) ? xc[k] : 0.0);
        }
#pragma unroll
        for (int t = 0; t < kBlkTiles; ++t) {
            s8_t b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + kq + e;
                b[e] = to_bf16((jv[t] && k < k_end) ? yc[t][k] : 0.0);
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, a), __builtin_bit_cast(bf8_t, b),
                                                             acc[t], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t)
        for (int v = 0; v < 4; ++v) {
            const int gi = bi * kBlk + wave * 16 + 4 * (lane >> 4) + v;
            const int gj = bj * kBlk + t * 16 + (lane & 15);
            if (gi < s1 && gj < s2) part[((size_t)split * s2 + gj) * s1 + gi] = (double)acc[t][v];
        }
}

// Wide Gram for s2 <= 16 kWideMaxCT: grid.x = row blocks of rt row tiles,
// grid.y = K chunk.  A workgroup of eight waves stages the K step's rows of
// Y for all CT column tiles in LDS (double-buffered), so a K chunk of Y is
// read once per row block, and waves 0 .. rt-1 each compute one 16-row tile
// of the output against the CT column tiles (CT matrix-core accumulators).
// The output is covered by 16 x 16 tiles instead of 128 x 128 blocks (s =
// 220: 224^2 instead of 256^2 products).  For X = Y (self) a wave's A
// operand comes from the same staged rows, so X is not read at all.
constexpr int kWideKC = 32, kWideMaxCT = 16;
__host__ __device__ constexpr int wide_ld(int ct) { return 16 * ct + 16; }  // rows k, k + 1 in different bank halves

template <int CT>
__global__ __launch_bounds__(512) void k_gram_wide(int n, int s1, int s2, int chunk, int rt, int self,
                                                   const double* __restrict__ X, int ldx,
                                                   const double* __restrict__ Y, int ldy,
                                                   double* __restrict__ part) {
    extern __shared__ double wsh[];  // [2][kWideKC][LD]
    constexpr int LD = wide_ld(CT), SEG = 16 * CT * (kWideKC / 8), SPT = (SEG + 511) / 512;
    int blk, split;
    xcd_block_chunk(gridDim.x, gridDim.y, blk, split);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rtile = blk * rt + wave;
    const bool rows_on = wave < rt && rtile * 16 < s1;  // this wave has output rows (all waves stage Y)
    const int i = rtile * 16 + (lane & 15);
    const int kr = lane >> 4;
    const int k_begin = split * chunk;
    const int k_end = min(n, k_begin + chunk);
    const double* xc = X + (size_t)(i < s1 ? i : 0) * ldx;
    // staging: segment g = 8 consecutive rows (g mod 4) of column g / 4
    double stg[SPT][8];
    auto load_stage = [&](int k0) {
#pragma unroll
        for (int sp = 0; sp < SPT; ++sp) {
            const int g = threadIdx.x + 512 * sp;
            const int j = g >> 2, r8 = (g & 3) * 8;
            const bool jok = g < SEG && j < s2;
            const double* yc = Y + (size_t)(jok ? j : 0) * ldy;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + r8 + e;
                stg[sp][e] = (jok && k < k_end) ? yc[k] : 0.0;
            }
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int sp = 0; sp < SPT; ++sp) {
            const int g = threadIdx.x + 512 * sp;
            if (g < SEG) {
                const int j = g >> 2, r8 = (g & 3) * 8;
#pragma unroll
                for (int e = 0; e < 8; ++e) wsh[(buf * kWideKC + r8 + e) * LD + j] = stg[sp][e];
            }
        }
    };
    // X != Y: a wave's A operand of the next K step is loaded with the staging
    // loads, a step ahead of its use
    double xa[kWideKC / 4];
    auto load_x = [&](int k0) {
#pragma unroll
        for (int u = 0; u < kWideKC / 4; ++u) {
            const int k = k0 + 4 * u + kr;
            xa[u] = (!self && rows_on && i < s1 && k < k_end) ? xc[k] : 0.0;
        }
    };
    d4_t acc[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) acc[t] = d4_t{0.0, 0.0, 0.0, 0.0};
    load_stage(k_begin);
    load_x(k_begin);
    store_stage(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = k_begin; k0 < k_end; k0 += kWideKC) {
        const bool more = k0 + kWideKC < k_end;
        double a[kWideKC / 4];
#pragma unroll
        for (int u = 0; u < kWideKC / 4; ++u) a[u] = xa[u];
        if (more) {
            load_stage(k0 + kWideKC);
            load_x(k0 + kWideKC);
        }
        if (rows_on) {
            // A[l % 16][l / 16] = X[k0 + 4 u + l / 16][i], B[l / 16][l % 16] = Y[k0 + 4 u + l / 16][16 t + l % 16]
            const double* yb = wsh + (buf * kWideKC + kr) * LD + (lane & 15);
            if (self) {
#pragma unroll
                for (int u = 0; u < kWideKC / 4; ++u) a[u] = yb[4 * u * LD + 16 * rtile];
            }
#pragma unroll
            for (int u = 0; u < kWideKC / 4; ++u)
#pragma unroll
                for (int t = 0; t < CT; ++t)
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], yb[4 * u * LD + t * 16], acc[t], 0, 0, 0);
        }
        // the other buffer was last read before the previous barrier
        if (more) store_stage(1 - buf);
        __syncthreads();
        buf = 1 - buf;
    }
    if (!rows_on) return;
#pragma unroll
    for (int t = 0; t < CT; ++t)
        for (int v = 0; v < 4; ++v) {
            const int gi = rtile * 16 + 4 * v + (lane >> 4);
            const int gj = t * 16 + (lane & 15);
            if (gi < s1 && gj < s2) part[((size_t)split * s2 + gj) * s1 + gi] = acc[t][v];
        }
}

template <int CT>
void launch_gram_wide(Ctx* ctx, double flops, dim3 g, size_t shm, int n, int s1, int s2, int chunk, int rt, int self,
                      const double* X, int ldx, const double* Y, int ldy, double* part) {
    timed_launch_shm(ctx, kKGram, flops, k_gram_wide<CT>, g, dim3(512), shm, ctx->stream, n, s1, s2, chunk, rt, self,
                     X, ldx, Y, ldy, part);
}

// C = sum of the nsplit partial products.  A workgroup of 64 x kRedLanes
// threads owns 64 consecutive entries: lane y sums chunks y, y + kRedLanes, ...
// and the kRedLanes sums are added in lane order (a fixed order).
constexpr int kRedLanes = 16;
__global__ __launch_bounds__(64 * kRedLanes) void k_gram_reduce(int s1, int s2, int nsplit,
                                                                const double* __restrict__ part,
                                                                double* __restrict__ C, int ldc) {
    __shared__ double acc[kRedLanes][64];
    const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
    const int id = blockIdx.x * 64 + x;
    const size_t tot = (size_t)s1 * s2;
    double s = 0.0;
    if (id < s1 * s2)
        for (int p = y; p < nsplit; p += kRedLanes) s += part[(size_t)p * tot + id];
    acc[y][x] = s;
    __syncthreads();
    if (y == 0 && id < s1 * s2) {
        double t = 0.0;
        for (int l = 0; l < kRedLanes; ++l) t += acc[l][x];
        C[id % s1 + (size_t)(id / s1) * ldc] = t;
    }
}

// C = alpha X B + beta C (X: n x s, B: s x t).  grid.x: strips of 16
// kBlkWaves rows (one 16-row strip per wave), grid.y: 128-column blocks; a
// wave computes its 16 rows against the block's kBlkTiles column tiles, so
// X is read once per column block.  The block's columns of B are staged in
// LDS kGramKC rows at a time and shared by the eight waves, as in the Gram.
__global__ __launch_bounds__(512) void k_gemm_tall(int n, int s, int t, double alpha,
                                                   const double* __restrict__ X, int ldx,
                                                   const double* __restrict__ B, int ldb,
                                                   double beta, double* __restrict__ C, int ldc) {
    __shared__ double bsh[2][kGramKC * kGramLd];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the column blocks of one row strip read the same rows of X: they run on
    // one XCD one after another (grid: row strips x column blocks)
    int cb, strip;
    xcd_block_chunk(gridDim.y, gridDim.x, cb, strip);
    const int r0 = (strip * kBlkWaves + wave) * 16;
    const bool rows_on = r0 < n;  // this wave has output rows (all waves stage B)
    const int c0 = cb * kBlk;
    const int row = r0 + (lane & 15), kr = lane >> 4;
    const int jj = threadIdx.x >> 2, r8 = (threadIdx.x & 3) * 8;
    const bool jok = c0 + jj < t;
    const double* bcol = B + (size_t)(jok ? c0 + jj : 0) * ldb;
    double stg[8];
    auto load_stage = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + r8 + e;
            stg[e] = (jok && k < s) ? bcol[k] : 0.0;
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 8; ++e) bsh[buf][(r8 + e) * kGramLd + jj] = stg[e];
    };
    d4_t acc[kBlkTiles];
#pragma unroll
    for (int tt = 0; tt < kBlkTiles; ++tt) acc[tt] = d4_t{0.0, 0.0, 0.0, 0.0};
    load_stage(0);
    store_stage(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < s; k0 += kGramKC) {
        const bool more = k0 + kGramKC < s;
        if (more) load_stage(k0 + kGramKC);
        if (rows_on) {
            double a[kGramKC / 4];
#pragma unroll
            for (int u = 0; u < kGramKC / 4; ++u) {
                const int k = k0 + 4 * u + kr;
                a[u] = (row < n && k < s) ? X[(size_t)k * ldx + row] : 0.0;
            }
            const double* bb = bsh[buf] + kr * kGramLd + (lane & 15);
#pragma unroll
            for (int u = 0; u < kGramKC / 4; ++u)
#pragma unroll
                for (int tt = 0; tt < kBlkTiles; ++tt)
                    acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bb[4 * u * kGramLd + tt * 16], acc[tt], 0,
                                                                   0, 0);
        }
        // the other buffer was last read before the previous barrier
        if (more) store_stage(1 - buf);
        __syncthreads();
        buf = 1 - buf;
    }
    if (!rows_on) return;
#pragma unroll
    for (int tt = 0; tt < kBlkTiles; ++tt) {
        const int cc = c0 + tt * 16 + (lane & 15);
        if (cc >= t) continue;
        for (int v = 0; v < 4; ++v) {
            const int rr = r0 + 4 * v + (lane >> 4);
            if (rr < n) {
                double* dst = C + (size_t)cc * ldc + rr;
                *dst = alpha * acc[tt][v] + (beta != 0.0 ? beta * *dst : 0.0);
            }
        }
    }
}

// The one-workgroup factorizations below run on matrices addressed through a
// pointer and a leading dimension, either in place in global memory or, for
// small s, on copies staged in LDS (the _lds kernels: dynamic LDS, ld = s).
// A launch factors nb independent matrices, one workgroup each: workgroup b
// takes the matrices at base + b * stride (strides in elements).

// Upper Cholesky in place, one workgroup; A(a, c) = A[a + c lda].  Step j
// reads the pivot A(j, j), final since the previous step, in every thread,
// updates the trailing upper triangle by the outer product of row j scaled by
// 1 / sqrt(pivot), and scales row j - 1, which that update does not read:
// one barrier per step.
// With U > 1, U items of the trailing update per thread are loaded before
// they are stored; item indices advance by the workgroup size without
// dividing.  (Measured: U = 8 gains nothing in global memory, where the
// single-CU bandwidth bounds the update.)
template <int U>
__device__ __forceinline__ void cholesky_body(int s, double* A, int lda, double shift, int* __restrict__ flag) {
    for (int i = threadIdx.x; i < s; i += blockDim.x) A[i + (size_t)i * lda] += shift;
    __syncthreads();
    int bad = 0;
    double rprev = 1.0;  // sqrt of the previous pivot
    for (int j = 0; j <= s; ++j) {
        if (j > 0)  // row j - 1 by its pivot root
            for (int c = j - 1 + threadIdx.x; c < s; c += blockDim.x)
                A[j - 1 + (size_t)c * lda] = c == j - 1 ? rprev : A[j - 1 + (size_t)c * lda] / rprev;
        if (j == s) break;
        const double piv = A[j + (size_t)j * lda];
        if (!(piv > 0.0)) {
            bad = 1;
            break;
        }
        const double rj = sqrt(piv), irj = 1.0 / rj;
        const int m = s - j - 1, bd = blockDim.x;
        if (m > 0) {
            const int da = bd % m, dc = bd / m;
            int a = threadIdx.x % m, c = threadIdx.x / m;  // trailing block offsets, a fastest
            for (int id = threadIdx.x; id < m * m; id += U * bd) {
                double x[U], ya[U], yc[U];
                int as[U], cs[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    as[u] = a;
                    cs[u] = c;
                    x[u] = ya[u] = yc[u] = 0.0;
                    if (id + u * bd < m * m && a <= c) {
                        ya[u] = A[j + (size_t)(j + 1 + a) * lda];
                        yc[u] = A[j + (size_t)(j + 1 + c) * lda];
                        x[u] = A[j + 1 + a + (size_t)(j + 1 + c) * lda];
                    }
                    a += da;
                    c += dc;
                    if (a >= m) {
                        a -= m;
                        ++c;
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (id + u * bd < m * m && as[u] <= cs[u])
                        A[j + 1 + as[u] + (size_t)(j + 1 + cs[u]) * lda] = x[u] - (ya[u] * irj) * (yc[u] * irj);
            }
        }
        rprev = rj;
        __syncthreads();
    }
    __syncthreads();
    for (int id = threadIdx.x; id < s * s; id += blockDim.x) {
        const int a = id % s, c = id / s;
        if (a > c) A[a + (size_t)c * lda] = 0.0;
    }
    if (threadIdx.x == 0) *flag = bad;
}

// shift: per-matrix diagonal shifts (device) or null
__global__ __launch_bounds__(1024) void k_cholesky(int s, double* __restrict__ A, int lda, size_t sa, const double* __restrict__ shift,
                           int* __restrict__ flag) {
    cholesky_body<1>(s, A + blockIdx.x * sa, lda, shift ? shift[blockIdx.x] : 0.0, flag + blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_cholesky_lds(int s, double* __restrict__ A, int lda, size_t sa, const double* __restrict__ shift,
                               int* __restrict__ flag) {
    extern __shared__ double sm[];
    A += blockIdx.x * sa;
    for (int id = threadIdx.x; id < s * s; id += blockDim.x) sm[id] = A[id % s + (size_t)(id / s) * lda];
    __syncthreads();
    cholesky_body<1>(s, sm, s, shift ? shift[blockIdx.x] : 0.0, flag + blockIdx.x);
    __syncthreads();
    for (int id = threadIdx.x; id < s * s; id += blockDim.x) A[id % s + (size_t)(id / s) * lda] = sm[id];
}

// Rinv = R^-1 (upper), one workgroup: thread j solves R x = e_j for column j
// by back substitution (no barriers; the longest chain is s^2 / 2 products,
// which LDS keeps short for small s).
__device__ __forceinline__ void tri_inverse_body(int s, const double* R, int ldr, double* Ri, int ldi) {
    for (int j = threadIdx.x; j < s; j += blockDim.x) {
        double* x = Ri + (size_t)j * ldi;
        for (int i = j + 1; i < s; ++i) x[i] = 0.0;
        for (int i = j; i >= 0; --i) {
            double acc = i == j ? 1.0 : 0.0;
#pragma unroll 4
            for (int k = i + 1; k <= j; ++k) acc -= R[i + (size_t)k * ldr] * x[k];
            x[i] = acc / R[i + (size_t)i * ldr];
        }
    }
}

__global__ void k_tri_inverse_lds(int s, const double* __restrict__ R, int ldr, size_t sr,
                                  double* __restrict__ Ri, int ldi, size_t si) {
    extern __shared__ double sm[];
    R += blockIdx.x * sr;
    Ri += blockIdx.x * si;
    double* lr = sm;
    double* li = sm + (size_t)s * s;
    for (int id = threadIdx.x; id < s * s; id += blockDim.x) lr[id] = R[id % s + (size_t)(id / s) * ldr];
    __syncthreads();
    tri_inverse_body(s, lr, s, li, s);
    __syncthreads();
    for (int id = threadIdx.x; id < s * s; id += blockDim.x) Ri[id % s + (size_t)(id / s) * ldi] = li[id];
}

// Pair k of step `step` of the round-robin ordering of an even number m of
// indices (every pair meets once in m - 1 steps), ordered so that p < q.
__device__ __forceinline__ void rr_pair(int step, int k, int m, int& p, int& q) {
    if (k == 0) {
        p = step;
        q = m - 1;
    } else {
        p = (step + k) % (m - 1);
        q = (step - k + (m - 1)) % (m - 1);
    }
    if (p > q) {
        const int tmp = p;
        p = q;
        q = tmp;
    }
}

// Plane rotation (c, sv) that zeroes the off-diagonal entry of the symmetric
// 2 x 2 block [app apq; apq aqq] (the smaller of the two rotation angles).
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double& c, double& sv) {
    c = 1.0;
    sv = 0.0;
    if (apq != 0.0) {
        const double th = (aqq - app) / (2.0 * apq);
        const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
        c = 1.0 / sqrt(1.0 + tt * tt);
        sv = tt * c;
    }
}

// Squared off-diagonal and total Frobenius norms of the s x s matrix T (ld),
// summed in a fixed order; every thread returns both.
__device__ __forceinline__ void jacobi_norms(int s, const double* T, int ld, double& offn, double& totn) {
    __shared__ double wsum[32];
    double o = 0.0, t = 0.0;
    for (int id = threadIdx.x; id < s * s; id += blockDim.x) {
        const int a = id % s, c = id / s;
        const double v = T[a + (size_t)c * ld];
        t += v * v;
        if (a != c) o += v * v;
    }
    for (int off = 32; off > 0; off >>= 1) {
        o += __shfl_xor(o, off, 64);
        t += __shfl_xor(t, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        wsum[threadIdx.x >> 6] = o;
        wsum[16 + (threadIdx.x >> 6)] = t;
    }
    __syncthreads();
    double so = 0.0, st = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        so += wsum[w];
        st += wsum[16 + w];
    }
    offn = so;
    totn = st;
    __syncthreads();  // wsum is reused by the next call
}

// Stopping test of the Jacobi sweeps: the off-diagonal Frobenius norm is below
// 1e-12 of the total, or, once it is below 1e-8, a sweep no longer halves it
// (rounding in the rotations keeps it near s eps |T|, so a fixed tighter
// bound may never be met).  prev: squared off-diagonal norm of the previous
// sweep (negative before the first).
__device__ __forceinline__ bool jacobi_done(double offn, double totn, double prev) {
    if (offn <= 1e-24 * totn || totn == 0.0) return true;
    return prev >= 0.0 && offn <= 1e-16 * totn && offn > 0.25 * prev;
}

// One step of the parallel Jacobi sweep: the np rotations (pp, qq, cs, sn)
// applied to both sides of T and to the columns of S.  The thread of pair
// block (k, l) forms rows p_k, q_k of J^T T on columns p_l, q_l and rotates
// those columns: the same products in the same order as a row pass followed
// by a column pass, with every entry of T read and written once.  A pair
// with q >= s (odd s) has the identity rotation and no row or column q.  Each
// thread keeps U items' loads in flight before their stores, and advances
// its item indices by the workgroup size without dividing.
template <int U, bool kS>
__device__ __forceinline__ void jacobi_apply(int s, int np, double* T, int ldt, double* S, int lds,
                                             const int* pp, const int* qq, const double* cs, const double* sn) {
    const int bd = blockDim.x;
    {
        const int nb = np * np, dk = bd % np, dl = bd / np;
        int k = threadIdx.x % np, l = threadIdx.x / np;
        for (int id = threadIdx.x; id < nb; id += U * bd) {
            double va[U], vb[U], vc[U], vd[U];
            int ks[U], ls[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                ks[u] = k;
                ls[u] = l;
                va[u] = vb[u] = vc[u] = vd[u] = 0.0;
                if (id + u * bd < nb) {
                    const int pk = pp[k], qk = qq[k], pl = pp[l], ql = qq[l];
                    va[u] = T[pk + (size_t)pl * ldt];
                    if (ql < s) vb[u] = T[pk + (size_t)ql * ldt];
                    if (qk < s) vc[u] = T[qk + (size_t)pl * ldt];
                    if (qk < s && ql < s) vd[u] = T[qk + (size_t)ql * ldt];
                }
                k += dk;
                l += dl;
                if (k >= np) {
                    k -= np;
                    ++l;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (id + u * bd >= nb) break;
                const int kk = ks[u], ll = ls[u];
                const int pk = pp[kk], qk = qq[kk], pl = pp[ll], ql = qq[ll];
                const double ck = cs[kk], sk = sn[kk], cl = cs[ll], sl = sn[ll];
                const double r0x = ck * va[u] - sk * vc[u], r0y = ck * vb[u] - sk * vd[u];
                const double r1x = sk * va[u] + ck * vc[u], r1y = sk * vb[u] + ck * vd[u];
                T[pk + (size_t)pl * ldt] = cl * r0x - sl * r0y;
                if (ql < s) T[pk + (size_t)ql * ldt] = sl * r0x + cl * r0y;
                if (qk < s) T[qk + (size_t)pl * ldt] = cl * r1x - sl * r1y;
                if (qk < s && ql < s) T[qk + (size_t)ql * ldt] = sl * r1x + cl * r1y;
            }
        }
    }
    if (kS) {
        const int ns = np * s, dr = bd % s, dq = bd / s;
        int r = threadIdx.x % s, k = threadIdx.x / s;
        for (int id = threadIdx.x; id < ns; id += U * bd) {
            double vp[U], vq[U];
            int rs[U], ks[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                rs[u] = r;
                ks[u] = k;
                vp[u] = vq[u] = 0.0;
                if (id + u * bd < ns && qq[k] < s) {
                    vp[u] = S[r + (size_t)pp[k] * lds];
                    vq[u] = S[r + (size_t)qq[k] * lds];
                }
                r += dr;
                k += dq;
                if (r >= s) {
                    r -= s;
                    ++k;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (id + u * bd >= ns) break;
                const int kk = ks[u], rr = rs[u];
                if (qq[kk] >= s) continue;
                S[rr + (size_t)pp[kk] * lds] = cs[kk] * vp[u] - sn[kk] * vq[u];
                S[rr + (size_t)qq[kk] * lds] = sn[kk] * vp[u] + cs[kk] * vq[u];
            }
        }
    }
}

// Parallel cyclic Jacobi (round-robin pairing), one workgroup, on T and S
// (ld ldt, lds): per step, the np disjoint rotations, then jacobi_apply.
// With rot given, S is left alone: step t of the run stores its rotations
// (c, s) at rot[t np + k] and the number of sweeps run goes to *nsweeps.
template <int U, bool kS>
__device__ __forceinline__ void jacobi_sweeps(int s, double* T, int ldt, double* S, int lds, int max_sweeps,
                                              double2* __restrict__ rot = nullptr, int* nsweeps = nullptr) {
    const int m = s + (s & 1);
    const int np = m / 2;
    __shared__ double cs[256], sn[256];
    __shared__ int pp[256], qq[256];
    double prev = -1.0;  // off-diagonal norm^2 of the previous sweep
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        double offn, totn;
        jacobi_norms(s, T, ldt, offn, totn);
        if (jacobi_done(offn, totn, prev)) break;
        prev = offn;
        for (int step = 0; step < m - 1; ++step) {
            for (int k = threadIdx.x; k < np; k += blockDim.x) {
                int p, q;
                rr_pair(step, k, m, p, q);
                double c = 1.0, sv = 0.0;
                if (q < s)
                    jacobi_rotation(T[p + (size_t)p * ldt], T[q + (size_t)q * ldt], T[p + (size_t)q * ldt], c, sv);
                pp[k] = p;
                qq[k] = q;
                cs[k] = c;
                sn[k] = sv;
                if (!kS) rot[((size_t)sweep * (m - 1) + step) * np + k] = make_double2(c, sv);
            }
            __syncthreads();
            jacobi_apply<U, kS>(s, np, T, ldt, S, lds, pp, qq, cs, sn);
            __syncthreads();
        }
    }
    if (!kS && threadIdx.x == 0) *nsweeps = sweep;
}

// In place in global memory (large s); six items per thread in flight.
// The rotations are recorded (rot: max_sweeps (m - 1) np per matrix, stride
// srot) and applied to S afterwards by k_jacobi_rows, so each step moves T
// alone through the one CU.
__global__ __launch_bounds__(1024) void k_jacobi(int s, double* __restrict__ T, int ldt, size_t st,
                                                 double2* __restrict__ rot, size_t srot, int* __restrict__ nsweeps,
                                                 int max_sweeps) {
    T += blockIdx.x * st;
    // symmetrize
    for (int id = threadIdx.x; id < s * s; id += blockDim.x) {
        const int a = id % s, c = id / s;
        if (a < c) {
            const double v = 0.5 * (T[a + (size_t)c * ldt] + T[c + (size_t)a * ldt]);
            T[a + (size_t)c * ldt] = v;
            T[c + (size_t)a * ldt] = v;
        }
    }
    __syncthreads();
    jacobi_sweeps<6, false>(s, T, ldt, nullptr, 0, max_sweeps, rot + blockIdx.x * srot, nsweeps + blockIdx.x);
}

// S = J_1 J_2 ... (the recorded rotations in order, S starting as I).  Rows of
// S never mix, so workgroup (x, b) takes kRotRows rows of matrix b into LDS
// and applies every recorded step to them; the rotations of kRotSteps steps
// (with their pairs) are staged in LDS at a time.
constexpr int kRotRows = 4, kRotSteps = 8;
__global__ __launch_bounds__(256) void k_jacobi_rows(int s, const double2* __restrict__ rot, size_t srot,
                                                     const int* __restrict__ nsweeps, double* __restrict__ S,
                                                     int lds, size_t ss) {
    __shared__ double rows[kRotRows][512];
    __shared__ double2 rcs[kRotSteps][256];
    __shared__ short rp[kRotSteps][256], rq[kRotSteps][256];
    const int b = blockIdx.y, r0 = blockIdx.x * kRotRows;
    const int m = s + (s & 1), np = m / 2;
    rot += b * srot;
    S += b * ss;
    for (int t = threadIdx.x; t < kRotRows * s; t += blockDim.x) {
        const int r = t / s, c = t - r * s;
        rows[r][c] = r0 + r == c ? 1.0 : 0.0;
    }
    const int nst = nsweeps[b] * (m - 1);
    for (int st0 = 0; st0 < nst; st0 += kRotSteps) {
        const int nk = min(kRotSteps, nst - st0);
        __syncthreads();  // the previous chunk is applied (and rows initialized)
        for (int t = threadIdx.x; t < nk * np; t += blockDim.x) {
            const int j = t / np, k = t - j * np;
            int p, q;
            rr_pair((st0 + j) % (m - 1), k, m, p, q);
            rp[j][k] = (short)p;
            rq[j][k] = (short)q;
            rcs[j][k] = rot[(size_t)(st0 + j) * np + k];
        }
        __syncthreads();
        for (int j = 0; j < nk; ++j) {
            for (int t = threadIdx.x; t < kRotRows * np; t += blockDim.x) {
                const int r = t / np, k = t - r * np;
                const int p = rp[j][k], q = rq[j][k];
                if (q >= s) continue;
                const double2 c = rcs[j][k];
                const double sp = rows[r][p], sq = rows[r][q];
                rows[r][p] = c.x * sp - c.y * sq;
                rows[r][q] = c.y * sp + c.x * sq;
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kRotRows * s; t += blockDim.x) {
        const int r = t / s, c = t - r * s;
        if (r0 + r < s) S[r0 + r + (size_t)c * lds] = rows[r][c];
    }
}

// The same sweeps on copies of T and S in LDS (ld s), written back at the end;
// one item per thread at a time (LDS latency needs no loads in flight).
__global__ __launch_bounds__(1024) void k_jacobi_lds(int s, double* __restrict__ T, int ldt, size_t st,
                                                     double* __restrict__ S, int lds, size_t ss, int max_sweeps) {
    extern __shared__ double sm[];
    T += blockIdx.x * st;
    S += blockIdx.x * ss;
    double* tl = sm;
    double* sl = sm + (size_t)s * s;
    for (int id = threadIdx.x; id < s * s; id += blockDim.x) {
        const int a = id % s, c = id / s;
        tl[id] = a == c ? T[a + (size_t)a * ldt] : 0.5 * (T[a + (size_t)c * ldt] + T[c + (size_t)a * ldt]);
        sl[id] = a == c ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi_sweeps<1, true>(s, tl, s, sl, s, max_sweeps);
    for (int id = threadIdx.x; id < s * s; id += blockDim.x) {
        const int a = id % s, c = id / s;
        T[a + (size_t)c * ldt] = tl[id];
        S[a + (size_t)c * lds] = sl[id];
    }
}

// Sorts the eigenpairs by decreasing eigenvalue: column c of S goes to column
// rank(c) of Sout, and lam[rank(c)] = lam_unsorted[c] (ties keep index order).
// grid.y: matrix of the batch (S, Sout, lam_unsorted and lam at their strides).
__global__ void k_eig_permute(int s, const double* __restrict__ lam_unsorted, size_t slu,
                              const double* __restrict__ S, int lds, size_t ss, double* __restrict__ Sout, int ldo,
                              size_t so, double* __restrict__ lam, size_t sl) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= s * s) return;
    lam_unsorted += blockIdx.y * slu;
    S += blockIdx.y * ss;
    Sout += blockIdx.y * so;
    lam += blockIdx.y * sl;
    const int r = id % s, c = id / s;
    const double lc = lam_unsorted[c];
    int rank = 0;
    for (int j = 0; j < s; ++j) {
        const double lj = lam_unsorted[j];
        rank += (lj > lc) || (lj == lc && j < c);
    }
    Sout[r + (size_t)rank * ldo] = S[r + (size_t)c * lds];
    if (r == 0) lam[rank] = lc;
}

__global__ void k_diag_copy(int s, const double* __restrict__ T, int ldt, size_t st, double* __restrict__ d,
                            size_t sd) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < s) d[blockIdx.y * sd + i] = T[blockIdx.y * st + i + (size_t)i * ldt];
}

// out[b] = factor * trace(A_b), one workgroup per matrix.
__global__ void k_scaled_trace(int s, const double* __restrict__ A, int lda, size_t sa, double factor,
                               double* __restrict__ out) {
    __shared__ double w[16];
    A += blockIdx.x * sa;
    double v = 0.0;
    for (int i = threadIdx.x; i < s; i += blockDim.x) v += A[i + (size_t)i * lda];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += w[k];
        out[blockIdx.x] = factor * t;
    }
}

// C_b (m x n) = alpha A_b (m x kk) B_b (kk x n), one thread per entry of C
// (column-major, grid.y: matrix of the batch, strides in elements).
__global__ void k_small_gemm(int m, int n, int kk, double alpha, const double* __restrict__ A, int lda,
                             size_t sa, const double* __restrict__ B, int ldb, size_t sb, double* __restrict__ C,
                             int ldc, size_t sc) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= m * n) return;
    const int i = id % m, j = id / m;
    A += blockIdx.y * sa;
    B += blockIdx.y * sb;
    C += blockIdx.y * sc;
    double acc = 0.0;
#pragma unroll 8
    for (int k = 0; k < kk; ++k) acc += A[i + (size_t)k * lda] * B[k + (size_t)j * ldb];
    C[i + (size_t)j * ldc] = alpha * acc;
}

// C (m x n) = alpha op(A) op(B) + beta C with op(X) = X or X^T (flags ta, tb),
// one thread per entry of C; the small s x s products of the single-pass
// eigensolver.
__global__ void k_small_gemm_t(int m, int n, int kk, int ta, int tb, double alpha, const double* __restrict__ A,
                               int lda, const double* __restrict__ B, int ldb, double beta, double* __restrict__ C,
                               int ldc) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= m * n) return;
    const int i = id % m, j = id / m;
    const size_t ai = ta ? (size_t)i * lda : i, ak = ta ? 1 : lda;
    const size_t bj = tb ? j : (size_t)j * ldb, bk = tb ? ldb : 1;
    double acc = 0.0;
    for (int k = 0; k < kk; ++k) acc += A[ai + k * ak] * B[bj + k * bk];
    double* c = C + i + (size_t)j * ldc;
    *c = beta == 0.0 ? alpha * acc : alpha * acc + beta * *c;
}

// C[i, j] /= d[i] + d[j] (s x s): the solution of the Sylvester equation
// D X + X D = C for diagonal D.
__global__ void k_sylvester_diag(int s, const double* __restrict__ d, double* __restrict__ C, int ldc) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= s * s) return;
    const int i = id % s, j = id / s;
    C[i + (size_t)j * ldc] /= d[i] + d[j];
}

// out[i] = base[i] (0 when null) + sum_j w[j] V[i, j]^2 (V: n x k, ldv).
__global__ void k_weighted_squares(int n, int k, const double* __restrict__ V, int ldv, const double* __restrict__ w,
                                   const double* __restrict__ base, double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int j = 0; j < k; ++j) {
        const double v = V[i + (size_t)j * ldv];
        acc += w[j] * v * v;
    }
    out[i] = (base ? base[i] : 0.0) + acc;
}

__global__ void k_zero_matrix(int m, int n, double* __restrict__ C, int ldc, size_t sc) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id < m * n) C[blockIdx.y * sc + id % m + (size_t)(id / m) * ldc] = 0.0;
}

__global__ void k_scale_rows(int s, int t, const double* __restrict__ d, double* __restrict__ B, int ldb) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= s * t) return;
    const int i = id % s, j = id / s;
    B[i + (size_t)j * ldb] *= d[i];
}

}  // namespace

void gram(Ctx* ctx, DenseWork& w, int n, int s1, int s2, const double* X, int ldx, const double* Y,
          int ldy, double* C, int ldc, bool bf16) {
    if (!bf16 && s2 <= 16 * kWideMaxCT) {
        const int ct = ceil_div(s2, 16), rtt = ceil_div(s1, 16);
        const int nrb = ceil_div(rtt, 8), rt = ceil_div(rtt, nrb);
        int cus = 0;
        HINV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        // about one workgroup a compute unit (the staging takes most of the
        // LDS), chunks of at least 256 rows in whole K steps
        int nsplit = std::max(1, std::min(ceil_div(cus, nrb), ceil_div(n, 256)));
        const int chunk = ceil_div(ceil_div(n, nsplit), kWideKC) * kWideKC;
        nsplit = ceil_div(n, chunk);
        w.part.ensure((size_t)nsplit * s1 * s2);
        const size_t shm = sizeof(double) * 2 * kWideKC * wide_ld(ct);
        const int self = X == Y && ldx == ldy && s1 <= s2;
        const dim3 g(nrb, nsplit);
        const double flops = 2.0 * n * s1 * s2;
        switch (ct) {
#define HINV_WIDE(c) \
    case c: launch_gram_wide<c>(ctx, flops, g, shm, n, s1, s2, chunk, rt, self, X, ldx, Y, ldy, w.part.get()); break;
            HINV_WIDE(1) HINV_WIDE(2) HINV_WIDE(3) HINV_WIDE(4) HINV_WIDE(5) HINV_WIDE(6) HINV_WIDE(7) HINV_WIDE(8)
            HINV_WIDE(9) HINV_WIDE(10) HINV_WIDE(11) HINV_WIDE(12) HINV_WIDE(13) HINV_WIDE(14) HINV_WIDE(15)
            default: launch_gram_wide<16>(ctx, flops, g, shm, n, s1, s2, chunk, rt, self, X, ldx, Y, ldy, w.part.get());
#undef HINV_WIDE
        }
        HINV_LAUNCH_CHECK();
        k_gram_reduce<<<ceil_div(s1 * s2, 64), 64 * kRedLanes, 0, ctx->stream>>>(s1, s2, nsplit, w.part.get(), C,
                                                                                ldc);
        HINV_LAUNCH_CHECK();
        return;
    }
    const int blocks = ((s1 + kBlk - 1) / kBlk) * ((s2 + kBlk - 1) / kBlk);
    // K split: about 2048 workgroups, chunks of at least 256 rows (a multiple
    // of the 16-row matrix-core step)
    int nsplit = std::max(1, std::min(ceil_div(2048, blocks), ceil_div(n, 256)));
    const int chunk = ceil_div(ceil_div(n, nsplit), kGramKC) * kGramKC;  // a multiple of both kernels' K steps
    nsplit = ceil_div(n, chunk);
    w.part.ensure((size_t)nsplit * s1 * s2);
    const double flops = 2.0 * n * s1 * s2;
    if (bf16)
        timed_launch(ctx, kKGram, flops, k_gram_bf16, dim3(blocks, nsplit), dim3(64 * kBlkWaves), ctx->stream,
                     n, s1, s2, chunk, X, ldx, Y, ldy, w.part.get());
    else
        timed_launch(ctx, kKGram, flops, k_gram_f64, dim3(blocks, nsplit), dim3(64 * kBlkWaves), ctx->stream,
                     n, s1, s2, chunk, X, ldx, Y, ldy, w.part.get());
    HINV_LAUNCH_CHECK();
    k_gram_reduce<<<ceil_div(s1 * s2, 64), 64 * kRedLanes, 0, ctx->stream>>>(s1, s2, nsplit, w.part.get(), C,
                                                                            ldc);
    HINV_LAUNCH_CHECK();
}

void gemm_tall(Ctx* ctx, int n, int s, int t, double alpha, const double* X, int ldx,
               const double* B, int ldb, double beta, double* C, int ldc) {
    if (n <= 0 || t <= 0) return;
    const dim3 g(ceil_div(ceil_div(n, 16), kBlkWaves), ceil_div(t, kBlk));
    k_gemm_tall<<<g, 64 * kBlkWaves, 0, ctx->stream>>>(n, s, t, alpha, X, ldx, B, ldb, beta, C, ldc);
    HINV_LAUNCH_CHECK();
}

// Whether a one-workgroup kernel may stage `bytes` of dynamic LDS on the
// context's device (with room for its static LDS, at most 8 KB here).
bool lds_fits(Ctx* ctx, size_t bytes) {
    int v = 0;
    HINV_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device));
    return bytes + 8192 <= (size_t)v;
}

bool cholesky_upper(Ctx* ctx, DenseWork& w, int nb, int s, double* A, int lda, size_t sa,
                    const double* shift) {
    if (nb <= 0) return true;
    w.flag.ensure(nb);
    const size_t shm = sizeof(double) * s * s;
    if (lds_fits(ctx, shm))
        k_cholesky_lds<<<nb, 1024, shm, ctx->stream>>>(s, A, lda, sa, shift, w.flag.get());
    else
        k_cholesky<<<nb, 1024, 0, ctx->stream>>>(s, A, lda, sa, shift, w.flag.get());
    HINV_LAUNCH_CHECK();
    std::vector<int> bad(nb);
    HINV_HIP(hipMemcpyAsync(bad.data(), w.flag.get(), sizeof(int) * nb, hipMemcpyDeviceToHost, ctx->stream));
    HINV_HIP(hipStreamSynchronize(ctx->stream));
    for (int b : bad)
        if (b) return false;
    return true;
}

void tri_inverse_upper(Ctx* ctx, DenseWork& w, int nb, int s, const double* R, int ldr, size_t sr, double* Rinv,
                       int ldi, size_t si) {
    if (nb <= 0 || s <= 0) return;
    auto diag_inverse = [&](int o, int sz) {
        k_tri_inverse_lds<<<nb, 1024, sizeof(double) * 2 * sz * sz, ctx->stream>>>(
            sz, R + o + (size_t)o * ldr, ldr, sr, Rinv + o + (size_t)o * ldi, ldi, si);
        HINV_LAUNCH_CHECK();
    };
    if (lds_fits(ctx, sizeof(double) * 2 * s * s)) {
        diag_inverse(0, s);
        return;
    }
    // Blocked for large s: the diagonal blocks (at most bs, in LDS), then block
    // rows bottom-up, Rinv(I, J) = -Rinv(I, I) [R(I, I+1..J) Rinv(I+1..J, J)].
    int bs = 128;
    while (bs > 8 && !lds_fits(ctx, sizeof(double) * 2 * bs * bs)) bs -= 8;
    const int nbk = ceil_div(s, bs);
    const dim3 gz(ceil_div(s * s, 256), nb);
    k_zero_matrix<<<gz, 256, 0, ctx->stream>>>(s, s, Rinv, ldi, si);
    HINV_LAUNCH_CHECK();
    for (int I = 0; I < nbk; ++I) diag_inverse(I * bs, std::min(bs, s - I * bs));
    const size_t ts = (size_t)bs * bs;
    w.tmp.ensure(nb * ts);
    double* tmp = w.tmp.get();
    for (int I = nbk - 2; I >= 0; --I) {
        const int oi = I * bs, mi = std::min(bs, s - oi), k0 = oi + mi;
        for (int J = I + 1; J < nbk; ++J) {
            const int oj = J * bs, nj = std::min(bs, s - oj), k1 = oj + nj;
            const dim3 g(ceil_div(mi * nj, 256), nb);
            k_small_gemm<<<g, 256, 0, ctx->stream>>>(mi, nj, k1 - k0, 1.0, R + oi + (size_t)k0 * ldr, ldr, sr,
                                                    Rinv + k0 + (size_t)oj * ldi, ldi, si, tmp, mi, ts);
            HINV_LAUNCH_CHECK();
            k_small_gemm<<<g, 256, 0, ctx->stream>>>(mi, nj, mi, -1.0, Rinv + oi + (size_t)oi * ldi, ldi, si, tmp,
                                                    mi, ts, Rinv + oi + (size_t)oj * ldi, ldi, si);
            HINV_LAUNCH_CHECK();
        }
    }
}

void sym_eig(Ctx* ctx, DenseWork& w, int nb, int s, double* T, int ldt, size_t st, double* S, int lds, size_t ss,
             double* lam, size_t sl) {
    if (s > 512) fail(HINV_EINVAL, "eigenproblem larger than 512");
    if (nb <= 0 || s <= 0) return;
    const size_t s2 = (size_t)s * s;
    w.part.ensure(nb * (s2 + s));
    double* Stmp = w.part.get();
    double* lam_u = Stmp + nb * s2;
    const size_t shm = sizeof(double) * 2 * s2;
    constexpr int kMaxSweeps = 40;
    if (lds_fits(ctx, shm)) {
        k_jacobi_lds<<<nb, 1024, shm, ctx->stream>>>(s, T, ldt, st, Stmp, s, s2, kMaxSweeps);
        HINV_LAUNCH_CHECK();
    } else {
        const int m = s + (s & 1), np = m / 2;
        const size_t srot = (size_t)kMaxSweeps * (m - 1) * np;
        w.rot.ensure(nb * srot * 2);
        w.flag.ensure(nb);
        double2* rot = reinterpret_cast<double2*>(w.rot.get());
        k_jacobi<<<nb, 1024, 0, ctx->stream>>>(s, T, ldt, st, rot, srot, w.flag.get(), kMaxSweeps);
        HINV_LAUNCH_CHECK();
        k_jacobi_rows<<<dim3(ceil_div(s, kRotRows), nb), 256, 0, ctx->stream>>>(s, rot, srot, w.flag.get(), Stmp, s,
                                                                                 s2);
        HINV_LAUNCH_CHECK();
    }
    k_diag_copy<<<dim3(ceil_div(s, 256), nb), 256, 0, ctx->stream>>>(s, T, ldt, st, lam_u, s);
    HINV_LAUNCH_CHECK();
    k_eig_permute<<<dim3(ceil_div(s * s, 256), nb), 256, 0, ctx->stream>>>(s, lam_u, s, Stmp, s, s2, S, lds, ss,
                                                                            lam, sl);
    HINV_LAUNCH_CHECK();
}

void scaled_trace(Ctx* ctx, int nb, int s, const double* A, int lda, size_t sa, double factor, double* out) {
    if (nb <= 0) return;
    k_scaled_trace<<<nb, 1024, 0, ctx->stream>>>(s, A, lda, sa, factor, out);
    HINV_LAUNCH_CHECK();
}

void small_gemm(Ctx* ctx, bool ta, bool tb, int m, int n, int kk, double alpha, const double* A, int lda,
                const double* B, int ldb, double beta, double* C, int ldc) {
    if (m * n == 0) return;
    k_small_gemm_t<<<ceil_div((long)m * n, 256), 256, 0, ctx->stream>>>(m, n, kk, ta, tb, alpha, A, lda, B, ldb,
                                                                         beta, C, ldc);
    HINV_LAUNCH_CHECK();
}

void sylvester_diag(Ctx* ctx, int s, const double* d, double* C, int ldc) {
    if (s == 0) return;
    k_sylvester_diag<<<ceil_div((long)s * s, 256), 256, 0, ctx->stream>>>(s, d, C, ldc);
    HINV_LAUNCH_CHECK();
}

void weighted_squares(Ctx* ctx, int n, int k, const double* V, int ldv, const double* w, const double* base,
                      double* out) {
    k_weighted_squares<<<ceil_div(n, 256), 256, 0, ctx->stream>>>(n, k, V, ldv, w, base, out);
    HINV_LAUNCH_CHECK();
}

void scale_rows(Ctx* ctx, int s, int t, const double* d, double* B, int ldb) {
    if (s * t == 0) return;
    k_scale_rows<<<ceil_div(s * t, 256), 256, 0, ctx->stream>>>(s, t, d, B, ldb);
    HINV_LAUNCH_CHECK();
}

}  // namespace hinv
