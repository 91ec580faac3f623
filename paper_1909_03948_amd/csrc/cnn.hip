// Residual CNN of the learned preconditioner: forward, backward and Adam on
// the device (see cnn.h).
//
// Convolutions are implicit GEMMs on the BF16 matrix cores (FP32
// accumulation): gfx950's v_mfma_f32_16x16x32_bf16 for K-steps of 32, the
// 16x16x16 form where a layer has only 16 (padded) input channels.  A
// workgroup owns a 16 x 16 pixel tile of one image and all output channels;
// its input tile with a one-pixel halo and the layer's 3x3 x C_out x C_in
// weights sit in LDS.  Each of the 4 waves computes 4 rows of 16 pixels; per
// tap (dy, dx) and K-step of input channels, operand A is 16 pixels x K
// channels read from the halo tile at the shifted position and operand B the
// tap's K x 16 weight block.  Operand layouts (wave64; checked on the device
// against a host product): with K = 32, A: lane l holds A[l % 16][8 (l / 16) + e],
// B: lane l holds B[8 (l / 16) + e][l % 16] (e < 8); with K = 16 the same
// with 4 (l / 16) + e (e < 4); D: lane l item v holds D[4 (l / 16) + v][l % 16].
//
// The backward pass reuses the same kernel: the input gradient of a
// convolution is a convolution of the output gradient with the weights
// transposed in the channels and flipped in space.  Weight gradients are
// per-tile MFMA products (pixels as the K dimension) reduced over tiles in a
// fixed order.
#include <algorithm>
#include <cmath>
#include <vector>

#include "cnn.h"

namespace hinv {

namespace {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));
typedef short s8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

// D += A B with K = 32 (operands as BF16 bit patterns)
__device__ inline f4_t mfma_k32(s8_t a, s8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8_t, a), __builtin_bit_cast(bf8_t, b), c, 0,
                                                   0, 0);
}

constexpr int kT = 16;       // output tile side (pixels)
constexpr int kH = kT + 2;   // tile side with halo
constexpr int kWgStride = 9 * 32 * 32 + 32;  // floats per workgroup in the weight-gradient partials

enum { EPI_RELU = 0, EPI_RELU_RES = 1, EPI_LINEAR = 2, EPI_BWD = 3 };

__device__ inline short bf16_bits(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (short)(u >> 16);
}

__device__ inline float bf16_value(short s) { return __uint_as_float(((unsigned)(unsigned short)s) << 16); }

struct LayerDesc {
    int co, ci;    // real channel counts
    int COp, CIp;  // padded
    int woff, boff;  // offsets of W and b in the packed parameters
};

const LayerDesc* layers() {
    static LayerDesc L[Cnn::kLayers];
    static bool init = false;
    if (!init) {
        const int co[6] = {32, 32, 32, 32, 32, 1}, ci[6] = {3, 32, 32, 32, 32, 32};
        int off = 0;
        for (int l = 0; l < 6; ++l) {
            L[l].co = co[l];
            L[l].ci = ci[l];
            L[l].COp = co[l] == 1 ? Cnn::kPadIn : co[l];
            L[l].CIp = ci[l] == 3 ? Cnn::kPadIn : ci[l];
            L[l].woff = off;
            off += co[l] * ci[l] * 9;
            L[l].boff = off;
            off += co[l];
        }
        init = true;
    }
    return L;
}

// Padded BF16 weights: forward wf[t][co][ci] = W[co][ci][t], backward
// wb[t][ci][co] = W[co][ci][8 - t] (channels transposed, taps flipped).
__global__ void k_weights_prep(const float* __restrict__ W, int co_r, int ci_r, int COp, int CIp,
                               short* __restrict__ wf, short* __restrict__ wb) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= 9 * COp * CIp) return;
    const int t = id / (COp * CIp), rem = id % (COp * CIp), co = rem / CIp, ci = rem % CIp;
    const bool real = co < co_r && ci < ci_r;
    wf[id] = real ? bf16_bits(W[(co * ci_r + ci) * 9 + t]) : (short)0;
    wb[(t * CIp + ci) * COp + co] = real ? bf16_bits(W[(co * ci_r + ci) * 9 + (8 - t)]) : (short)0;
}

// Planar FP32 [B][3][S][S] -> pixel-major BF16 with 16 channels (3 used).
__global__ void k_pack_input(int B, int S, const float* __restrict__ in, short* __restrict__ out) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long np = (long long)S * S;
    if (id >= np * B) return;
    const long long b = id / np, p = id % np;
    short* o = out + id * Cnn::kPadIn;
    for (int c = 0; c < Cnn::kPadIn; ++c)
        o[c] = c < Cnn::kInCh ? bf16_bits(in[(b * Cnn::kInCh + c) * np + p]) : (short)0;
}

// Channel 0 of a 16-channel FP32 image -> planar [B][S][S].
__global__ void k_unpack_output(long long npix, const float* __restrict__ y, float* __restrict__ out) {
    const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id < npix) out[id] = y[id * Cnn::kPadIn];
}

// Convolution with fused epilogue.  Grid: (tiles x, tiles y, images).
//   EPI_RELU:     z = conv + b; h = relu(z)
//   EPI_RELU_RES: z = conv + b; h = res + relu(z)
//   EPI_LINEAR:   z = conv + b
//   EPI_BWD:      g = conv + res (res optional); out16 = bf16(g * [zmask > 0])
template <int CI, int CO, int EPI>
__global__ __launch_bounds__(256) void k_conv(int S, const short* __restrict__ in, const short* __restrict__ w,
                                              const float* __restrict__ bias, int co_real,
                                              const float* __restrict__ res, const float* __restrict__ zmask,
                                              float* __restrict__ zout, float* __restrict__ out32,
                                              short* __restrict__ out16) {
    __shared__ __attribute__((aligned(16))) short sin[kH * kH * CI];
    __shared__ __attribute__((aligned(16))) short sw[9 * CO * CI];
    const int tx0 = blockIdx.x * kT, ty0 = blockIdx.y * kT, b = blockIdx.z;
    for (int e = threadIdx.x; e < 9 * CO * CI / 4; e += blockDim.x)
        reinterpret_cast<long long*>(sw)[e] = reinterpret_cast<const long long*>(w)[e];
    for (int e = threadIdx.x; e < kH * kH * (CI / 4); e += blockDim.x) {
        const int pix = e / (CI / 4), q = e % (CI / 4);
        const int gy = ty0 + pix / kH - 1, gx = tx0 + pix % kH - 1;
        long long v = 0;
        if (gy >= 0 && gy < S && gx >= 0 && gx < S)
            v = reinterpret_cast<const long long*>(in + (((size_t)b * S + gy) * S + gx) * CI)[q];
        reinterpret_cast<long long*>(sin)[e] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pi = lane & 15, kq = (lane >> 4) * 4;
    constexpr int NT = CO / 16;
    f4_t acc[4][NT];
    for (int r = 0; r < 4; ++r)
        for (int nt = 0; nt < NT; ++nt) acc[r][nt] = f4_t{0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 9; ++t) {
        const int dy = t / 3, dx = t % 3;
        if constexpr (CI % 32 == 0) {
            const int k8 = (lane >> 4) * 8;
            for (int c0 = 0; c0 < CI; c0 += 32) {
                s8_t bw[NT];
                for (int nt = 0; nt < NT; ++nt)
                    bw[nt] = *reinterpret_cast<const s8_t*>(sw + (t * CO + nt * 16 + pi) * CI + c0 + k8);
                for (int r = 0; r < 4; ++r) {
                    const int ly = wave * 4 + r + dy, lx = pi + dx;
                    const s8_t a = *reinterpret_cast<const s8_t*>(sin + (ly * kH + lx) * CI + c0 + k8);
                    for (int nt = 0; nt < NT; ++nt) acc[r][nt] = mfma_k32(a, bw[nt], acc[r][nt]);
                }
            }
        } else {
            for (int c0 = 0; c0 < CI; c0 += 16) {
                s4_t bw[NT];
                for (int nt = 0; nt < NT; ++nt)
                    bw[nt] = *reinterpret_cast<const s4_t*>(sw + (t * CO + nt * 16 + pi) * CI + c0 + kq);
                for (int r = 0; r < 4; ++r) {
                    const int ly = wave * 4 + r + dy, lx = pi + dx;
                    const s4_t a = *reinterpret_cast<const s4_t*>(sin + (ly * kH + lx) * CI + c0 + kq);
                    for (int nt = 0; nt < NT; ++nt)
                        acc[r][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw[nt], acc[r][nt], 0, 0, 0);
                }
            }
        }
    }
    for (int r = 0; r < 4; ++r) {
        const int gy = ty0 + wave * 4 + r;
        if (gy >= S) continue;
        for (int nt = 0; nt < NT; ++nt) {
            const int co = nt * 16 + pi;
            const float bco = (EPI != EPI_BWD && co < co_real) ? bias[co] : 0.f;
            for (int v = 0; v < 4; ++v) {
                const int gx = tx0 + kq + v;
                if (gx >= S) continue;
                const size_t o = (((size_t)b * S + gy) * S + gx) * CO + co;
                const float val = acc[r][nt][v];
                if constexpr (EPI == EPI_RELU || EPI == EPI_RELU_RES) {
                    const float z = val + bco;
                    zout[o] = z;
                    float h = fmaxf(z, 0.f);
                    if constexpr (EPI == EPI_RELU_RES) h += res[o];
                    out32[o] = h;
                    out16[o] = bf16_bits(h);
                } else if constexpr (EPI == EPI_LINEAR) {
                    zout[o] = val + bco;
                } else {
                    const float g = val + (res ? res[o] : 0.f);
                    out32[o] = g;
                    out16[o] = bf16_bits(zmask[o] > 0.f ? g : 0.f);
                }
            }
        }
    }
}

// Weight and bias gradients of one layer, per tile: part[wg][t][co][ci] =
// sum over the tile's pixels p of dz[p][co] in[p + tap t][ci]; part[wg][9 CO CI + co]
// = sum_p dz[p][co].
template <int CI, int CO>
__global__ __launch_bounds__(256) void k_conv_dw(int S, const short* __restrict__ in, const short* __restrict__ dz,
                                                 float* __restrict__ part) {
    __shared__ short sin[kH * kH * CI];
    __shared__ short sdz[kT * kT * CO];
    const int tx0 = blockIdx.x * kT, ty0 = blockIdx.y * kT, b = blockIdx.z;
    const size_t wg = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    for (int e = threadIdx.x; e < kH * kH * (CI / 4); e += blockDim.x) {
        const int pix = e / (CI / 4), q = e % (CI / 4);
        const int gy = ty0 + pix / kH - 1, gx = tx0 + pix % kH - 1;
        long long v = 0;
        if (gy >= 0 && gy < S && gx >= 0 && gx < S)
            v = reinterpret_cast<const long long*>(in + (((size_t)b * S + gy) * S + gx) * CI)[q];
        reinterpret_cast<long long*>(sin)[e] = v;
    }
    for (int e = threadIdx.x; e < kT * kT * (CO / 4); e += blockDim.x) {
        const int pix = e / (CO / 4), q = e % (CO / 4);
        const int gy = ty0 + pix / kT, gx = tx0 + pix % kT;
        long long v = 0;
        if (gy < S && gx < S)
            v = reinterpret_cast<const long long*>(dz + (((size_t)b * S + gy) * S + gx) * CO)[q];
        reinterpret_cast<long long*>(sdz)[e] = v;
    }
    __syncthreads();
    float* pw = part + wg * kWgStride;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int pi = lane & 15, kq = (lane >> 4) * 4;
    constexpr int NCO = CO / 16, NCI = CI / 16, NTILE = 9 * NCO * NCI;
    for (int tile = wave; tile < NTILE; tile += 4) {
        const int t = tile / (NCO * NCI), cot = (tile / NCI) % NCO, cit = tile % NCI;
        const int dy = t / 3, dx = t % 3;
        f4_t acc = {0.f, 0.f, 0.f, 0.f};
        // K = the tile's pixels, 32 (two rows) per step: pixel 32 st + 8 (l / 16) + e
        const int k8 = (lane >> 4) * 8;
        for (int st = 0; st < kT * kT / 32; ++st) {
            const int p0 = 32 * st + k8, rr = p0 / kT, cc = p0 % kT;
            s8_t a, bb;
            for (int e = 0; e < 8; ++e) {
                a[e] = sdz[(p0 + e) * CO + cot * 16 + pi];
                bb[e] = sin[((rr + dy) * kH + cc + e + dx) * CI + cit * 16 + pi];
            }
            acc = mfma_k32(a, bb, acc);
        }
        for (int v = 0; v < 4; ++v) {
            const int co = cot * 16 + kq + v, ci = cit * 16 + pi;
            pw[(t * CO + co) * CI + ci] = acc[v];
        }
    }
    for (int co = threadIdx.x; co < CO; co += blockDim.x) {
        float s = 0.f;
        for (int p = 0; p < kT * kT; ++p) s += bf16_value(sdz[p * CO + co]);
        pw[9 * CO * CI + co] = s;
    }
}

// Sum of the per-tile partials (fixed order) into the packed gradient of a layer.
// Weight and bias gradients from the per-tile partials, in two fixed-order
// stages that read the partials coalesced (index j runs over one tile's
// partial layout [t][co][ci] then the biases):
//   tmp[sp][j] = sum over the tiles of split sp of part[tile][j],
//   then the kDwSplit sums in order, scattered into the packed gradient.
constexpr int kDwSplit = 16;
__global__ void k_dw_partial(int nwg, int J, const float* __restrict__ part, double* __restrict__ tmp) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int sp = blockIdx.y;
    if (j >= J) return;
    const int g0 = (int)((long long)sp * nwg / kDwSplit), g1 = (int)((long long)(sp + 1) * nwg / kDwSplit);
    double s = 0.0;
    for (int g = g0; g < g1; ++g) s += part[(size_t)g * kWgStride + j];
    tmp[(size_t)sp * J + j] = s;
}

__global__ void k_dw_reduce(int J, int co_r, int ci_r, int COp, int CIp, const double* __restrict__ tmp,
                            float* __restrict__ gW, float* __restrict__ gb) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= J) return;
    double s = 0.0;
    for (int sp = 0; sp < kDwSplit; ++sp) s += tmp[(size_t)sp * J + j];
    const int nw = 9 * COp * CIp;
    if (j < nw) {
        const int t = j / (COp * CIp), r = j - t * COp * CIp, co = r / CIp, ci = r - co * CIp;
        if (co < co_r && ci < ci_r) gW[(co * ci_r + ci) * 9 + t] = (float)s;
    } else if (j - nw < co_r) {
        gb[j - nw] = (float)s;
    }
}

// Per-sample partial sums of |y - t|^2 and |t|^2 (grid: chunks x images).
__global__ void k_loss_part(long long np, const float* __restrict__ y, const float* __restrict__ tg,
                            double* __restrict__ part) {
    const int b = blockIdx.y;
    double num = 0.0, den = 0.0;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
        const double yv = y[((size_t)b * np + p) * Cnn::kPadIn], tv = tg[(size_t)b * np + p];
        num += (yv - tv) * (yv - tv);
        den += tv * tv;
    }
    __shared__ double sn[256], sd[256];
    sn[threadIdx.x] = num;
    sd[threadIdx.x] = den;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) {
            a += sn[i];
            c += sd[i];
        }
        part[((size_t)b * gridDim.x + blockIdx.x) * 2] = a;
        part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 1] = c;
    }
}

// dL/dy = 2 (y - t) / (|t|^2 B) in channel 0 of a 16-channel BF16 image; the
// first workgroup of each image records |y - t|^2 / |t|^2.
__global__ void k_loss_grad(int B, long long np, int nchunk, const float* __restrict__ y,
                            const float* __restrict__ tg, const double* __restrict__ part,
                            short* __restrict__ gy, double* __restrict__ ratio) {
    const int b = blockIdx.y;
    double num = 0.0, den = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        num += part[((size_t)b * nchunk + c) * 2];
        den += part[((size_t)b * nchunk + c) * 2 + 1];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ratio[b] = den > 0 ? num / den : 0.0;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const double yv = y[((size_t)b * np + p) * Cnn::kPadIn], tv = tg[(size_t)b * np + p];
    const float g = den > 0 ? (float)(2.0 * (yv - tv) / (den * B)) : 0.f;
    short* o = gy + ((size_t)b * np + p) * Cnn::kPadIn;
    o[0] = bf16_bits(g);
    for (int c = 1; c < Cnn::kPadIn; ++c) o[c] = 0;
}

// Relative energy norm: per pixel d = (y - t) m, (A d) from the 5-point
// stencil (wE, wN, diag) of the target channels 1..3, neighbours outside the
// image zero; A t likewise.  Partials of d^T A d and t^T A t per chunk.
struct EnergyPix {
    double dAd, tAt, Ad;
};

__device__ inline EnergyPix energy_at(int S, long long b, int row, int col, const float* __restrict__ y,
                                      const float* __restrict__ tg, const float* __restrict__ in) {
    const long long np = (long long)S * S;
    const float* t = tg + b * 4 * np;
    const float* wE = t + np;
    const float* wN = t + 2 * np;
    const float* dg = t + 3 * np;
    const float* mk = in + (b * Cnn::kInCh + 2) * np;
    auto dv = [&](int r, int c) -> double {
        const long long p = (long long)r * S + c;
        return ((double)y[(b * np + p) * Cnn::kPadIn] - (double)t[p]) * (double)mk[p];
    };
    auto tv = [&](int r, int c) -> double {
        const long long p = (long long)r * S + c;
        return (double)t[p] * (double)mk[p];
    };
    const long long p = (long long)row * S + col;
    const double d0 = dv(row, col), t0 = tv(row, col);
    double Ad = (double)dg[p] * d0, At = (double)dg[p] * t0;
    if (col + 1 < S) {
        Ad -= (double)wE[p] * dv(row, col + 1);
        At -= (double)wE[p] * tv(row, col + 1);
    }
    if (col > 0) {
        Ad -= (double)wE[p - 1] * dv(row, col - 1);
        At -= (double)wE[p - 1] * tv(row, col - 1);
    }
    if (row + 1 < S) {
        Ad -= (double)wN[p] * dv(row + 1, col);
        At -= (double)wN[p] * tv(row + 1, col);
    }
    if (row > 0) {
        Ad -= (double)wN[p - S] * dv(row - 1, col);
        At -= (double)wN[p - S] * tv(row - 1, col);
    }
    const double m = (double)mk[p];
    return EnergyPix{d0 * Ad * m, t0 * At * m, Ad * m};
}

__global__ void k_energy_part(int S, const float* __restrict__ y, const float* __restrict__ tg,
                              const float* __restrict__ in, double* __restrict__ part) {
    const int b = blockIdx.y;
    const long long np = (long long)S * S;
    double num = 0.0, den = 0.0;
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (long long)gridDim.x * blockDim.x) {
        const EnergyPix e = energy_at(S, b, (int)(p / S), (int)(p % S), y, tg, in);
        num += e.dAd;
        den += e.tAt;
    }
    __shared__ double sn[256], sd[256];
    sn[threadIdx.x] = num;
    sd[threadIdx.x] = den;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) {
            a += sn[i];
            c += sd[i];
        }
        part[((size_t)b * gridDim.x + blockIdx.x) * 2] = a;
        part[((size_t)b * gridDim.x + blockIdx.x) * 2 + 1] = c;
    }
}

// dL/dy = 2 m (A d) / (t^T A t B) in channel 0 of the BF16 gradient image.
__global__ void k_energy_grad(int B, int S, int nchunk, const float* __restrict__ y, const float* __restrict__ tg,
                              const float* __restrict__ in, const double* __restrict__ part,
                              short* __restrict__ gy, double* __restrict__ ratio) {
    const int b = blockIdx.y;
    const long long np = (long long)S * S;
    double num = 0.0, den = 0.0;
    for (int c = 0; c < nchunk; ++c) {
        num += part[((size_t)b * nchunk + c) * 2];
        den += part[((size_t)b * nchunk + c) * 2 + 1];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ratio[b] = den > 0 ? num / den : 0.0;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const EnergyPix e = energy_at(S, b, (int)(p / S), (int)(p % S), y, tg, in);
    const float g = den > 0 ? (float)(2.0 * e.Ad / (den * B)) : 0.f;
    short* o = gy + ((size_t)b * np + p) * Cnn::kPadIn;
    o[0] = bf16_bits(g);
    for (int c = 1; c < Cnn::kPadIn; ++c) o[c] = 0;
}

__global__ void k_adam(int n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float mi = b1 * m[i] + (1.f - b1) * g[i];
    const float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void k_fill_f(int n, float v, float* __restrict__ a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

}  // namespace

Cnn::Cnn(Ctx* ctx) : ctx_(ctx) {
    const int n = nparams();
    theta_.ensure(n);
    grad_.ensure(n);
    m_.ensure(n);
    v_.ensure(n);
    const LayerDesc* L = layers();
    for (int l = 0; l < kLayers; ++l) {
        wf_[l].ensure((size_t)9 * L[l].COp * L[l].CIp);
        wb_[l].ensure((size_t)9 * L[l].COp * L[l].CIp);
    }
    loss_.ensure(1);
    hipStream_t s = ctx_->stream;
    for (DBuf<float>* b : {&theta_, &grad_, &m_, &v_}) {
        k_fill_f<<<ceil_div(n, 256), 256, 0, s>>>(n, 0.f, b->get());
        HINV_LAUNCH_CHECK();
    }
}

int Cnn::nparams() {
    const LayerDesc* L = layers();
    return L[kLayers - 1].boff + L[kLayers - 1].co;
}

void Cnn::set_params(const float* host) {
    const int n = nparams();
    hipStream_t s = ctx_->stream;
    HINV_HIP(hipMemcpyAsync(theta_.get(), host, sizeof(float) * n, hipMemcpyHostToDevice, s));
    k_fill_f<<<ceil_div(n, 256), 256, 0, s>>>(n, 0.f, m_.get());
    k_fill_f<<<ceil_div(n, 256), 256, 0, s>>>(n, 0.f, v_.get());
    HINV_LAUNCH_CHECK();
    HINV_HIP(hipStreamSynchronize(s));
    step_ = 0;
    weights_fresh_ = false;
}

void Cnn::get_params(float* host) const {
    HINV_HIP(hipMemcpyAsync(host, theta_.get(), sizeof(float) * nparams(), hipMemcpyDeviceToHost, ctx_->stream));
    HINV_HIP(hipStreamSynchronize(ctx_->stream));
}

void Cnn::refresh_weights() {
    if (weights_fresh_) return;
    const LayerDesc* L = layers();
    for (int l = 0; l < kLayers; ++l) {
        const int tot = 9 * L[l].COp * L[l].CIp;
        k_weights_prep<<<ceil_div(tot, 256), 256, 0, ctx_->stream>>>(theta_.get() + L[l].woff, L[l].co, L[l].ci,
                                                                     L[l].COp, L[l].CIp, wf_[l].get(),
                                                                     wb_[l].get());
        HINV_LAUNCH_CHECK();
    }
    weights_fresh_ = true;
}

void Cnn::ensure(int B, int S) {
    if (B <= 0 || S <= 0) fail(HINV_EINVAL, "empty image batch");
    if (S > 8193) fail(HINV_EINVAL, "image side above 8193");
    const size_t np = (size_t)B * S * S;
    const int tiles = ceil_div(S, kT);
    const int nwg = tiles * tiles * B;
    if (np > (size_t)B_ * S_ * S_ || nwg > nwg_) {
        in0_.ensure(np * kPadIn);
        for (int l = 0; l < kLayers - 1; ++l) {
            a_[l].ensure(np * kCh);
            h_[l].ensure(np * kCh);
        }
        for (int l = 0; l < kLayers; ++l) z_[l].ensure(np * (l == kLayers - 1 ? kPadIn : kCh));
        for (int i = 0; i < 2; ++i) {
            dz_[i].ensure(np * kCh);
            gh_[i].ensure(np * kCh);
        }
        gy_.ensure(np * kPadIn);
        part_.ensure((size_t)nwg * kWgStride);
        B_ = B;
        S_ = S;
        nwg_ = nwg;
    }
}

void Cnn::run_forward(int B, int S) {
    refresh_weights();
    const LayerDesc* L = layers();
    hipStream_t s = ctx_->stream;
    const int tiles = ceil_div(S, kT);
    const dim3 g(tiles, tiles, B);
    const float* th = theta_.get();
    k_conv<16, 32, EPI_RELU><<<g, 256, 0, s>>>(S, in0_.get(), wf_[0].get(), th + L[0].boff, L[0].co, nullptr,
                                                nullptr, z_[0].get(), h_[0].get(), a_[0].get());
    HINV_LAUNCH_CHECK();
    for (int l = 1; l < kLayers - 1; ++l) {
        k_conv<32, 32, EPI_RELU_RES><<<g, 256, 0, s>>>(S, a_[l - 1].get(), wf_[l].get(), th + L[l].boff, L[l].co,
                                                        h_[l - 1].get(), nullptr, z_[l].get(), h_[l].get(),
                                                        a_[l].get());
        HINV_LAUNCH_CHECK();
    }
    k_conv<32, 16, EPI_LINEAR><<<g, 256, 0, s>>>(S, a_[kLayers - 2].get(), wf_[kLayers - 1].get(),
                                                  th + L[kLayers - 1].boff, L[kLayers - 1].co, nullptr, nullptr,
                                                  z_[kLayers - 1].get(), nullptr, nullptr);
    HINV_LAUNCH_CHECK();
}

void Cnn::forward(int B, int S, const float* in, float* out) {
    ensure(B, S);
    const long long np = (long long)B * S * S;
    k_pack_input<<<(unsigned)ceil_div((int)std::min<long long>(np, 1LL << 30), 256), 256, 0, ctx_->stream>>>(
        B, S, in, in0_.get());
    HINV_LAUNCH_CHECK();
    run_forward(B, S);
    k_unpack_output<<<(unsigned)ceil_div((int)np, 256), 256, 0, ctx_->stream>>>(np, z_[kLayers - 1].get(), out);
    HINV_LAUNCH_CHECK();
}

short* Cnn::packed_input(int S) {
    ensure(1, S);
    return in0_.get();
}

void Cnn::forward_packed(int B, int S) {
    ensure(B, S);
    run_forward(B, S);
}

double Cnn::gradient(int B, int S, const float* in, const float* target, int tchan, float* grad_host) {
    ensure(B, S);
    hipStream_t s = ctx_->stream;
    const long long np = (long long)S * S;
    k_pack_input<<<(unsigned)ceil_div((int)(np * B), 256), 256, 0, s>>>(B, S, in, in0_.get());
    HINV_LAUNCH_CHECK();
    run_forward(B, S);
    // loss and dL/dy
    const int nchunk = std::min(64, ceil_div((int)np, 256));
    lpart_.ensure((size_t)2 * B * nchunk);
    ratio_.ensure(B);
    if (tchan == 1) {
        k_loss_part<<<dim3(nchunk, B), 256, 0, s>>>(np, z_[kLayers - 1].get(), target, lpart_.get());
        HINV_LAUNCH_CHECK();
        k_loss_grad<<<dim3(ceil_div((int)np, 256), B), 256, 0, s>>>(B, np, nchunk, z_[kLayers - 1].get(), target,
                                                                     lpart_.get(), gy_.get(), ratio_.get());
    } else {
        k_energy_part<<<dim3(nchunk, B), 256, 0, s>>>(S, z_[kLayers - 1].get(), target, in, lpart_.get());
        HINV_LAUNCH_CHECK();
        k_energy_grad<<<dim3(ceil_div((int)np, 256), B), 256, 0, s>>>(B, S, nchunk, z_[kLayers - 1].get(), target,
                                                                       in, lpart_.get(), gy_.get(), ratio_.get());
    }
    HINV_LAUNCH_CHECK();
    // backward
    const LayerDesc* L = layers();
    const int tiles = ceil_div(S, kT);
    const dim3 g(tiles, tiles, B);
    const int nwg = tiles * tiles * B;
    float* gr = grad_.get();
    dwtmp_.ensure((size_t)kDwSplit * (9 * 32 * 32 + 32));
    auto reduce = [&](int l) {
        const int J = 9 * L[l].COp * L[l].CIp + L[l].COp;
        k_dw_partial<<<dim3(ceil_div(J, 256), kDwSplit), 256, 0, s>>>(nwg, J, part_.get(), dwtmp_.get());
        HINV_LAUNCH_CHECK();
        k_dw_reduce<<<ceil_div(J, 256), 256, 0, s>>>(J, L[l].co, L[l].ci, L[l].COp, L[l].CIp, dwtmp_.get(),
                                                      gr + L[l].woff, gr + L[l].boff);
        HINV_LAUNCH_CHECK();
    };
    const int top = kLayers - 1;
    k_conv_dw<32, 16><<<g, 256, 0, s>>>(S, a_[top - 1].get(), gy_.get(), part_.get());
    HINV_LAUNCH_CHECK();
    reduce(top);
    // dL/dh4 and dZ4 = dL/dh4 * [z4 > 0]
    k_conv<16, 32, EPI_BWD><<<g, 256, 0, s>>>(S, gy_.get(), wb_[top].get(), nullptr, 0, nullptr,
                                               z_[top - 1].get(), nullptr, gh_[0].get(), dz_[0].get());
    HINV_LAUNCH_CHECK();
    int cur = 0;
    for (int l = top - 1; l >= 1; --l) {
        k_conv_dw<32, 32><<<g, 256, 0, s>>>(S, a_[l - 1].get(), dz_[cur].get(), part_.get());
        HINV_LAUNCH_CHECK();
        reduce(l);
        // dL/dh_{l-1} = conv^T(dZ_l) + dL/dh_l (identity path), dZ_{l-1}
        k_conv<32, 32, EPI_BWD><<<g, 256, 0, s>>>(S, dz_[cur].get(), wb_[l].get(), nullptr, 0, gh_[cur].get(),
                                                   z_[l - 1].get(), nullptr, gh_[1 - cur].get(),
                                                   dz_[1 - cur].get());
        HINV_LAUNCH_CHECK();
        cur = 1 - cur;
    }
    k_conv_dw<16, 32><<<g, 256, 0, s>>>(S, in0_.get(), dz_[cur].get(), part_.get());
    HINV_LAUNCH_CHECK();
    reduce(0);
    std::vector<double> r(B);
    HINV_HIP(hipMemcpyAsync(r.data(), ratio_.get(), sizeof(double) * B, hipMemcpyDeviceToHost, s));
    if (grad_host)
        HINV_HIP(hipMemcpyAsync(grad_host, gr, sizeof(float) * nparams(), hipMemcpyDeviceToHost, s));
    HINV_HIP(hipStreamSynchronize(s));
    double Lsum = 0.0;
    for (double v : r) Lsum += v;
    return Lsum / B;
}

double Cnn::train_step(int B, int S, const float* in, const float* target, int tchan, float lr) {
    const double L = gradient(B, S, in, target, tchan, nullptr);
    ++step_;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, step_)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, step_)));
    const int n = nparams();
    k_adam<<<ceil_div(n, 256), 256, 0, ctx_->stream>>>(n, theta_.get(), grad_.get(), m_.get(), v_.get(), lr, c1, c2);
    HINV_LAUNCH_CHECK();
    weights_fresh_ = false;
    return L;
}

}  // namespace hinv
