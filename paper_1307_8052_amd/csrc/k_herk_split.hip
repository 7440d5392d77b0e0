// Split-precision grouped rank-k update of chi0 (Eq. zher_multi) on BF16 or
// FP16 MFMA.
//
// chi0(w) += X_w rho^H with X_w = rho diag(a(w)): every FP32 operand value x is
// split as x = hi + lo with hi = round16(x), lo = round16(x - hi), and each
// real product is formed as hi*hi' + hi*lo' + lo*hi' on
// v_mfma_f32_16x16x32_{bf16,f16} with FP32 accumulation. Every kFlush K-steps
// the FP32 accumulators are added into FP64 registers and cleared, so the FP32
// rounding of a long pair sum does not grow with the number of pairs; the FP64
// tile is added to the FP64 chi0 accumulator at the end of the pair chunk. A
// complex product needs four real ones: Re = Xr Br^T + Xi Bi^T,
// Im = Xi Br^T - Xr Bi^T.
//
// FP16 keeps 11 significant bits per half (BF16 keeps 8) but has a narrow
// exponent range, so both operands are multiplied by powers of two that put
// their largest element near 2^14 (k_split_scales) and the tile is divided by
// the product afterwards (exact).
#include "internal.hpp"

namespace rpa {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

// Sign flip of eight 16-bit floats held in four registers: one XOR per register (negating the vector as
// a value compiles to three instructions per register). Exact, as negation is.
template <typename V>
__device__ __forceinline__ V neg8(V v) {
    typedef unsigned v4u32 __attribute__((ext_vector_type(4)));
    const v4u32 s = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    return __builtin_bit_cast(V, __builtin_bit_cast(v4u32, v) ^ s);
}

constexpr int kBK = 32;          // K per MFMA
constexpr int kFlush = 8;        // K-steps between FP64 flushes of the accumulators
constexpr int kLd = kBK + 8;     // LDS row stride (elements): 80 bytes, keeps 16-byte alignment

template <bool F16>
struct Half;

template <>
struct Half<false> {
    typedef __bf16 t;
    typedef v8bf v8;
    static __device__ __forceinline__ void split(float x, t& hi, t& lo) {
        hi = (__bf16)x;
        lo = (__bf16)(x - (float)hi);
    }
    static __device__ __forceinline__ v4f mfma(v8 a, v8 b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

template <>
struct Half<true> {
    typedef _Float16 t;
    typedef v8h v8;
    static __device__ __forceinline__ void split(float x, t& hi, t& lo) {
        hi = (_Float16)x;
        lo = (_Float16)(x - (float)hi);
    }
    static __device__ __forceinline__ v4f mfma(v8 a, v8 b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

__device__ __forceinline__ void tile_of(int t, int& I, int& J) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
}

// One 64x64 lower tile of one frequency per workgroup; four waves, each a
// 32x32 quadrant as 2x2 blocks of 16x16. Fragment layout of the 16x16x32
// MFMA: A lane l holds A[l%16][8*(l/16) .. +7], B lane l holds
// B[8*(l/16) .. +7][l%16], D lane l element r holds D[4*(l/16)+r][l%16].
// LDS tiles are [row][k] so each lane reads its 8 k values as one 16-byte word.
template <bool F16>
__global__ __launch_bounds__(256) void k_herk_split(HerkSplitArgs h) {
    typedef typename Half<F16>::t ht;
    typedef typename Half<F16>::v8 hv;
    // [operand A/B][re/im][hi/lo][64][kLd]
    __shared__ __align__(16) ht s[2][2][2][kTile][kLd];
    int I, J;
    tile_of(blockIdx.x, I, J);
    const int w = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int ci = I * kTile, cj = J * kTile;
    const double* aw = h.w + (size_t)w * h.lda;
    const float sa = (F16 && h.wscale) ? h.wscale[w] : 1.0f;
    const float sb = (F16 && h.wscale) ? h.wscale[h.nw] : 1.0f;
    v4f accR[2][2], accI[2][2];
    double totR[2][2][4], totI[2][2][4];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) {
            accR[x][y] = v4f{0, 0, 0, 0};
            accI[x][y] = v4f{0, 0, 0, 0};
            for (int r = 0; r < 4; ++r) totR[x][y][r] = totI[x][y][r] = 0.0;
        }
    int steps = 0;
    for (int k0 = 0; k0 < h.K; k0 += kBK) {
        // 32 (k) x 64 (column) per operand; thread -> (k, 4 consecutive columns)
        for (int e = tid; e < kBK * kTile; e += 256) {
            const int kk = e >> 6, c = e & 63, k = k0 + kk;
            float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
            if (k < h.K) {
                const size_t row = (size_t)k * h.ldA;
                const float wk = (float)aw[k] * sa;
                ar = h.Are[row + ci + c] * wk;
                ai = h.Aim[row + ci + c] * wk;
                br = h.Are[row + cj + c] * sb;
                bi = h.Aim[row + cj + c] * sb;
            }
            Half<F16>::split(ar, s[0][0][0][c][kk], s[0][0][1][c][kk]);
            Half<F16>::split(ai, s[0][1][0][c][kk], s[0][1][1][c][kk]);
            Half<F16>::split(br, s[1][0][0][c][kk], s[1][0][1][c][kk]);
            Half<F16>::split(bi, s[1][1][0][c][kk], s[1][1][1][c][kk]);
        }
        __syncthreads();
        const int kq = 8 * (lane >> 4), rr = lane & 15;
        hv a[2][2][2], b[2][2][2];  // [block][re/im][hi/lo]
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    a[x][c][l] = *reinterpret_cast<const hv*>(&s[0][c][l][wr + x * 16 + rr][kq]);
                    b[x][c][l] = *reinterpret_cast<const hv*>(&s[1][c][l][wc + x * 16 + rr][kq]);
                }
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            hv nar[2];
#pragma unroll
            for (int l = 0; l < 2; ++l) nar[l] = neg8(a[x][0][l]);
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                v4f r = accR[x][y], im = accI[x][y];
                // Re += Xr Br + Xi Bi
                r = Half<F16>::mfma(a[x][0][0], b[y][0][0], r);
                r = Half<F16>::mfma(a[x][0][0], b[y][0][1], r);
                r = Half<F16>::mfma(a[x][0][1], b[y][0][0], r);
                r = Half<F16>::mfma(a[x][1][0], b[y][1][0], r);
                r = Half<F16>::mfma(a[x][1][0], b[y][1][1], r);
                r = Half<F16>::mfma(a[x][1][1], b[y][1][0], r);
                // Im += Xi Br - Xr Bi
                im = Half<F16>::mfma(a[x][1][0], b[y][0][0], im);
                im = Half<F16>::mfma(a[x][1][0], b[y][0][1], im);
                im = Half<F16>::mfma(a[x][1][1], b[y][0][0], im);
                im = Half<F16>::mfma(nar[0], b[y][1][0], im);
                im = Half<F16>::mfma(nar[0], b[y][1][1], im);
                im = Half<F16>::mfma(nar[1], b[y][1][0], im);
                accR[x][y] = r;
                accI[x][y] = im;
            }
        }
        if (++steps == kFlush || k0 + kBK >= h.K) {
            steps = 0;
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        totR[x][y][r] += (double)accR[x][y][r];
                        totI[x][y][r] += (double)accI[x][y][r];
                    }
                    accR[x][y] = v4f{0, 0, 0, 0};
                    accI[x][y] = v4f{0, 0, 0, 0};
                }
        }
        __syncthreads();
    }
    const double inv = 1.0 / ((double)sa * (double)sb);
    double* Cre = h.Cre + (size_t)w * h.sC;
    double* Cim = h.Cim + (size_t)w * h.sC;
    // C += acc, one row block x at a time: all loads of the block are issued before its stores (which
    // could alias them as far as the compiler knows)
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        double cre[2][4], cim[2][4];
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ci + wr + x * 16 + 4 * (lane >> 4) + r;
                const int col = cj + wc + y * 16 + (lane & 15);
                const size_t o = (size_t)row * h.ldC + col;
                cre[y][r] = Cre[o];
                cim[y][r] = Cim[o];
            }
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ci + wr + x * 16 + 4 * (lane >> 4) + r;
                const int col = cj + wc + y * 16 + (lane & 15);
                const size_t o = (size_t)row * h.ldC + col;
                Cre[o] = cre[y][r] + totR[x][y][r] * inv;
                Cim[o] = cim[y][r] + totI[x][y][r] * inv;
            }
    }
}

// Power-of-two operand scales for the FP16 split: scales[w] for X_w = rho a(w)
// and scales[nw] for rho, each putting the largest magnitude in [2^13, 2^14).
// Pass 1: per-block maxima of |rho| (re and im parts) and of |a(w)|.
__global__ void k_absmax_rho(const float* __restrict__ rre, const float* __restrict__ rim, size_t n,
                             float* __restrict__ part) {
    __shared__ float red[256];
    float m = 0.f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fmaxf(fabsf(rre[i]), fabsf(rim[i])));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__device__ __forceinline__ float pow2_scale(float maxabs) {
    if (!(maxabs > 0.f) || !isfinite(maxabs)) return 1.0f;
    int e;
    frexpf(maxabs, &e);   // maxabs in [2^(e-1), 2^e)
    return ldexpf(1.0f, 14 - e);
}

// Pass 2: one block per frequency (max |a|) plus one for rho; writes the scales.
__global__ void k_split_scales(const float* __restrict__ part, int nparts, const double* __restrict__ a, int lda,
                               int K, int nw, float* __restrict__ scales) {
    __shared__ float red[256];
    const int b = blockIdx.x;
    float m = 0.f;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmaxf(m, part[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    const float rmax = red[0];
    __syncthreads();
    if (b == nw) {
        if (threadIdx.x == 0) scales[nw] = pow2_scale(rmax);
        return;
    }
    float am = 0.f;
    for (int k = threadIdx.x; k < K; k += blockDim.x) am = fmaxf(am, (float)fabs(a[(size_t)b * lda + k]));
    red[threadIdx.x] = am;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scales[b] = pow2_scale(red[0] * rmax);
}

}  // namespace

constexpr int kScaleParts = 256;

hipError_t launch_split_scales(const float* rre, const float* rim, size_t n, const double* a, int lda, int K, int nw,
                               float* scales, float* part, hipStream_t s) {
    hipLaunchKernelGGL(k_absmax_rho, dim3(kScaleParts), dim3(256), 0, s, rre, rim, n, part);
    hipLaunchKernelGGL(k_split_scales, dim3((unsigned)nw + 1), dim3(256), 0, s, part, kScaleParts, a, lda, K, nw,
                       scales);
    return hipGetLastError();
}

hipError_t launch_herk_split(const HerkSplitArgs& h, hipStream_t s) {
    if (h.nT <= 0 || h.nw <= 0 || h.K <= 0) return hipSuccess;
    const unsigned ntiles = (unsigned)(h.nT * (h.nT + 1) / 2);
    if (h.fp16)
        hipLaunchKernelGGL(k_herk_split<true>, dim3(ntiles, (unsigned)h.nw), dim3(256), 0, s, h);
    else
        hipLaunchKernelGGL(k_herk_split<false>, dim3(ntiles, (unsigned)h.nw), dim3(256), 0, s, h);
    return hipGetLastError();
}

}  // namespace rpa
