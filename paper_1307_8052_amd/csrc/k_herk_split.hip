// Split-precision grouped rank-k update of chi0 (Eq. zher_multi) on BF16 or
// FP16 MFMA.
//
// chi0(w) += X_w rho^H with X_w = rho diag(a(w)): every FP32 operand value x is
// split as x = hi + lo with hi = round16(x), lo = round16(x - hi), and each
// real product is formed as hi*hi' + hi*lo' + lo*hi' on
// v_mfma_f32_16x16x32_{bf16,f16} with FP32 accumulation; the tile is added to
// the FP64 chi0 accumulator at the end of the pair chunk. A complex product
// needs four real ones: Re = Xr Br^T + Xi Bi^T, Im = Xi Br^T - Xr Bi^T.
//
// FP16 keeps 11 significant bits per half (BF16 keeps 8) but has a narrow
// exponent range, so X_w is multiplied by a per-frequency power of two before
// the split and the tile by its inverse afterwards.
#include "internal.hpp"

namespace rpa {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int kBK = 32;          // K per MFMA
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
    const float sc = (F16 && h.wscale) ? h.wscale[w] : 1.0f;
    v4f accR[2][2], accI[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) {
            accR[x][y] = v4f{0, 0, 0, 0};
            accI[x][y] = v4f{0, 0, 0, 0};
        }
    for (int k0 = 0; k0 < h.K; k0 += kBK) {
        // 32 (k) x 64 (column) per operand; thread -> (k, 4 consecutive columns)
        for (int e = tid; e < kBK * kTile; e += 256) {
            const int kk = e >> 6, c = e & 63, k = k0 + kk;
            float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
            if (k < h.K) {
                const size_t row = (size_t)k * h.ldA;
                const float wk = (float)aw[k] * sc;
                ar = h.Are[row + ci + c] * wk;
                ai = h.Aim[row + ci + c] * wk;
                br = h.Are[row + cj + c];
                bi = h.Aim[row + cj + c];
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
            for (int l = 0; l < 2; ++l) nar[l] = -a[x][0][l];
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
        __syncthreads();
    }
    const double inv = 1.0 / (double)sc;
    double* Cre = h.Cre + (size_t)w * h.sC;
    double* Cim = h.Cim + (size_t)w * h.sC;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ci + wr + x * 16 + 4 * (lane >> 4) + r;
                const int col = cj + wc + y * 16 + (lane & 15);
                const size_t o = (size_t)row * h.ldC + col;
                Cre[o] += (double)accR[x][y][r] * inv;
                Cim[o] += (double)accI[x][y][r] * inv;
            }
}

}  // namespace

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
