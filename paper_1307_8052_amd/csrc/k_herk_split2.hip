// Split-precision grouped rank-k update of chi0 (Eq. zher_multi), large-tile
// form.
//
// Per pair chunk, k_pack_split rewrites rho once into two K-blocked copies,
// [K/32][NGq][32] with the 32 pairs of a block contiguous per G:
//   X  FP32 (re, im), the operand that each frequency scales by a(w);
//   B  16-bit hi/lo (re_hi, re_lo, im_hi, im_lo) of rho, split once.
// k_herk_split4 / k_herk_split5 then compute one 64x128 lower tile of chi0(w)
// per workgroup: every K-step they load 32 pairs of X, multiply by a(w), split
// into hi/lo in registers and stage both operands in LDS, and issue 12
// v_mfma_f32_16x16x32 per 16x16 block (Re = Xr Br^T + Xi Bi^T,
// Im = Xi Br^T - Xr Bi^T, three split products each).
//
// Workgroups are numbered so that the nw frequencies of one tile go to the
// same XCD (consecutive workgroup ids are dealt round-robin to the 8 XCDs),
// so the operand rows of a tile are fetched into one L2 and reused nw times.
#include "internal.hpp"

namespace rpa {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned short u16;
typedef u16 v8u16 __attribute__((ext_vector_type(8)));

constexpr int TM = 128;       // workgroup tile edge
constexpr int KS = 32;        // pairs per K-step (MFMA K)
constexpr int LDR = 40;       // LDS row stride in 16-bit elements (80 bytes)
constexpr int kXcds = 8;

template <bool F16> struct H;
template <> struct H<false> {
    typedef v8bf v8;
    static __device__ __forceinline__ u16 bits(float x) {
        __bf16 h = (__bf16)x;
        return __builtin_bit_cast(u16, h);
    }
    static __device__ __forceinline__ float back(u16 b) { return (float)__builtin_bit_cast(__bf16, b); }
    static __device__ __forceinline__ v4f mfma(v8 a, v8 b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct H<true> {
    typedef v8h v8;
    static __device__ __forceinline__ u16 bits(float x) {
        _Float16 h = (_Float16)x;
        return __builtin_bit_cast(u16, h);
    }
    static __device__ __forceinline__ float back(u16 b) { return (float)__builtin_bit_cast(_Float16, b); }
    static __device__ __forceinline__ v4f mfma(v8 a, v8 b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

// Sign flip of eight 16-bit floats held in four registers: one XOR per register (negating the vector as
// a value compiles to three instructions per register). Exact, as negation is.
template <typename V>
__device__ __forceinline__ V neg8(V v) {
    typedef unsigned v4u32 __attribute__((ext_vector_type(4)));
    const v4u32 s = {0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
    return __builtin_bit_cast(V, __builtin_bit_cast(v4u32, v) ^ s);
}

template <bool F16>
__device__ __forceinline__ void split(float x, u16& hi, u16& lo) {
    hi = H<F16>::bits(x);
    lo = H<F16>::bits(x - H<F16>::back(hi));
}

// rho planar [K][ldr] -> X blocked FP32 and B blocked 16-bit hi/lo; one
// workgroup per (64 G, 32 pairs); entries past K or past ldr are zero.
template <bool F16>
__global__ __launch_bounds__(256) void k_pack_split(const float* __restrict__ rre, const float* __restrict__ rim,
                                                     int K, int ldr, int NGq, const float* __restrict__ scales,
                                                     int nw, float* __restrict__ Xre, float* __restrict__ Xim,
                                                     u16* __restrict__ B0, u16* __restrict__ B1,
                                                     u16* __restrict__ B2, u16* __restrict__ B3) {
    __shared__ float tr[KS][65], ti[KS][65];
    const int g0 = blockIdx.x * 64, kb = blockIdx.y, k0 = kb * KS;
    const int tid = threadIdx.x;
    for (int e = tid; e < KS * 64; e += 256) {
        const int kk = e >> 6, c = e & 63, k = k0 + kk, g = g0 + c;
        float vr = 0.f, vi = 0.f;
        if (k < K && g < ldr) {
            vr = rre[(size_t)k * ldr + g];
            vi = rim[(size_t)k * ldr + g];
        }
        tr[kk][c] = vr;
        ti[kk][c] = vi;
    }
    __syncthreads();
    const float sb = (F16 && scales) ? scales[nw] : 1.0f;
    const int c = tid >> 2, kq = (tid & 3) * 8;
    const size_t o = ((size_t)kb * NGq + g0 + c) * KS + kq;
    v8u16 hr, lr, hi_, li;
    float xr[8], xi[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        xr[e] = tr[kq + e][c];
        xi[e] = ti[kq + e][c];
        u16 a, b;
        split<F16>(xr[e] * sb, a, b);
        hr[e] = a;
        lr[e] = b;
        split<F16>(xi[e] * sb, a, b);
        hi_[e] = a;
        li[e] = b;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        Xre[o + e] = xr[e];
        Xim[o + e] = xi[e];
    }
    *reinterpret_cast<v8u16*>(B0 + o) = hr;
    *reinterpret_cast<v8u16*>(B1 + o) = lr;
    *reinterpret_cast<v8u16*>(B2 + o) = hi_;
    *reinterpret_cast<v8u16*>(B3 + o) = li;
}

// Variant 4: a software-pipelined K loop with FP64 accumulation. LDS holds two
// K-steps (double buffer with an XOR swizzle of the 16-byte chunks of a row
// instead of padding), so one barrier per K-step separates writing step k+1
// from reading step k, and the global loads of step k+1 are in flight while
// the MFMAs of step k run. A workgroup computes a 64-row x 128-column tile
// (each wave all 64 rows x 32 columns); the MFMAs accumulate in FP32 for 8
// K-steps (256 pairs), then the partial sums are added into FP64 registers,
// which bounds the FP32 rounding of the long sum over pairs. The 64-row side
// is the one scaled by a(w) and split in the kernel. Row block I of the
// lower triangle holds column blocks 0 .. I/2.
constexpr int kFlush4 = 8;

// LDS offset (in 16-bit elements) of 16-byte chunk `chunk` of row `row`: an XOR swizzle of the chunks of
// a row so that the fragment reads of a K-step spread over the banks without padding
__device__ __forceinline__ int swz(int row, int chunk) { return 8 * (chunk ^ ((row >> 1) & 3)); }

template <bool F16>
__global__ __launch_bounds__(256, 1) void k_herk_split4(HerkSplit2Args h) {
    typedef typename H<F16>::v8 hv;
    constexpr int TR = 64, TC = 128;
    __shared__ __align__(16) u16 sA[2][4][TR][KS];
    __shared__ __align__(16) u16 sB[2][4][TC][KS];

    const int b = blockIdx.x;
    const int xcd = b % kXcds, local = b / kXcds;
    const int tile = (local / h.nw) * kXcds + xcd;
    const int w = local % h.nw;
    if (tile >= h.ntiles) return;
    int I = 0, t = tile;
    while (t >= I / 2 + 1) {
        t -= I / 2 + 1;
        ++I;
    }
    const int ci = I * TR, cj = t * TC;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wc = wave * 32;
    const double* aw = h.w + (size_t)w * h.lda;
    const float sa = (F16 && h.scales) ? h.scales[w] : 1.0f;
    const float sb = (F16 && h.scales) ? h.scales[h.nw] : 1.0f;
    const int K = h.K;

    // staging: A row ar, pairs ak .. ak+7; B row br, pairs bk .. bk+15
    const int ar = tid >> 2, ak = (tid & 3) * 8;
    const int br = tid >> 1, bk = (tid & 1) * 16;
    float pxr[8], pxi[8];
    double pw[8];
    v8u16 pb[4][2];
    const int nkb = (K + KS - 1) / KS;
    auto fetch = [&](int kb) {
        const size_t oa = ((size_t)kb * h.NGq + ci + ar) * KS + ak;
        const size_t ob = ((size_t)kb * h.NGq + cj + br) * KS + bk;
#pragma unroll
        for (int e = 0; e < 8; e += 4) {
            const v4f a = *reinterpret_cast<const v4f*>(h.Xre + oa + e);
            const v4f c = *reinterpret_cast<const v4f*>(h.Xim + oa + e);
            pxr[e] = a[0]; pxr[e + 1] = a[1]; pxr[e + 2] = a[2]; pxr[e + 3] = a[3];
            pxi[e] = c[0]; pxi[e + 1] = c[1]; pxi[e + 2] = c[2]; pxi[e + 3] = c[3];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pb[q][0] = *reinterpret_cast<const v8u16*>(h.B[q] + ob);
            pb[q][1] = *reinterpret_cast<const v8u16*>(h.B[q] + ob + 8);
        }
        const int k0 = kb * KS + ak;
#pragma unroll
        for (int e = 0; e < 8; ++e) pw[e] = aw[min(k0 + e, K - 1)];
    };
    auto store = [&](int kb, int buf) {
        const int k0 = kb * KS + ak;
        v8u16 xrh, xrl, xih, xil;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float wk = (k0 + e < K) ? (float)pw[e] * sa : 0.f;
            u16 a, c;
            split<F16>(pxr[e] * wk, a, c);
            xrh[e] = a;
            xrl[e] = c;
            split<F16>(pxi[e] * wk, a, c);
            xih[e] = a;
            xil[e] = c;
        }
        const int oa = swz(ar, ak >> 3);
        *reinterpret_cast<v8u16*>(&sA[buf][0][ar][oa]) = xrh;
        *reinterpret_cast<v8u16*>(&sA[buf][1][ar][oa]) = xrl;
        *reinterpret_cast<v8u16*>(&sA[buf][2][ar][oa]) = xih;
        *reinterpret_cast<v8u16*>(&sA[buf][3][ar][oa]) = xil;
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            const int ob = swz(br, (bk >> 3) + hf);
#pragma unroll
            for (int q = 0; q < 4; ++q) *reinterpret_cast<v8u16*>(&sB[buf][q][br][ob]) = pb[q][hf];
        }
    };

    v4f accR[4][2], accI[4][2];
    double dR[4][2][4], dI[4][2][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            accR[x][y] = v4f{0, 0, 0, 0};
            accI[x][y] = v4f{0, 0, 0, 0};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                dR[x][y][r] = 0.0;
                dI[x][y][r] = 0.0;
            }
        }
    auto flush = [&]() {
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    dR[x][y][r] += (double)accR[x][y][r];
                    dI[x][y][r] += (double)accI[x][y][r];
                }
                accR[x][y] = v4f{0, 0, 0, 0};
                accI[x][y] = v4f{0, 0, 0, 0};
            }
    };

    fetch(0);
    store(0, 0);
    fetch(min(1, nkb - 1));
    const int rr = lane & 15, kc = lane >> 4;
    for (int kb = 0; kb < nkb; ++kb) {
        __syncthreads();
        const int cur = kb & 1;
        hv bf[2][4], bn[2][2];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int row = wc + 16 * y + rr;
            const int o = swz(row, kc);
#pragma unroll
            for (int q = 0; q < 4; ++q) bf[y][q] = *reinterpret_cast<const hv*>(&sB[cur][q][row][o]);
            bn[y][0] = neg8(bf[y][2]);
            bn[y][1] = neg8(bf[y][3]);
        }
        hv af[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const int row = 16 * x + rr;
            const int o = swz(row, kc);
#pragma unroll
            for (int q = 0; q < 4; ++q) af[x][q] = *reinterpret_cast<const hv*>(&sA[cur][q][row][o]);
        }
        store(kb + 1, cur ^ 1);
        fetch(min(kb + 2, nkb - 1));
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                v4f r = accR[x][y], im = accI[x][y];
                r = H<F16>::mfma(af[x][1], bf[y][0], r);
                r = H<F16>::mfma(af[x][0], bf[y][1], r);
                r = H<F16>::mfma(af[x][3], bf[y][2], r);
                r = H<F16>::mfma(af[x][2], bf[y][3], r);
                r = H<F16>::mfma(af[x][0], bf[y][0], r);
                r = H<F16>::mfma(af[x][2], bf[y][2], r);
                im = H<F16>::mfma(af[x][3], bf[y][0], im);
                im = H<F16>::mfma(af[x][2], bf[y][1], im);
                im = H<F16>::mfma(af[x][1], bn[y][0], im);
                im = H<F16>::mfma(af[x][0], bn[y][1], im);
                im = H<F16>::mfma(af[x][2], bf[y][0], im);
                im = H<F16>::mfma(af[x][0], bn[y][0], im);
                accR[x][y] = r;
                accI[x][y] = im;
            }
        if ((kb & (kFlush4 - 1)) == kFlush4 - 1) flush();
    }
    flush();

    const double inv = 1.0 / ((double)sa * (double)sb);
    double* Cre = h.Cre + (size_t)w * h.sC;
    double* Cim = h.Cim + (size_t)w * h.sC;
    // C += acc (C = acc for the first update of a fresh accumulator: nothing read), one row block x at a
    // time: all loads of the block are issued before its stores (which could alias them as far as the
    // compiler knows); rows and columns past ldC read a valid address
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        double cre[2][4] = {}, cim[2][4] = {};
        if (!h.overwrite) {
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = ci + 16 * x + 4 * (lane >> 4) + r;
                    const int col = cj + wc + 16 * y + (lane & 15);
                    const size_t o = (row < h.ldC && col < h.ldC) ? (size_t)row * h.ldC + col : 0;
                    cre[y][r] = Cre[o];
                    cim[y][r] = Cim[o];
                }
        }
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ci + 16 * x + 4 * (lane >> 4) + r;
                const int col = cj + wc + 16 * y + (lane & 15);
                if (row < h.ldC && col < h.ldC) {
                    const size_t o = (size_t)row * h.ldC + col;
                    Cre[o] = cre[y][r] + dR[x][y][r] * inv;
                    Cim[o] = cim[y][r] + dI[x][y][r] * inv;
                }
            }
    }
}

// Variant 5: the tiles, operands and FP64 accumulation of variant 4 with eight
// waves per workgroup (two per SIMD), each a 32 x 32 sub-tile, so that one wave's
// MFMAs overlap the other's split, LDS and global traffic. Each thread stages
// 4 pairs of one row of the 64-row side and 8 pairs of one row of the other.
typedef u16 v4u16 __attribute__((ext_vector_type(4)));

template <bool F16>
__global__ __launch_bounds__(512, 1) void k_herk_split5(HerkSplit2Args h) {
    typedef typename H<F16>::v8 hv;
    constexpr int TR = 64, TC = 128;
    __shared__ __align__(16) u16 sA[2][4][TR][KS];
    __shared__ __align__(16) u16 sB[2][4][TC][KS];

    const int b = blockIdx.x;
    const int xcd = b % kXcds, local = b / kXcds;
    const int tile = (local / h.nw) * kXcds + xcd;
    const int w = local % h.nw;
    if (tile >= h.ntiles) return;
    int I = 0, t = tile;
    while (t >= I / 2 + 1) {
        t -= I / 2 + 1;
        ++I;
    }
    const int ci = I * TR, cj = t * TC;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 2) * 32, wc = (wave & 3) * 32;
    const double* aw = h.w + (size_t)w * h.lda;
    const float sa = (F16 && h.scales) ? h.scales[w] : 1.0f;
    const float sb = (F16 && h.scales) ? h.scales[h.nw] : 1.0f;
    const int K = h.K;

    // staging: A row ar, pairs ak .. ak+3; B row br, pairs bk .. bk+7
    const int ar = tid >> 3, ak = (tid & 7) * 4;
    const int br = tid >> 2, bk = (tid & 3) * 8;
    v4f pxr, pxi;
    double pw[4];
    v8u16 pb[4];
    const int nkb = (K + KS - 1) / KS;
    auto fetch = [&](int kb) {
        const size_t oa = ((size_t)kb * h.NGq + ci + ar) * KS + ak;
        const size_t ob = ((size_t)kb * h.NGq + cj + br) * KS + bk;
        pxr = *reinterpret_cast<const v4f*>(h.Xre + oa);
        pxi = *reinterpret_cast<const v4f*>(h.Xim + oa);
#pragma unroll
        for (int q = 0; q < 4; ++q) pb[q] = *reinterpret_cast<const v8u16*>(h.B[q] + ob);
        const int k0 = kb * KS + ak;
#pragma unroll
        for (int e = 0; e < 4; ++e) pw[e] = aw[min(k0 + e, K - 1)];
    };
    auto store = [&](int kb, int buf) {
        const int k0 = kb * KS + ak;
        v4u16 xrh, xrl, xih, xil;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float wk = (k0 + e < K) ? (float)pw[e] * sa : 0.f;
            u16 a, c;
            split<F16>(pxr[e] * wk, a, c);
            xrh[e] = a;
            xrl[e] = c;
            split<F16>(pxi[e] * wk, a, c);
            xih[e] = a;
            xil[e] = c;
        }
        const int oa = swz(ar, ak >> 3) + (ak & 7);
        *reinterpret_cast<v4u16*>(&sA[buf][0][ar][oa]) = xrh;
        *reinterpret_cast<v4u16*>(&sA[buf][1][ar][oa]) = xrl;
        *reinterpret_cast<v4u16*>(&sA[buf][2][ar][oa]) = xih;
        *reinterpret_cast<v4u16*>(&sA[buf][3][ar][oa]) = xil;
        const int ob = swz(br, bk >> 3);
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<v8u16*>(&sB[buf][q][br][ob]) = pb[q];
    };

    v4f accR[2][2], accI[2][2];
    double dR[2][2][4], dI[2][2][4];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            accR[x][y] = v4f{0, 0, 0, 0};
            accI[x][y] = v4f{0, 0, 0, 0};
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                dR[x][y][r] = 0.0;
                dI[x][y][r] = 0.0;
            }
        }
    auto flush = [&]() {
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    dR[x][y][r] += (double)accR[x][y][r];
                    dI[x][y][r] += (double)accI[x][y][r];
                }
                accR[x][y] = v4f{0, 0, 0, 0};
                accI[x][y] = v4f{0, 0, 0, 0};
            }
    };

    fetch(0);
    store(0, 0);
    fetch(min(1, nkb - 1));
    const int rr = lane & 15, kc = lane >> 4;
    for (int kb = 0; kb < nkb; ++kb) {
        __syncthreads();
        const int cur = kb & 1;
        hv bf[2][4], bn[2][2];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int row = wc + 16 * y + rr;
            const int o = swz(row, kc);
#pragma unroll
            for (int q = 0; q < 4; ++q) bf[y][q] = *reinterpret_cast<const hv*>(&sB[cur][q][row][o]);
            bn[y][0] = neg8(bf[y][2]);
            bn[y][1] = neg8(bf[y][3]);
        }
        hv af[2][4];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const int row = wr + 16 * x + rr;
            const int o = swz(row, kc);
#pragma unroll
            for (int q = 0; q < 4; ++q) af[x][q] = *reinterpret_cast<const hv*>(&sA[cur][q][row][o]);
        }
        store(kb + 1, cur ^ 1);
        fetch(min(kb + 2, nkb - 1));
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                v4f r = accR[x][y], im = accI[x][y];
                r = H<F16>::mfma(af[x][1], bf[y][0], r);
                r = H<F16>::mfma(af[x][0], bf[y][1], r);
                r = H<F16>::mfma(af[x][3], bf[y][2], r);
                r = H<F16>::mfma(af[x][2], bf[y][3], r);
                r = H<F16>::mfma(af[x][0], bf[y][0], r);
                r = H<F16>::mfma(af[x][2], bf[y][2], r);
                im = H<F16>::mfma(af[x][3], bf[y][0], im);
                im = H<F16>::mfma(af[x][2], bf[y][1], im);
                im = H<F16>::mfma(af[x][1], bn[y][0], im);
                im = H<F16>::mfma(af[x][0], bn[y][1], im);
                im = H<F16>::mfma(af[x][2], bf[y][0], im);
                im = H<F16>::mfma(af[x][0], bn[y][0], im);
                accR[x][y] = r;
                accI[x][y] = im;
            }
        if ((kb & (kFlush4 - 1)) == kFlush4 - 1) flush();
    }
    flush();

    const double inv = 1.0 / ((double)sa * (double)sb);
    double* Cre = h.Cre + (size_t)w * h.sC;
    double* Cim = h.Cim + (size_t)w * h.sC;
    // C += acc (C = acc for the first update of a fresh accumulator: nothing read), one row block x at a
    // time: all loads of the block are issued before its stores (which could alias them as far as the
    // compiler knows); rows and columns past ldC read a valid address
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        double cre[2][4] = {}, cim[2][4] = {};
        if (!h.overwrite) {
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = ci + wr + 16 * x + 4 * (lane >> 4) + r;
                    const int col = cj + wc + 16 * y + (lane & 15);
                    const size_t o = (row < h.ldC && col < h.ldC) ? (size_t)row * h.ldC + col : 0;
                    cre[y][r] = Cre[o];
                    cim[y][r] = Cim[o];
                }
        }
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = ci + wr + 16 * x + 4 * (lane >> 4) + r;
                const int col = cj + wc + 16 * y + (lane & 15);
                if (row < h.ldC && col < h.ldC) {
                    const size_t o = (size_t)row * h.ldC + col;
                    Cre[o] = cre[y][r] + dR[x][y][r] * inv;
                    Cim[o] = cim[y][r] + dI[x][y][r] * inv;
                }
            }
    }
}


}  // namespace

hipError_t launch_pack_split(const float* rre, const float* rim, int K, int ldr, int NGq, const float* scales, int nw,
                             int fp16, float* Xre, float* Xim, u16* const B[4], hipStream_t s) {
    if (K <= 0) return hipSuccess;
    dim3 grid((unsigned)(NGq / 64), (unsigned)((K + KS - 1) / KS));
    if (fp16)
        hipLaunchKernelGGL(k_pack_split<true>, grid, dim3(256), 0, s, rre, rim, K, ldr, NGq, scales, nw, Xre, Xim, B[0],
                           B[1], B[2], B[3]);
    else
        hipLaunchKernelGGL(k_pack_split<false>, grid, dim3(256), 0, s, rre, rim, K, ldr, NGq, scales, nw, Xre, Xim,
                           B[0], B[1], B[2], B[3]);
    return hipGetLastError();
}

hipError_t launch_herk_split4(const HerkSplit2Args& h, int eight_waves, hipStream_t s) {
    if (h.ntiles <= 0 || h.nw <= 0 || h.K <= 0) return hipSuccess;
    const int per_xcd = (h.ntiles + kXcds - 1) / kXcds;
    const unsigned blocks = (unsigned)(per_xcd * h.nw * kXcds);
    if (eight_waves) {
        if (h.fp16)
            hipLaunchKernelGGL(k_herk_split5<true>, dim3(blocks), dim3(512), 0, s, h);
        else
            hipLaunchKernelGGL(k_herk_split5<false>, dim3(blocks), dim3(512), 0, s, h);
    } else {
        if (h.fp16)
            hipLaunchKernelGGL(k_herk_split4<true>, dim3(blocks), dim3(256), 0, s, h);
        else
            hipLaunchKernelGGL(k_herk_split4<false>, dim3(blocks), dim3(256), 0, s, h);
    }
    return hipGetLastError();
}

}  // namespace rpa
