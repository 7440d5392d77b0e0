// Grid transforms with whole lines in registers, for grid axes whose length
// has a compiled register transform: the orbitals of Eq. get_wfs (Table 1
// step 3) and the pair densities of Eq. fft (Table 1 steps 5-6).
//
// Orbitals: k_fft_z_reg transforms the z-lines in place (lanes take
// consecutive x, so each load and store is coalesced without LDS), only those
// of the (x, y) columns that hold plane-wave coefficients (the others are zero);
// k_fft_xy_reg takes one z-plane per workgroup through LDS, one thread per
// x-row and then one per y-column. Each axis pair uses its register kernel when
// its length has one, so a grid such as 40 x 40 x 160 runs x and y in registers
// and z through the LDS passes.
//
// Same data flow and outputs as the LDS-pass kernels: k_pair_xy_reg leaves the
// K2 x K1 kept (x, y) outputs of every z-plane of a pair in tbuf
// [pair][z][K2][K1]; k_pair_z_reg transforms those columns along z and gathers
// the G-sphere, scaled by 1/N. What changes is the mapping onto the CU:
//   * conj(phi_n) phi_m of a slab of S z-planes is formed with coalesced loads
//     into LDS rows padded to N1 + 1 elements (so one thread per row reads
//     without bank conflicts);
//   * one thread transforms one x-line in registers (compile-time radix-4/3/2/5
//     splits, constant twiddles) and writes it back into its own row;
//   * one thread transforms one kept x-frequency column along y in place;
//   * the kept K2 x K1 block of every plane goes to tbuf with coalesced stores
//     (unconditional register stores keep the transforms branch-free);
//   * along z one thread owns one column, LDS only holds the spectra for the
//     sphere gather.
#include "internal.hpp"

namespace rpa {

namespace {

// threads per xy workgroup at most: whole FP64 lines need up to 512 registers
// (one wave per SIMD), FP32 lines fit two waves per SIMD
template <typename T, int N>
constexpr int xy_threads() {
    return (sizeof(T) == 8 && N >= 32) || N >= 64 ? 256 : 512;
}

// LDS of one pair-transform slab: one plane of 48^2, FP32 or FP64. Small slabs leave room for several
// workgroups per CU, each running its loads, x pass and y pass on its own, which overlaps the phases
// better than fewer, larger slabs (measured on the FP32 48^3 grid: 3.0 ms per launch for 1 plane,
// 3.04 for 2, 3.57 for 4 (before the load batch below covered a whole slab: 3.43 for 2), 4.44 for 3)
template <typename T>
constexpr size_t reg_lds_budget() {
    return sizeof(T) == 4 ? 20 * 1024 : 40 * 1024;
}

// planes per slab and threads per workgroup of the pair kernel, known at compile time (the launcher computes
// the same from the geometry), and the load batch: each thread issues the loads of all its elements of the
// slab (at most 48 FP32 or 16 FP64 pairs of loads) before the first is used
// Lane exchange inside quads of lanes (DPP quad permutation): 0x4E reads lane r ^ 2, 0xB1 lane r ^ 1.
template <int CTRL>
__device__ __forceinline__ float quad_xchg(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_xchg(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <int CTRL, typename T>
__device__ __forceinline__ cplx<T> quad_xchg(cplx<T> v) {
    return mk(quad_xchg<CTRL>(v.x), quad_xchg<CTRL>(v.y));
}

// Forward transform of N samples spread over the four lanes of a quad: lane r holds the samples 4 i + r in
// v[i] and transforms them (length N/4), multiplies output k by w^(r k) (w = exp(-2 pi i / N)), and a
// four-point transform across the quad (two lane exchanges) leaves outputs k + (N/4) s in v[k] of lane r;
// the return value is s = (r >> 1) + 2 (r & 1).
template <typename T, int N>
__device__ __forceinline__ int fft_quad_core(cplx<T> (&v)[N / 4], int r) {
    constexpr int M = N / 4;
    constexpr Roots<N> W{};
    RegFft<M, -1, T>::run(v);
#pragma unroll
    for (int k = 1; k < M; ++k) {
        // the three lanes' constants split at compile time, then selected by lane
        const int e1 = k % N, e2 = (2 * k) % N, e3 = (3 * k) % N;
        const Split2<T> c1 = split2<T>(W.c[e1]), c2 = split2<T>(W.c[e2]), c3 = split2<T>(W.c[e3]);
        const Split2<T> s1 = split2<T>(-W.s[e1]), s2 = split2<T>(-W.s[e2]), s3 = split2<T>(-W.s[e3]);
        const Split2<T> c = r == 1 ? c1 : r == 2 ? c2 : c3;
        const Split2<T> sn = r == 1 ? s1 : r == 2 ? s2 : s3;
        if (r != 0) v[k] = cmulk(v[k], c, sn);
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
        // r = r0 + 2 r1: sum over r1, twiddle exp(-i pi/2) for r0 = 1 at output bit 1, then sum over r0
        cplx<T> p = quad_xchg<0x4E>(v[k]);
        cplx<T> u = (r & 2) ? p - v[k] : v[k] + p;
        if (r == 3) u = imul<-1>(u);
        p = quad_xchg<0xB1>(u);
        v[k] = (r & 1) ? p - u : u + p;
    }
    return (r >> 1) + 2 * (r & 1);
}

// Forward transform of one column of N (stride LD) by the four lanes of a quad, in place. A kept column
// thus costs a quarter of a whole-line transform per lane.
template <typename T, int N, int LD>
__device__ __forceinline__ void fft_column_quad(cplx<T>* col, int r) {
    constexpr int M = N / 4;
    cplx<T> v[M];
#pragma unroll
    for (int i = 0; i < M; ++i) v[i] = col[(4 * i + r) * LD];
    const int s = fft_quad_core<T, N>(v, r);
#pragma unroll
    for (int k = 0; k < M; ++k) col[(k + M * s) * LD] = v[k];
}

// Inverse transform (sign +1) of one line of N (stride STR) by a quad, in place, as conj(F(conj x)). The
// samples i with (i - lo) mod N >= cnt are read as zero: the entries outside a kept range of cnt indices
// starting at lo, which may hold anything.
template <typename T, int N, int STR>
__device__ __forceinline__ void ifft_line_quad(cplx<T>* line, int r, int lo, int cnt) {
    constexpr int M = N / 4;
    cplx<T> v[M];
#pragma unroll
    for (int i = 0; i < M; ++i) {
        int d = 4 * i + r - lo;
        if (d < 0) d += N;
        const cplx<T> x = line[(4 * i + r) * STR];
        v[i] = d < cnt ? mk(x.x, -x.y) : mk(T(0), T(0));
    }
    const int s = fft_quad_core<T, N>(v, r);
#pragma unroll
    for (int k = 0; k < M; ++k) line[(k + M * s) * STR] = mk(v[k].x, -v[k].y);
}

template <typename T, int N1, int N2>
constexpr int xy_planes() {
    const int s = (int)(reg_lds_budget<T>() / ((size_t)N2 * (N1 + 1) * sizeof(cplx<T>)));
    const int t = xy_threads<T, N1>() / N2;
    return s < t ? (s < 1 ? 1 : s) : t;
}
template <typename T, int N1, int N2>
constexpr int xy_batch() {
    const int rows = xy_planes<T, N1, N2>() * N2;
    const int thr = (rows + 63) / 64 * 64 < xy_threads<T, N1>() ? (rows + 63) / 64 * 64 : xy_threads<T, N1>();
    const int u = (xy_planes<T, N1, N2>() * N1 * N2 + thr - 1) / thr;
    const int cap = sizeof(T) == 4 ? 48 : 16;
    return u < cap ? u : cap;
}

template <typename T, int N1, int N2>
__global__ __launch_bounds__((xy_threads<T, N1>())) void k_pair_xy_reg(const cplx<T>* __restrict__ phik,
                                                     const cplx<T>* __restrict__ phikq,
                                                     const int32_t* __restrict__ pn,
                                                     const int32_t* __restrict__ pm, int npairs, PairGeom g,
                                                     int S, cplx<T>* __restrict__ tbuf) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* X = reinterpret_cast<cplx<T>*>(smem);
    constexpr int LD = N1 + 1;
    constexpr int plane = N1 * N2;
    // Tasks t = slab * npairs + pair. Workgroup w runs on XCD w % 8; each XCD
    // takes a contiguous range of t, so the pairs that share an orbital (the
    // pair list runs over n fastest) meet in the same L2.
    const unsigned ntask = gridDim.x, w = blockIdx.x;
    const unsigned xcd = w & 7u, q = ntask >> 3, r = ntask & 7u;
    const unsigned t = xcd * q + min(xcd, r) + (w >> 3);
    const int slab = (int)(t / (unsigned)npairs);
    const int p = (int)(t - (unsigned)slab * npairs);
    const int z0 = slab * S;
    const int ns = min(S, g.N3 - z0);
    const size_t vol = (size_t)plane * g.N3;
    const cplx<T>* a0 = phik + (size_t)pn[p] * vol + (size_t)z0 * plane;
    const cplx<T>* b0 = phikq + (size_t)pm[p] * vol + (size_t)z0 * plane;

    // conj(phi_n) phi_m on the slab, row (zs, y) at X[(zs N2 + y) LD]; the loads of U elements are
    // issued before any is used
    const int tot = ns * plane;
    constexpr int U = xy_batch<T, N1, N2>();
    for (int f0 = threadIdx.x; f0 < tot; f0 += U * blockDim.x) {
        cplx<T> va[U], vb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int f = min(f0 + u * (int)blockDim.x, tot - 1);
            va[u] = a0[f];
            vb[u] = b0[f];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int f = f0 + u * (int)blockDim.x;
            if (f < tot) {
                const int row = f / N1, col = f - row * N1;
                X[row * LD + col] = cmulc(va[u], vb[u]);
            }
        }
    }
    __syncthreads();

    // x: one line per thread, transformed in place
    const int l = threadIdx.x;
    if (l < ns * N2) {
        cplx<T>* row = X + l * LD;
        cplx<T> v[N1];
#pragma unroll
        for (int i = 0; i < N1; ++i) v[i] = row[i];
        RegFft<N1, -1, T>::run(v);
#pragma unroll
        for (int i = 0; i < N1; ++i) row[i] = v[i];
    }
    __syncthreads();

    // y: each kept x-frequency column transformed in place by a quad of lanes where the workgroup has
    // enough of them, else by one thread
    const int K1 = g.K1, K2 = g.K2;
    bool quad = false;
    if constexpr (N2 % 4 == 0) quad = 4 * ns * K1 <= (int)blockDim.x;
    if (quad) {
        if constexpr (N2 % 4 == 0) {
            if (l < 4 * ns * K1) {
                const int cq = l >> 2;
                const int zs = cq / K1, ix = cq - zs * K1;
                int kx = g.x0 + ix;
                if (kx >= N1) kx -= N1;
                fft_column_quad<T, N2, LD>(X + zs * N2 * LD + kx, l & 3);
            }
        }
    } else if (l < ns * K1) {
        const int zs = l / K1, ix = l - zs * K1;
        int kx = g.x0 + ix;
        if (kx >= N1) kx -= N1;
        cplx<T>* col = X + zs * N2 * LD + kx;
        cplx<T> v[N2];
#pragma unroll
        for (int y = 0; y < N2; ++y) v[y] = col[y * LD];
        RegFft<N2, -1, T>::run(v);
#pragma unroll
        for (int y = 0; y < N2; ++y) col[y * LD] = v[y];
    }
    __syncthreads();

    // kept (ky, kx) block of every plane to tbuf [pair][z][K2][K1], coalesced
    const int kk = K1 * K2;
    cplx<T>* to = tbuf + ((size_t)p * g.N3 + z0) * kk;
    for (int f = threadIdx.x; f < ns * kk; f += blockDim.x) {
        const int zs = f / kk, r = f - zs * kk;
        const int iy = r / K1, ix = r - iy * K1;
        int kx = g.x0 + ix, ky = g.y0 + iy;
        if (kx >= N1) kx -= N1;
        if (ky >= N2) ky -= N2;
        to[f] = X[(zs * N2 + ky) * LD + kx];
    }
}

template <typename T, int N3>
__global__ __launch_bounds__(256) void k_pair_z_reg(const cplx<T>* __restrict__ tbuf, PairGeom g,
                                                    const int32_t* __restrict__ zcol,
                                                    const int32_t* __restrict__ col_start,
                                                    const int32_t* __restrict__ col_g,
                                                    const int32_t* __restrict__ col_kz, T* __restrict__ rre,
                                                    T* __restrict__ rim) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* Z = reinterpret_cast<cplx<T>*>(smem);
    constexpr int LD = N3 + 1;
    const int ncols = g.ncols;
    const size_t p = blockIdx.x;
    const int CB = blockDim.x;
    const int c0 = blockIdx.y * CB;
    const int nc = min(CB, g.nzc - c0);
    const int c = threadIdx.x;
    if (c < nc) {
        const cplx<T>* src = tbuf + p * N3 * ncols + zcol[c0 + c];
        cplx<T> v[N3];
#pragma unroll
        for (int z = 0; z < N3; ++z) v[z] = src[(size_t)z * ncols];
        RegFft<N3, -1, T>::run(v);
#pragma unroll
        for (int z = 0; z < N3; ++z) Z[c * LD + z] = v[z];
    }
    __syncthreads();
    const Split2<T> invN = split2<T>(1.0 / ((double)g.N1 * g.N2 * N3));
    const int e0 = col_start[c0], e1 = col_start[c0 + nc];
    T* ore = rre + p * g.NGp;
    T* oim = rim + p * g.NGp;
    for (int i = e0 + threadIdx.x; i < e1; i += CB) {
        const int gi = col_g[i];
        const int kz = col_kz[i] >> 16;  // packed (kz << 16) | column
        const int cc = col_kz[i] & 0xffff;
        const cplx<T> v = Z[(cc - c0) * LD + kz];
        ore[gi] = mulk(v.x, invN);
        oim[gi] = mulk(v.y, invN);
    }
    if (blockIdx.y == 0) {
        for (int gi = g.NG + threadIdx.x; gi < g.NGp; gi += CB) {
            ore[gi] = T(0);
            oim[gi] = T(0);
        }
    }
}

// Adjoint of the x-y pass of k_pair_xy_reg, with the product by the other orbital and the sum over the
// pairs of one owner band (FP64 gradients). A workgroup takes one segment of an owner's pairs on one
// z-plane; for each pair the kept K2 x K1 block of that plane's adjoint spectrum (tadj [pair][z][K2][K1])
// goes into its place in the plane, each kept x-frequency column is taken back along y (kept rows only
// read) and every row along x (kept columns only read), both by quads of lanes, and the result xbar is
// multiplied by the other band's orbital:
//   side 1 (owner m): acc += phi_n xbar,   side 0 (owner n): acc += phi_m conj(xbar).
// seg holds per segment (owner, first, end into list, slot): the sum is added into phibar[band0 + owner]
// where the owner has this one segment (slot < 0), else written to partial [slot][z][plane] and added by
// k_xyadj_reduce. Tasks run z-plane by z-plane, so the orbital planes they read meet in L2.
template <typename T, int N>
constexpr int adj_threads() {
    return (4 * N + 63) / 64 * 64;
}

template <typename T, int N>
__global__ __launch_bounds__((adj_threads<T, N>())) void k_xyadj_reg(const cplx<T>* __restrict__ tadj, PairGeom g,
                                                     const int32_t* __restrict__ seg, int nseg,
                                                     const int32_t* __restrict__ list,
                                                     const int32_t* __restrict__ other,
                                                     const cplx<T>* __restrict__ phio, int band0, int side,
                                                     cplx<T>* __restrict__ phibar, cplx<T>* __restrict__ partial) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* X = reinterpret_cast<cplx<T>*>(smem);
    constexpr int NT = adj_threads<T, N>(), LD = N + 1, plane = N * N, kA = (plane + NT - 1) / NT;
    // each XCD (workgroup w runs on XCD w % 8) takes a contiguous range of tasks t = z nseg + segment
    const unsigned ntask = gridDim.x, w = blockIdx.x;
    const unsigned xcd = w & 7u, q = ntask >> 3, rq = ntask & 7u;
    const unsigned t = xcd * q + min(xcd, rq) + (w >> 3);
    const int z = (int)(t / (unsigned)nseg), sgi = (int)(t - (unsigned)z * nseg);
    const int owner = seg[4 * sgi], e0 = seg[4 * sgi + 1], e1 = seg[4 * sgi + 2], slot = seg[4 * sgi + 3];
    const int K1 = g.K1, K2 = g.K2, kk = K1 * K2;
    const size_t vol = (size_t)plane * g.N3;
    const int l = threadIdx.x;
    cplx<T> acc[kA];
#pragma unroll
    for (int a = 0; a < kA; ++a) acc[a] = mk(T(0), T(0));
    for (int e = e0; e < e1; ++e) {
        const int p = list[e];
        const cplx<T>* src = tadj + ((size_t)p * g.N3 + z) * kk;
        __syncthreads();  // the previous pair's product has read the plane
        for (int f = l; f < kk; f += NT) {
            const int iy = f / K1, ix = f - iy * K1;
            int kx = g.x0 + ix, ky = g.y0 + iy;
            if (kx >= N) kx -= N;
            if (ky >= N) ky -= N;
            X[ky * LD + kx] = src[f];
        }
        __syncthreads();
        if (l < 4 * K1) {
            int kx = g.x0 + (l >> 2);
            if (kx >= N) kx -= N;
            ifft_line_quad<T, N, LD>(X + kx, l & 3, g.y0, K2);
        }
        __syncthreads();
        if (l < 4 * N) ifft_line_quad<T, N, 1>(X + (l >> 2) * LD, l & 3, g.x0, K1);
        __syncthreads();
        // the other band's orbital on this plane
        const cplx<T>* ph = phio + (size_t)other[p] * vol + (size_t)z * plane;
        cplx<T> o[kA];
#pragma unroll
        for (int a = 0; a < kA; ++a) o[a] = ph[min(l + a * NT, plane - 1)];
#pragma unroll
        for (int a = 0; a < kA; ++a) {
            const int f = l + a * NT;
            if (f < plane) {
                const cplx<T> xb = X[(f / N) * LD + f % N];
                acc[a] = acc[a] + (side == 1 ? o[a] * xb : o[a] * conj(xb));
            }
        }
    }
    cplx<T>* out = slot < 0 ? phibar + (size_t)(band0 + owner) * vol + (size_t)z * plane
                            : partial + ((size_t)slot * g.N3 + z) * plane;
#pragma unroll
    for (int a = 0; a < kA; ++a) {
        const int f = l + a * NT;
        if (f < plane) out[f] = slot < 0 ? out[f] + acc[a] : acc[a];
    }
}

// phibar[band0 + own[j]] += the sum of its partial slots [ostart[j], ostart[j + 1]), in slot order
template <typename T>
__global__ __launch_bounds__(256) void k_xyadj_reduce(const cplx<T>* __restrict__ partial, size_t vol,
                                                      const int32_t* __restrict__ own,
                                                      const int32_t* __restrict__ ostart, int band0,
                                                      cplx<T>* __restrict__ phibar) {
    const int j = blockIdx.y, s0 = ostart[j], s1 = ostart[j + 1];
    cplx<T>* out = phibar + (size_t)(band0 + own[j]) * vol;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < vol; i += (size_t)gridDim.x * blockDim.x) {
        cplx<T> v = out[i];
        for (int s = s0; s < s1; ++s) v = v + partial[(size_t)s * vol + i];
        out[i] = v;
    }
}

// z pass by quads of lanes for N3 = 4 M (M a register length), where a whole FP32 or FP64 line of N3 does
// not fit one lane's registers: a workgroup of 256 lanes takes 64 held columns of one pair, the quad of lanes
// 4c..4c+3 transforms column c (lane r the samples z = 4 i + r) and keeps the outputs that fall in the
// sphere's z window [z0, z0 + K3) in LDS row c; the sphere entries of those columns are then read from LDS,
// scaled by 1/N and stored.
constexpr int kZQuadCols = 64;

template <typename T, int N3>
__global__ __launch_bounds__(4 * kZQuadCols) void k_pair_z_quad(const cplx<T>* __restrict__ tbuf, PairGeom g,
                                                                const int32_t* __restrict__ zcol,
                                                                const int32_t* __restrict__ col_start,
                                                                const int32_t* __restrict__ col_g,
                                                                const int32_t* __restrict__ col_kz,
                                                                T* __restrict__ rre, T* __restrict__ rim) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* Z = reinterpret_cast<cplx<T>*>(smem);
    constexpr int M = N3 / 4, CB = kZQuadCols;
    const int LDZ = g.K3 + 1, ncols = g.ncols;
    const size_t p = blockIdx.x;
    const int c0 = blockIdx.y * CB;
    const int nc = min(CB, g.nzc - c0);
    const int l = threadIdx.x, c = l >> 2, r = l & 3;
    if (c < nc) {
        const cplx<T>* src = tbuf + p * N3 * ncols + zcol[c0 + c];
        cplx<T> v[M];
#pragma unroll
        for (int i = 0; i < M; ++i) v[i] = src[(size_t)(4 * i + r) * ncols];
        const int s = fft_quad_core<T, N3>(v, r);
#pragma unroll
        for (int k = 0; k < M; ++k) {
            int d = k + M * s - g.z0;
            if (d < 0) d += N3;
            if (d < g.K3) Z[c * LDZ + d] = v[k];
        }
    }
    __syncthreads();
    const Split2<T> invN = split2<T>(1.0 / ((double)g.N1 * g.N2 * N3));
    const int e0 = col_start[c0], e1 = col_start[c0 + nc];
    T* ore = rre + p * g.NGp;
    T* oim = rim + p * g.NGp;
    for (int i = e0 + l; i < e1; i += 4 * CB) {
        const int gi = col_g[i];
        int d = (col_kz[i] >> 16) - g.z0;  // packed (kz << 16) | column
        if (d < 0) d += N3;
        const int cc = col_kz[i] & 0xffff;
        const cplx<T> v = Z[(cc - c0) * LDZ + d];
        ore[gi] = mulk(v.x, invN);
        oim[gi] = mulk(v.y, invN);
    }
    if (blockIdx.y == 0) {
        for (int gi = g.NG + l; gi < g.NGp; gi += 4 * CB) {
            ore[gi] = T(0);
            oim[gi] = T(0);
        }
    }
}

template <typename T, int N3, int DIR>
__global__ __launch_bounds__(256) void k_fft_z_reg(cplx<T>* __restrict__ data, long long nlines, int plane,
                                                   const int32_t* __restrict__ cols, int ncols) {
    const long long L = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (L >= nlines) return;
    const long long b = L / ncols;
    const int i = (int)(L - b * ncols);
    cplx<T>* base = data + b * (long long)plane * N3 + (cols ? cols[i] : i);
    cplx<T> v[N3];
#pragma unroll
    for (int z = 0; z < N3; ++z) v[z] = base[(long long)z * plane];
    RegFft<N3, DIR, T>::run(v);
#pragma unroll
    for (int z = 0; z < N3; ++z) base[(long long)z * plane] = v[z];
}

template <typename T, int N, int DIR>
__global__ __launch_bounds__(64) void k_fft_xy_reg(cplx<T>* __restrict__ data) {
    __shared__ cplx<T> X[N][N + 1];
    cplx<T>* base = data + (size_t)blockIdx.x * N * N;
    constexpr int U = sizeof(T) == 4 ? 16 : 8;
    for (int f0 = threadIdx.x; f0 < N * N; f0 += U * blockDim.x) {
        cplx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = base[min(f0 + u * (int)blockDim.x, N * N - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int f = f0 + u * (int)blockDim.x;
            if (f < N * N) X[f / N][f % N] = v[u];
        }
    }
    __syncthreads();
    const int t = threadIdx.x;
    if (t < N) {
        cplx<T> v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = X[t][i];
        RegFft<N, DIR, T>::run(v);
#pragma unroll
        for (int i = 0; i < N; ++i) X[t][i] = v[i];
    }
    __syncthreads();
    if (t < N) {
        cplx<T> v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = X[i][t];
        RegFft<N, DIR, T>::run(v);
#pragma unroll
        for (int i = 0; i < N; ++i) X[i][t] = v[i];
    }
    __syncthreads();
    for (int f = threadIdx.x; f < N * N; f += blockDim.x) base[f] = X[f / N][f % N];
}


bool reg_size(int n) {
    switch (n) {
#define RPA_CASE(L) case L:
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        return true;
        default: return false;
    }
}

template <typename T>
int xy_threads_rt(int N) {
    switch (N) {
#define RPA_CASE(L) case L: return xy_threads<T, L>();
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return 0;
    }
}

// planes per xy workgroup: as many as keep the padded slab within the budget,
// at most one row per thread
template <typename T>
int xy_slab(const PairGeom& g) {
    const size_t per_plane = (size_t)g.N2 * (g.N1 + 1) * sizeof(cplx<T>);
    int S = (int)(reg_lds_budget<T>() / per_plane);
    S = std::min(S, std::max(1, xy_threads_rt<T>(g.N1) / g.N2));
    S = std::min(S, g.N3);
    return S;
}

template <typename T>
int z_block() {
    return sizeof(T) == 8 ? 64 : 128;
}

}  // namespace

template <typename T>
bool pair_xy_reg_supported(const PairGeom& g) {
    if (g.N1 != g.N2 || !reg_size(g.N1)) return false;
    // a 64-point FP64 line does not fit the register file
    if (sizeof(T) == 8 && g.N1 > 48) return false;
    return xy_slab<T>(g) >= 1;
}

template <typename T>
bool pair_z_reg_supported(const PairGeom& g) {
    if (!reg_size(g.N3)) return false;
    if (sizeof(T) == 8 && g.N3 > 48) return false;
    return g.ncols <= 0xffff;
}

template <typename T>
hipError_t launch_grid_fft_z_reg(cplx<T>* data, int nb, int N1, int N2, int N3, int dir, const int32_t* cols,
                                 int ncols, hipStream_t s) {
    if (!nb) return hipSuccess;
    PairGeom g{};
    g.N1 = N1;
    g.N2 = N2;
    g.N3 = N3;
    if (!pair_z_reg_supported<T>(g)) return hipErrorNotSupported;
    const int plane = N1 * N2;
    if (!cols) ncols = plane;
    if (ncols <= 0) return hipSuccess;
    const long long nlines = (long long)nb * ncols;
    const unsigned zb = (unsigned)((nlines + 255) / 256);
    switch (N3) {
#define RPA_CASE(L)                                                                                             \
    case L:                                                                                                     \
        if (dir > 0)                                                                                            \
            hipLaunchKernelGGL((k_fft_z_reg<T, L, 1>), dim3(zb), dim3(256), 0, s, data, nlines, plane, cols,     \
                               ncols);                                                                          \
        else                                                                                                    \
            hipLaunchKernelGGL((k_fft_z_reg<T, L, -1>), dim3(zb), dim3(256), 0, s, data, nlines, plane, cols,    \
                               ncols);                                                                          \
        break;
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grid_fft_xy_reg(cplx<T>* data, int nb, int N1, int N2, int N3, int dir, hipStream_t s) {
    if (!nb) return hipSuccess;
    PairGeom g{};
    g.N1 = N1;
    g.N2 = N2;
    g.N3 = N3;
    g.K1 = 1;
    if (!pair_xy_reg_supported<T>(g)) return hipErrorNotSupported;
    const unsigned planes = (unsigned)((long long)nb * N3);
    switch (N1) {
#define RPA_CASE(L)                                                                                   \
    case L:                                                                                           \
        if (dir > 0)                                                                                  \
            hipLaunchKernelGGL((k_fft_xy_reg<T, L, 1>), dim3(planes), dim3(64), 0, s, data);           \
        else                                                                                          \
            hipLaunchKernelGGL((k_fft_xy_reg<T, L, -1>), dim3(planes), dim3(64), 0, s, data);          \
        break;
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pair_xy_reg(const cplx<T>* phik, const cplx<T>* phikq, const int32_t* pn, const int32_t* pm,
                              int npairs, const PairGeom& g, cplx<T>* tbuf, hipStream_t s) {
    if (!npairs) return hipSuccess;
    if (!pair_xy_reg_supported<T>(g)) return hipErrorNotSupported;
    const int S = xy_slab<T>(g);
    const int rows = S * g.N2;
    const int threads = std::min(xy_threads_rt<T>(g.N1), (rows + 63) / 64 * 64);
    if (rows > threads || S * g.K1 > threads) return hipErrorInvalidValue;  // one line per thread
    const size_t lds = (size_t)S * g.N2 * (g.N1 + 1) * sizeof(cplx<T>);
    const long long tasks = (long long)npairs * ((g.N3 + S - 1) / S);
    if (tasks > 0x7fffffffLL) return hipErrorInvalidValue;
    dim3 grid((unsigned)tasks);
    switch (g.N1) {
#define RPA_CASE(L)                                                                                              \
    case L:                                                                                                      \
        hipLaunchKernelGGL((k_pair_xy_reg<T, L, L>), grid, dim3(threads), lds, s, phik, phikq, pn, pm, npairs,   \
                           g, S, tbuf);                                                                          \
        break;
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pair_z_reg(const cplx<T>* tbuf, int npairs, const PairGeom& g, const int32_t* zcol,
                             const int32_t* col_start, const int32_t* col_g, const int32_t* col_kz, T* rho_re,
                             T* rho_im, hipStream_t s) {
    if (!npairs) return hipSuccess;
    if (!pair_z_reg_supported<T>(g)) return hipErrorNotSupported;
    if (g.nzc < 1 || g.nzc > g.ncols) return hipErrorInvalidValue;
    const int CB = z_block<T>();
    const size_t lds = (size_t)CB * (g.N3 + 1) * sizeof(cplx<T>);
    dim3 grid((unsigned)npairs, (unsigned)((g.nzc + CB - 1) / CB));
    switch (g.N3) {
#define RPA_CASE(L)                                                                                                \
    case L:                                                                                                        \
        hipLaunchKernelGGL((k_pair_z_reg<T, L>), grid, dim3(CB), lds, s, tbuf, g, zcol, col_start, col_g, col_kz,   \
                           rho_re, rho_im);                                                                        \
        break;
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template <typename T>
bool pair_z_quad_supported(const PairGeom& g) {
    if (g.N3 % 4 != 0 || !reg_size(g.N3 / 4)) return false;
    if (sizeof(T) == 8 && g.N3 / 4 > 48) return false;  // 48 complex FP64 values per lane at most
    return g.ncols <= 0xffff && g.K3 >= 1 && g.K3 <= g.N3 && g.z0 >= 0 && g.z0 < g.N3;
}

namespace {
template <typename T, int M>
hipError_t z_quad_case(const cplx<T>* tbuf, int npairs, const PairGeom& g, const int32_t* zcol,
                       const int32_t* col_start, const int32_t* col_g, const int32_t* col_kz, T* rre, T* rim,
                       hipStream_t s) {
    if constexpr (sizeof(T) == 8 && M > 48) {
        return hipErrorNotSupported;
    } else {
        const size_t lds = (size_t)kZQuadCols * (g.K3 + 1) * sizeof(cplx<T>);
        dim3 grid((unsigned)npairs, (unsigned)((g.nzc + kZQuadCols - 1) / kZQuadCols));
        hipLaunchKernelGGL((k_pair_z_quad<T, 4 * M>), grid, dim3(4 * kZQuadCols), lds, s, tbuf, g, zcol, col_start,
                           col_g, col_kz, rre, rim);
        return hipGetLastError();
    }
}
}  // namespace

template <typename T>
hipError_t launch_pair_z_quad(const cplx<T>* tbuf, int npairs, const PairGeom& g, const int32_t* zcol,
                              const int32_t* col_start, const int32_t* col_g, const int32_t* col_kz, T* rho_re,
                              T* rho_im, hipStream_t s) {
    if (!npairs) return hipSuccess;
    if (!pair_z_quad_supported<T>(g)) return hipErrorNotSupported;
    if (g.nzc < 1 || g.nzc > g.ncols) return hipErrorInvalidValue;
    switch (g.N3 / 4) {
#define RPA_CASE(L)                                                                                             \
    case L:                                                                                                     \
        return z_quad_case<T, L>(tbuf, npairs, g, zcol, col_start, col_g, col_kz, rho_re, rho_im, s);
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return hipErrorNotSupported;
    }
}

namespace {
template <int L>
hipError_t xyadj_case(long long tasks, const cplx<double>* tadj, const PairGeom& g, const int32_t* seg, int nseg,
                      const int32_t* list, const int32_t* other, const cplx<double>* phio, int band0, int side,
                      cplx<double>* phibar, cplx<double>* partial, hipStream_t s) {
    if constexpr (L % 4 == 0 && L <= 64) {
        const size_t lds = (size_t)L * (L + 1) * sizeof(cplx<double>);
        hipLaunchKernelGGL((k_xyadj_reg<double, L>), dim3((unsigned)tasks), dim3(adj_threads<double, L>()), lds, s,
                           tadj, g, seg, nseg, list, other, phio, band0, side, phibar, partial);
        return hipGetLastError();
    } else {
        return hipErrorNotSupported;
    }
}
}  // namespace

bool xyadj_reg_supported(const PairGeom& g) {
    if (g.N1 != g.N2 || g.N1 % 4 != 0 || !reg_size(g.N1) || g.N1 > 64) return false;
    return g.K1 >= 1 && g.K1 <= g.N1 && g.K2 >= 1 && g.K2 <= g.N2;
}

hipError_t launch_xyadj_reg(const cplx<double>* tadj, const PairGeom& g, const int32_t* seg, int nseg,
                            const int32_t* list, const int32_t* other, const cplx<double>* phio, int band0, int side,
                            cplx<double>* phibar, cplx<double>* partial, hipStream_t s) {
    if (!nseg) return hipSuccess;
    if (!xyadj_reg_supported(g)) return hipErrorNotSupported;
    const long long tasks = (long long)nseg * g.N3;
    if (tasks * 4 * g.N1 >= (1LL << 32)) return hipErrorInvalidValue;  // grid of at most 2^32 - 1 lanes
    switch (g.N1) {
#define RPA_CASE(L)                                                                                             \
    case L:                                                                                                     \
        return xyadj_case<L>(tasks, tadj, g, seg, nseg, list, other, phio, band0, side, phibar, partial, s);
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return hipErrorNotSupported;
    }
}

hipError_t launch_xyadj_reduce(const cplx<double>* partial, size_t vol, const int32_t* own, const int32_t* ostart,
                               int nown, int band0, cplx<double>* phibar, hipStream_t s) {
    if (nown <= 0) return hipSuccess;
    const unsigned bx = (unsigned)std::min<size_t>((vol + 255) / 256, 1024);
    hipLaunchKernelGGL(k_xyadj_reduce<double>, dim3(bx, (unsigned)nown), dim3(256), 0, s, partial, vol, own, ostart,
                       band0, phibar);
    return hipGetLastError();
}

#define RPA_INST(T)                                                                                              \
    template bool pair_xy_reg_supported<T>(const PairGeom&);                                                     \
    template bool pair_z_reg_supported<T>(const PairGeom&);                                                      \
    template hipError_t launch_grid_fft_z_reg<T>(cplx<T>*, int, int, int, int, int, const int32_t*, int, hipStream_t);                 \
    template hipError_t launch_grid_fft_xy_reg<T>(cplx<T>*, int, int, int, int, int, hipStream_t);                \
    template hipError_t launch_pair_xy_reg<T>(const cplx<T>*, const cplx<T>*, const int32_t*, const int32_t*, int, \
                                              const PairGeom&, cplx<T>*, hipStream_t);                           \
    template bool pair_z_quad_supported<T>(const PairGeom&);                                                    \
    template hipError_t launch_pair_z_quad<T>(const cplx<T>*, int, const PairGeom&, const int32_t*, const int32_t*, \
                                              const int32_t*, const int32_t*, T*, T*, hipStream_t);              \
    template hipError_t launch_pair_z_reg<T>(const cplx<T>*, int, const PairGeom&, const int32_t*, const int32_t*, \
                                             const int32_t*, const int32_t*, T*, T*, hipStream_t);
RPA_INST(double)
RPA_INST(float)
#undef RPA_INST

}  // namespace rpa
