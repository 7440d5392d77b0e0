// Pair-density transforms (Eq. fft, Table 1 steps 5-6) with whole lines in
// registers, for grid axes whose length has a compiled register transform.
//
// Same data flow and outputs as the LDS-pass kernels: k_pair_xy_reg leaves the
// K2 x K1 kept (x, y) outputs of every z-plane of a pair in tbuf
// [pair][z][K2][K1]; k_pair_z_reg transforms those columns along z and gathers
// the G-sphere, scaled by 1/N. What changes is the mapping onto the CU:
//   * conj(phi_n) phi_m of a slab of S z-planes is formed with coalesced loads
//     into LDS rows padded to N1 + 1 elements (so one thread per row reads
//     without bank conflicts);
//   * one thread transforms one x-line in registers (compile-time radix-4/3/2/5
//     splits, constant twiddles) and writes its K1 kept outputs back into the
//     start of its own row;
//   * one thread transforms one kept y-column in registers and writes its K2
//     kept outputs straight to tbuf;
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

template <typename T, int N1, int N2>
__global__ __launch_bounds__((xy_threads<T, N1>())) void k_pair_xy_reg(const cplx<T>* __restrict__ phik,
                                                     const cplx<T>* __restrict__ phikq,
                                                     const int32_t* __restrict__ pn,
                                                     const int32_t* __restrict__ pm, PairGeom g, int S,
                                                     cplx<T>* __restrict__ tbuf) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* X = reinterpret_cast<cplx<T>*>(smem);
    constexpr int LD = N1 + 1;
    constexpr int plane = N1 * N2;
    const int K1 = g.K1, K2 = g.K2;
    const int p = blockIdx.x;
    const int z0 = blockIdx.y * S;
    const int ns = min(S, g.N3 - z0);
    const size_t vol = (size_t)plane * g.N3;
    const cplx<T>* a0 = phik + (size_t)pn[p] * vol + (size_t)z0 * plane;
    const cplx<T>* b0 = phikq + (size_t)pm[p] * vol + (size_t)z0 * plane;

    // conj(phi_n) phi_m on the slab, row (zs, y) at X[(zs N2 + y) LD]
    const int tot = ns * plane;
    for (int f = threadIdx.x; f < tot; f += blockDim.x) {
        const int row = f / N1, col = f - row * N1;
        X[row * LD + col] = cmulc(a0[f], b0[f]);
    }
    __syncthreads();

    // x: one line per thread, K1 kept outputs back into the row
    for (int l = threadIdx.x; l < ns * N2; l += blockDim.x) {
        cplx<T>* row = X + l * LD;
        cplx<T> v[N1];
#pragma unroll
        for (int i = 0; i < N1; ++i) v[i] = row[i];
        RegFft<N1, -1, T>::run(v);
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            int ix = k - g.x0;
            if (ix < 0) ix += N1;
            if (ix < K1) row[ix] = v[k];
        }
    }
    __syncthreads();

    // y: one kept column per thread, K2 kept outputs to tbuf
    const int kk = K1 * K2;
    cplx<T>* to = tbuf + ((size_t)p * g.N3 + z0) * kk;
    for (int l = threadIdx.x; l < ns * K1; l += blockDim.x) {
        const int zs = l / K1, ix = l - zs * K1;
        const cplx<T>* col = X + zs * N2 * LD + ix;
        cplx<T> v[N2];
#pragma unroll
        for (int y = 0; y < N2; ++y) v[y] = col[y * LD];
        RegFft<N2, -1, T>::run(v);
        cplx<T>* o = to + (size_t)zs * kk + ix;
#pragma unroll
        for (int k = 0; k < N2; ++k) {
            int iy = k - g.y0;
            if (iy < 0) iy += N2;
            if (iy < K2) o[iy * K1] = v[k];
        }
    }
}

template <typename T, int N3>
__global__ __launch_bounds__(256) void k_pair_z_reg(const cplx<T>* __restrict__ tbuf, PairGeom g,
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
    const int nc = min(CB, ncols - c0);
    const int c = threadIdx.x;
    if (c < nc) {
        const cplx<T>* src = tbuf + p * N3 * ncols + c0 + c;
        cplx<T> v[N3];
#pragma unroll
        for (int z = 0; z < N3; ++z) v[z] = src[(size_t)z * ncols];
        RegFft<N3, -1, T>::run(v);
#pragma unroll
        for (int z = 0; z < N3; ++z) Z[c * LD + z] = v[z];
    }
    __syncthreads();
    const T invN = T(1.0 / ((double)g.N1 * g.N2 * N3));
    const int e0 = col_start[c0], e1 = col_start[c0 + nc];
    T* ore = rre + p * g.NGp;
    T* oim = rim + p * g.NGp;
    for (int i = e0 + threadIdx.x; i < e1; i += CB) {
        const int gi = col_g[i];
        const int kz = col_kz[i] >> 16;  // packed (kz << 16) | column
        const int cc = col_kz[i] & 0xffff;
        const cplx<T> v = Z[(cc - c0) * LD + kz];
        ore[gi] = v.x * invN;
        oim[gi] = v.y * invN;
    }
    if (blockIdx.y == 0) {
        for (int gi = g.NG + threadIdx.x; gi < g.NGp; gi += CB) {
            ore[gi] = T(0);
            oim[gi] = T(0);
        }
    }
}

constexpr size_t kRegLdsBudget = 80 * 1024;

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
    int S = (int)(kRegLdsBudget / per_plane);
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
bool pair_reg_supported(const PairGeom& g) {
    if (g.N1 != g.N2 || !reg_size(g.N1) || !reg_size(g.N3)) return false;
    // a 64-point FP64 line does not fit the register file
    if (sizeof(T) == 8 && (g.N1 > 48 || g.N3 > 48)) return false;
    if (xy_slab<T>(g) < 1) return false;
    if (g.ncols > 0xffff) return false;
    return true;
}

template <typename T>
hipError_t launch_pair_xy_reg(const cplx<T>* phik, const cplx<T>* phikq, const int32_t* pn, const int32_t* pm,
                              int npairs, const PairGeom& g, cplx<T>* tbuf, hipStream_t s) {
    if (!npairs) return hipSuccess;
    if (!pair_reg_supported<T>(g)) return hipErrorNotSupported;
    const int S = xy_slab<T>(g);
    const int rows = S * g.N2;
    const int threads = std::min(xy_threads_rt<T>(g.N1), (rows + 63) / 64 * 64);
    const size_t lds = (size_t)S * g.N2 * (g.N1 + 1) * sizeof(cplx<T>);
    dim3 grid((unsigned)npairs, (unsigned)((g.N3 + S - 1) / S));
    switch (g.N1) {
#define RPA_CASE(L)                                                                                              \
    case L:                                                                                                      \
        hipLaunchKernelGGL((k_pair_xy_reg<T, L, L>), grid, dim3(threads), lds, s, phik, phikq, pn, pm, g, S,     \
                           tbuf);                                                                                \
        break;
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return hipErrorNotSupported;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pair_z_reg(const cplx<T>* tbuf, int npairs, const PairGeom& g, const int32_t* col_start,
                             const int32_t* col_g, const int32_t* col_kz, T* rho_re, T* rho_im, hipStream_t s) {
    if (!npairs) return hipSuccess;
    if (!pair_reg_supported<T>(g)) return hipErrorNotSupported;
    const int CB = z_block<T>();
    const size_t lds = (size_t)CB * (g.N3 + 1) * sizeof(cplx<T>);
    dim3 grid((unsigned)npairs, (unsigned)((g.ncols + CB - 1) / CB));
    switch (g.N3) {
#define RPA_CASE(L)                                                                                                \
    case L:                                                                                                        \
        hipLaunchKernelGGL((k_pair_z_reg<T, L>), grid, dim3(CB), lds, s, tbuf, g, col_start, col_g, col_kz, rho_re, \
                           rho_im);                                                                                \
        break;
        RPA_REG_SIZES(RPA_CASE)
#undef RPA_CASE
        default: return hipErrorNotSupported;
    }
    return hipGetLastError();
}

#define RPA_INST(T)                                                                                              \
    template bool pair_reg_supported<T>(const PairGeom&);                                                        \
    template hipError_t launch_pair_xy_reg<T>(const cplx<T>*, const cplx<T>*, const int32_t*, const int32_t*, int, \
                                              const PairGeom&, cplx<T>*, hipStream_t);                           \
    template hipError_t launch_pair_z_reg<T>(const cplx<T>*, int, const PairGeom&, const int32_t*, const int32_t*, \
                                             const int32_t*, T*, T*, hipStream_t);
RPA_INST(double)
RPA_INST(float)
#undef RPA_INST

}  // namespace rpa
