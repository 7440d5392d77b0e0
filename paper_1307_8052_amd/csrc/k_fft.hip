// Real-space grid stages: orbitals from plane-wave coefficients (Eq. get_wfs,
// Table 1 step 3) and pruned pair-density transforms with the G-sphere gather
// (Eq. fft, Table 1 steps 5-6).
//
// Grid arrays are [band][z][y][x] with x fastest (axes a1, a2, a3). The pair
// transform runs in two kernels:
//   k_pair_xy      one z-plane of a few pairs: conj(phi_n) phi_m formed while
//                  loading, x-transform of every line, y-transform of the K1
//                  columns that reach the sphere, K2 x K1 kept outputs written;
//   k_pair_z_gather a block of (m1, m2) columns of one pair: z-transform, then
//                  every sphere G of those columns picked out and scaled by 1/N.
// Only the sphere's bounding box survives each axis, so the traffic after the
// first kernel is K1 K2 N3 per pair instead of N1 N2 N3.
#include "internal.hpp"

namespace rpa {

namespace {

constexpr size_t kLdsBudget = 64 * 1024;

template <int DIR, typename T, class Addr>
__device__ cplx<T>* run_stages(cplx<T>* src, cplx<T>* dst, const FftPlan& plan, int N, int nlines, bool line_fast,
                               Addr addr, const cplx<T>* tw) {
    int Ns = 1;
    for (int s = 0; s < plan.nstages; ++s) {
        const int R = plan.radix[s];
        stockham_dispatch<DIR>(R, src, dst, N, Ns, nlines, line_fast, addr, tw, (int)threadIdx.x, (int)blockDim.x);
        __syncthreads();
        cplx<T>* t = src;
        src = dst;
        dst = t;
        Ns *= R;
    }
    return src;
}

template <typename T>
__global__ void k_fill_zero(cplx<T>* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = mk(T(0), T(0));
}

template <typename T>
__global__ void k_orb_scatter(const double* __restrict__ C, int nQ, const int32_t* __restrict__ map, size_t vol,
                              cplx<T>* __restrict__ phi) {
    const size_t b = blockIdx.y;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nQ; q += gridDim.x * blockDim.x) {
        const double* c = C + 2 * (b * nQ + q);
        phi[b * vol + map[q]] = mk(T(c[0]), T(c[1]));
    }
}

// Lines of length N: line L starts at (L / inner_count) * outer_stride + (L % inner_count) * inner_stride,
// element e of a line is e * es further. LB consecutive lines per workgroup.
template <typename T, int DIR>
__global__ __launch_bounds__(kFftThreads) void k_fft_axis(cplx<T>* data, int N, FftPlan plan, long long es,
                                                          long long inner_count, long long inner_stride,
                                                          long long outer_stride, long long nlines, int LB,
                                                          const cplx<T>* __restrict__ twg) {
    extern __shared__ __align__(16) unsigned char smem[];
    cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* a = tw + twiddle_len<T>(N);
    cplx<T>* b = a + (size_t)LB * N;
    const long long l0 = (long long)blockIdx.x * LB;
    const int nl = (int)min((long long)LB, nlines - l0);
    for (int t = threadIdx.x; t < twiddle_len<T>(N); t += blockDim.x) tw[t] = twg[t];
    auto gaddr = [&](int l, int e) -> long long {
        const long long L = l0 + l;
        return (L / inner_count) * outer_stride + (L % inner_count) * inner_stride + (long long)e * es;
    };
    const int tot = nl * N;
    if (es == 1) {
        for (int f = threadIdx.x; f < tot; f += blockDim.x) a[f] = data[gaddr(f / N, f % N)];
    } else {
        for (int f = threadIdx.x; f < tot; f += blockDim.x) {
            const int e = f / nl, l = f % nl;
            a[l * N + e] = data[gaddr(l, e)];
        }
    }
    __syncthreads();
    auto laddr = [N](int l, int e) { return l * N + e; };
    cplx<T>* res = run_stages<DIR>(a, b, plan, N, nl, false, laddr, tw);
    if (es == 1) {
        for (int f = threadIdx.x; f < tot; f += blockDim.x) data[gaddr(f / N, f % N)] = res[f];
    } else {
        for (int f = threadIdx.x; f < tot; f += blockDim.x) {
            const int e = f / nl, l = f % nl;
            data[gaddr(l, e)] = res[l * N + e];
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_pair_xy(const cplx<T>* __restrict__ phik,
                                                         const cplx<T>* __restrict__ phikq,
                                                         const int32_t* __restrict__ pn,
                                                         const int32_t* __restrict__ pm, int npairs, PairGeom g,
                                                         int PPW, const int32_t* __restrict__ kxg,
                                                         const int32_t* __restrict__ kyg,
                                                         const cplx<T>* __restrict__ tw1g,
                                                         const cplx<T>* __restrict__ tw2g, cplx<T>* __restrict__ tbuf) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N1 = g.N1, N2 = g.N2, N3 = g.N3, K1 = g.K1, K2 = g.K2;
    const int plane = N1 * N2;
    cplx<T>* tw1 = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* tw2 = tw1 + twiddle_len<T>(N1);
    cplx<T>* A = tw2 + twiddle_len<T>(N2);
    cplx<T>* B = A + (size_t)PPW * plane;
    int* kx = reinterpret_cast<int*>(B + (size_t)PPW * plane);
    int* ky = kx + K1;

    const int z = blockIdx.y;
    const int p0 = blockIdx.x * PPW;
    const int np = min(PPW, npairs - p0);
    const size_t vol = (size_t)plane * N3;
    for (int t = threadIdx.x; t < twiddle_len<T>(N1); t += blockDim.x) tw1[t] = tw1g[t];
    for (int t = threadIdx.x; t < twiddle_len<T>(N2); t += blockDim.x) tw2[t] = tw2g[t];
    for (int t = threadIdx.x; t < K1; t += blockDim.x) kx[t] = kxg[t];
    for (int t = threadIdx.x; t < K2; t += blockDim.x) ky[t] = kyg[t];

    // conj(phi_n) phi_m on this z-plane
    for (int f = threadIdx.x; f < np * plane; f += blockDim.x) {
        const int pp = f / plane, r = f - pp * plane;
        const size_t n = pn[p0 + pp], m = pm[p0 + pp];
        const size_t off = (size_t)z * plane + r;
        A[f] = cmulc(phik[n * vol + off], phikq[m * vol + off]);
    }
    __syncthreads();

    // forward transform along x on every line
    auto ax = [N1](int l, int e) { return l * N1 + e; };
    cplx<T>* rx = run_stages<-1>(A, B, g.p1, N1, np * N2, false, ax, tw1);
    cplx<T>* ox = (rx == A) ? B : A;
    // forward transform along y on the kept x-columns only
    auto ay = [=](int l, int e) {
        const int pp = l / K1;
        return pp * plane + e * N1 + kx[l - pp * K1];
    };
    cplx<T>* ry = run_stages<-1>(rx, ox, g.p2, N2, np * K1, true, ay, tw2);

    const int kk = K1 * K2;
    for (int f = threadIdx.x; f < np * kk; f += blockDim.x) {
        const int pp = f / kk, r = f - pp * kk;
        const int iy = r / K1, ix = r - iy * K1;
        tbuf[((size_t)(p0 + pp) * N3 + z) * kk + r] = ry[pp * plane + ky[iy] * N1 + kx[ix]];
    }
}

template <typename T>
__global__ __launch_bounds__(kFftThreads) void k_pair_z_gather(const cplx<T>* __restrict__ tbuf, PairGeom g, int CB,
                                                               const int32_t* __restrict__ zcol,
                                                               const int32_t* __restrict__ col_start,
                                                               const int32_t* __restrict__ col_g,
                                                               const int32_t* __restrict__ col_kz,
                                                               const cplx<T>* __restrict__ tw3g, T* __restrict__ rre,
                                                               T* __restrict__ rim) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N3 = g.N3, ncols = g.ncols;
    cplx<T>* tw3 = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* A = tw3 + twiddle_len<T>(N3);
    cplx<T>* B = A + (size_t)CB * N3;
    const size_t p = blockIdx.x;
    const int c0 = blockIdx.y * CB;
    const int nc = min(CB, g.nzc - c0);
    for (int t = threadIdx.x; t < twiddle_len<T>(N3); t += blockDim.x) tw3[t] = tw3g[t];
    for (int f = threadIdx.x; f < N3 * nc; f += blockDim.x) {
        const int z = f / nc, c = f - z * nc;
        A[z * CB + c] = tbuf[(p * N3 + z) * ncols + zcol[c0 + c]];
    }
    __syncthreads();
    auto az = [CB](int l, int e) { return e * CB + l; };
    cplx<T>* rz = run_stages<-1>(A, B, g.p3, N3, nc, true, az, tw3);

    const Split2<T> invN = split2<T>(1.0 / ((double)g.N1 * g.N2 * N3));
    const int e0 = col_start[c0], e1 = col_start[c0 + nc];
    T* ore = rre + p * g.NGp;
    T* oim = rim + p * g.NGp;
    for (int i = e0 + threadIdx.x; i < e1; i += blockDim.x) {
        const int gi = col_g[i];
        const int kz = col_kz[i] >> 16;      // packed (kz << 16) | column
        const int c = col_kz[i] & 0xffff;
        const cplx<T> v = rz[kz * CB + (c - c0)];
        ore[gi] = mulk(v.x, invN);
        oim[gi] = mulk(v.y, invN);
    }
    if (blockIdx.y == 0) {
        for (int gi = g.NG + threadIdx.x; gi < g.NGp; gi += blockDim.x) {
            ore[gi] = T(0);
            oim[gi] = T(0);
        }
    }
}

template <typename T>
size_t fft_axis_lines(int N) {
    size_t per = kLdsBudget / sizeof(cplx<T>);
    size_t lb = (per - twiddle_len<T>(N)) / (2 * (size_t)N);
    return lb < 1 ? 1 : lb;
}

}  // namespace

template <typename T>
hipError_t launch_fill_zero(cplx<T>* p, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_zero<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_orb_scatter(const double* C, int nbands, int nQ, const int32_t* map, size_t vol, cplx<T>* phi,
                              hipStream_t s) {
    if (!nbands || !nQ) return hipSuccess;
    unsigned bx = (unsigned)((nQ + 255) / 256);
    hipLaunchKernelGGL(k_orb_scatter<T>, dim3(bx, (unsigned)nbands), dim3(256), 0, s, C, nQ, map, vol, phi);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_axis(cplx<T>* data, int nb, int N1, int N2, int N3, int axis, const FftPlan& plan,
                           const cplx<T>* tw, int dir, hipStream_t s) {
    const long long V = (long long)N1 * N2 * N3;
    long long es, ic, is, os, nlines;
    int N;
    if (axis == 0) { N = N1; es = 1; ic = 1; is = 0; os = N1; nlines = (long long)nb * N3 * N2; }
    else if (axis == 1) { N = N2; es = N1; ic = N1; is = 1; os = (long long)N1 * N2; nlines = (long long)nb * N3 * N1; }
    else { N = N3; es = (long long)N1 * N2; ic = (long long)N1 * N2; is = 1; os = V; nlines = (long long)nb * N1 * N2; }
    const int LB = (int)fft_axis_lines<T>(N);
    const size_t lds = ((size_t)twiddle_len<T>(N) + 2 * (size_t)LB * N) * sizeof(cplx<T>);
    const unsigned blocks = (unsigned)((nlines + LB - 1) / LB);
    if (dir > 0)
        hipLaunchKernelGGL((k_fft_axis<T, 1>), dim3(blocks), dim3(kFftThreads), lds, s, data, N, plan, es, ic, is, os,
                           nlines, LB, tw);
    else
        hipLaunchKernelGGL((k_fft_axis<T, -1>), dim3(blocks), dim3(kFftThreads), lds, s, data, N, plan, es, ic, is, os,
                           nlines, LB, tw);
    return hipGetLastError();
}

template <typename T>
int pair_xy_ppw(const PairGeom& g) {
    const size_t plane = (size_t)g.N1 * g.N2;
    const size_t fixed = (twiddle_len<T>(g.N1) + twiddle_len<T>(g.N2)) * sizeof(cplx<T>) + (g.K1 + g.K2) * sizeof(int);
    const size_t per = 2 * plane * sizeof(cplx<T>);
    size_t budget = kLdsBudget;
    if (fixed + per > budget) budget = 160 * 1024;
    size_t ppw = (budget - fixed) / per;
    if (ppw < 1) ppw = 0;
    if (ppw > 8) ppw = 8;
    return (int)ppw;
}

template <typename T>
hipError_t launch_pair_xy(const cplx<T>* phik, const cplx<T>* phikq, const int32_t* pn, const int32_t* pm, int npairs,
                          const PairGeom& g, const int32_t* kx_grid, const int32_t* ky_grid, const cplx<T>* tw1,
                          const cplx<T>* tw2, cplx<T>* tbuf, hipStream_t s) {
    if (!npairs) return hipSuccess;
    const int PPW = pair_xy_ppw<T>(g);
    if (PPW < 1) return hipErrorInvalidValue;
    const size_t plane = (size_t)g.N1 * g.N2;
    const size_t lds = (twiddle_len<T>(g.N1) + twiddle_len<T>(g.N2)) * sizeof(cplx<T>) +
                       2 * PPW * plane * sizeof(cplx<T>) + (g.K1 + g.K2) * sizeof(int);
    dim3 grid((unsigned)((npairs + PPW - 1) / PPW), (unsigned)g.N3);
    hipLaunchKernelGGL(k_pair_xy<T>, grid, dim3(kFftThreads), lds, s, phik, phikq, pn, pm, npairs, g, PPW, kx_grid,
                       ky_grid, tw1, tw2, tbuf);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pair_z_gather(const cplx<T>* tbuf, int npairs, const PairGeom& g, const int32_t* zcol,
                                const int32_t* col_start, const int32_t* col_g, const int32_t* col_kz,
                                const cplx<T>* tw3, T* rho_re, T* rho_im, hipStream_t s) {
    if (!npairs) return hipSuccess;
    if (g.nzc < 1 || g.nzc > g.ncols) return hipErrorInvalidValue;
    size_t per = kLdsBudget / sizeof(cplx<T>);
    int CB = (int)((per - twiddle_len<T>(g.N3)) / (2 * (size_t)g.N3));
    if (CB > g.nzc) CB = g.nzc;
    if (CB < 1) return hipErrorInvalidValue;
    const size_t lds = ((size_t)twiddle_len<T>(g.N3) + 2 * (size_t)CB * g.N3) * sizeof(cplx<T>);
    dim3 grid((unsigned)npairs, (unsigned)((g.nzc + CB - 1) / CB));
    hipLaunchKernelGGL(k_pair_z_gather<T>, grid, dim3(kFftThreads), lds, s, tbuf, g, CB, zcol, col_start, col_g,
                       col_kz, tw3, rho_re, rho_im);
    return hipGetLastError();
}

#define RPA_INST(T)                                                                                                 \
    template hipError_t launch_fill_zero<T>(cplx<T>*, size_t, hipStream_t);                                         \
    template hipError_t launch_orb_scatter<T>(const double*, int, int, const int32_t*, size_t, cplx<T>*,            \
                                              hipStream_t);                                                         \
    template hipError_t launch_fft_axis<T>(cplx<T>*, int, int, int, int, int, const FftPlan&, const cplx<T>*, int,  \
                                           hipStream_t);                                                            \
    template hipError_t launch_pair_xy<T>(const cplx<T>*, const cplx<T>*, const int32_t*, const int32_t*, int,      \
                                          const PairGeom&, const int32_t*, const int32_t*, const cplx<T>*,          \
                                          const cplx<T>*, cplx<T>*, hipStream_t);                                   \
    template hipError_t launch_pair_z_gather<T>(const cplx<T>*, int, const PairGeom&, const int32_t*,              \
                                                const int32_t*, const int32_t*, const int32_t*, const cplx<T>*, T*,  \
                                                T*, hipStream_t);
RPA_INST(double)
RPA_INST(float)
#undef RPA_INST

}  // namespace rpa
