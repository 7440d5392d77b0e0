// PAW correction of the pair densities on MFMA (Eq. n_G_2, Table 1 steps 7-9):
//   rho_nm(G) += sum_a sum_ij conj(P^a_ni) P'^a_mj Q^a_ij(q+G)
// factorised per band m of the k+q set (pairs come m-major, so the pairs of one m are adjacent):
//   Z_m[a i][G] = sum_j Q^a_ij(q+G) P'^a_mj                     (k_paw_z, once per m of a chunk)
//   rho_p[G]  += sum_{a i} conj(P_{n_p}[a i]) Z_{m_p}[a i][G]    (k_paw_mm, a GEMM with K = sum_a Np_a)
// The GEMM runs on v_mfma_f32_16x16x4_f32 (FP32 path, exact FP32 products) or
// v_mfma_f64_16x16x4_f64 (FP64 path). Complex products as four real ones:
//   Re += Pr Zr + Pi Zi,  Im += Pr Zi - Pi Zr   (P conjugated).
#include "internal.hpp"

namespace rpa {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    typedef v4f acc;
    static __device__ __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // output element r of lane l: row 4 (l / 16) + r, column l % 16
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mfma<double> {
    typedef v4d acc;
    static __device__ __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // output element r of lane l: row l / 16 + 4 r, column l % 16
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// Z[s][ai][g] for m = m_lo + s: sum_j Q[qoff_a + i Np_a + j][g] P'[m][a j]; zero for g >= NG. A thread
// takes kZSlots consecutive bands m, so each element of Q is read once per kZSlots bands.
constexpr int kZSlots = 8;
template <typename T>
__global__ __launch_bounds__(256) void k_paw_z(const double* __restrict__ Pkq, int ldP, int m_lo, int nslots,
                                               const int32_t* __restrict__ proj_off, const int32_t* __restrict__ qoff,
                                               int natoms, int nproj, const double* __restrict__ Q, int NG, int NGp,
                                               T* __restrict__ Zr, T* __restrict__ Zi) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int ai = blockIdx.y;
    const int s0 = blockIdx.z * kZSlots;
    if (g >= NGp) return;
    int a = 0;
    while (a + 1 < natoms && proj_off[a + 1] <= ai) ++a;
    const int lo = proj_off[a], np = proj_off[a + 1] - lo, i = ai - lo;
    const int ns = min(kZSlots, nslots - s0);
    double sr[kZSlots], si[kZSlots];
#pragma unroll
    for (int t = 0; t < kZSlots; ++t) {
        sr[t] = 0.0;
        si[t] = 0.0;
    }
    if (g < NG) {
        const double* qrow = Q + 2 * ((size_t)(qoff[a] + i * np) * NG + g);
        for (int j = 0; j < np; ++j) {
            const double qr = qrow[2 * (size_t)j * NG], qi = qrow[2 * (size_t)j * NG + 1];
#pragma unroll
            for (int t = 0; t < kZSlots; ++t) {
                // slots past the last are clamped to it (computed and not stored)
                const size_t m = (size_t)(m_lo + s0 + min(t, ns - 1));
                const double pr = Pkq[2 * (m * ldP + lo + j)], pi = Pkq[2 * (m * ldP + lo + j) + 1];
                sr[t] += qr * pr - qi * pi;
                si[t] += qr * pi + qi * pr;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kZSlots; ++t) {
        if (t < ns) {
            const size_t o = ((size_t)(s0 + t) * nproj + ai) * NGp + g;
            Zr[o] = T(sr[t]);
            Zi[o] = T(si[t]);
        }
    }
}

// Y[s][aj][g] for n = n_lo + s: sum_i conj(P[n][a i]) Q[qoff_a + i Np_a + j][g]; zero for g >= NG. As in
// k_paw_z a thread takes kZSlots consecutive bands n, so each element of Q is read once per kZSlots bands.
template <typename T>
__global__ __launch_bounds__(256) void k_paw_yn(const double* __restrict__ Pk, int ldP, int n_lo, int nslots,
                                                const int32_t* __restrict__ proj_off, const int32_t* __restrict__ qoff,
                                                int natoms, int nproj, const double* __restrict__ Q, int NG, int NGp,
                                                T* __restrict__ Yr, T* __restrict__ Yi) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int aj = blockIdx.y;
    const int s0 = blockIdx.z * kZSlots;
    if (g >= NGp) return;
    int a = 0;
    while (a + 1 < natoms && proj_off[a + 1] <= aj) ++a;
    const int lo = proj_off[a], np = proj_off[a + 1] - lo, j = aj - lo;
    const int ns = min(kZSlots, nslots - s0);
    double sr[kZSlots], si[kZSlots];
#pragma unroll
    for (int t = 0; t < kZSlots; ++t) {
        sr[t] = 0.0;
        si[t] = 0.0;
    }
    if (g < NG) {
        const double* qcol = Q + 2 * ((size_t)(qoff[a] + j) * NG + g);
        for (int i = 0; i < np; ++i) {
            const double qr = qcol[2 * (size_t)i * np * NG], qi = qcol[2 * (size_t)i * np * NG + 1];
#pragma unroll
            for (int t = 0; t < kZSlots; ++t) {
                // slots past the last are clamped to it (computed and not stored)
                const size_t n = (size_t)(n_lo + s0 + min(t, ns - 1));
                const double pr = Pk[2 * (n * ldP + lo + i)], pi = Pk[2 * (n * ldP + lo + i) + 1];
                // conj(p) q
                sr[t] += pr * qr + pi * qi;
                si[t] += pr * qi - pi * qr;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kZSlots; ++t) {
        if (t < ns) {
            const size_t o = ((size_t)(s0 + t) * nproj + aj) * NGp + g;
            Yr[o] = T(sr[t]);
            Yi[o] = T(si[t]);
        }
    }
}

// One workgroup per (64 G-vectors, 64 consecutive pairs of the chunk). The pairs of the window are taken
// in runs of equal m (one GEMM pass per run: the B operand Z_m is shared by the run's rows); rows outside
// the run are computed and discarded.
constexpr int kPawKB = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_paw_mm(const T* __restrict__ Zr, const T* __restrict__ Zi, int nproj,
                                                const double* __restrict__ Pk, int ldP, const int32_t* __restrict__ pn,
                                                const int32_t* __restrict__ pm, int npairs, int m_lo, int NGp,
                                                T* __restrict__ rre, T* __restrict__ rim) {
    typedef typename Mfma<T>::acc acc_t;
    __shared__ T sAr[64][kPawKB + 1], sAi[64][kPawKB + 1];
    __shared__ T sBr[kPawKB][64 + 4], sBi[kPawKB][64 + 4];
    __shared__ int s_m[64];
    const int g0 = blockIdx.x * 64;
    const int p0 = blockIdx.y * 64;
    const int nrows = min(64, npairs - p0);
    if (nrows <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid < 64) s_m[tid] = tid < nrows ? pm[p0 + tid] : -1;
    __syncthreads();
    // staging roles: A row ar, k ak .. ak+3; B k-row bk, columns bc .. bc+3
    const int ar = tid >> 2, ak = (tid & 3) * 4;
    const int bk = tid >> 4, bc = (tid & 15) * 4;
    const size_t nA = ar < nrows ? (size_t)pn[p0 + ar] : 0;
    int r0 = 0;
    while (r0 < nrows) {
        const int m = s_m[r0];
        int r1 = r0 + 1;
        while (r1 < nrows && s_m[r1] == m) ++r1;
        const size_t zb = (size_t)(m - m_lo) * nproj * NGp;
        acc_t accR[4], accI[4];
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            accR[y] = acc_t{0, 0, 0, 0};
            accI[y] = acc_t{0, 0, 0, 0};
        }
        for (int kb = 0; kb < nproj; kb += kPawKB) {
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = kb + ak + e;
                double vr = 0.0, vi = 0.0;
                if (k < nproj && ar < nrows) {
                    vr = Pk[2 * (nA * ldP + k)];
                    vi = Pk[2 * (nA * ldP + k) + 1];
                }
                sAr[ar][ak + e] = T(vr);
                sAi[ar][ak + e] = T(vi);
            }
            {
                const int k = kb + bk;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    T vr = T(0), vi = T(0);
                    if (k < nproj) {
                        const size_t o = zb + (size_t)k * NGp + g0 + bc + e;
                        vr = Zr[o];
                        vi = Zi[o];
                    }
                    sBr[bk][bc + e] = vr;
                    sBi[bk][bc + e] = vi;
                }
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < kPawKB; kk += 4) {
                const int kr = kk + (lane >> 4), rc = lane & 15;
                const T a_r = sAr[16 * wave + rc][kr], a_i = sAi[16 * wave + rc][kr];
                const T a_n = -a_i;
#pragma unroll
                for (int y = 0; y < 4; ++y) {
                    const T b_r = sBr[kr][16 * y + rc], b_i = sBi[kr][16 * y + rc];
                    accR[y] = Mfma<T>::step(a_r, b_r, accR[y]);
                    accR[y] = Mfma<T>::step(a_i, b_i, accR[y]);
                    accI[y] = Mfma<T>::step(a_r, b_i, accI[y]);
                    accI[y] = Mfma<T>::step(a_n, b_r, accI[y]);
                }
            }
        }
        // rows of this run only
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = 16 * wave + Mfma<T>::row(lane, r);
                if (row >= r0 && row < r1) {
                    const size_t o = (size_t)(p0 + row) * NGp + g0 + 16 * y + (lane & 15);
                    rre[o] += accR[y][r];
                    rim[o] += accI[y][r];
                }
            }
        r0 = r1;
    }
}

// The n-factorised form, for chunks whose pairs span fewer bands n than bands m:
//   Y_n[aj][G] = sum_i conj(P_ni) Q^a_ij(G)             (k_paw_yn, once per band n of a chunk)
//   rho_p[G]  += sum_{aj} P'_{m_p}[aj] Y_{n_p}[aj][G]   (this kernel, K = sum_a Np_a)
// One workgroup per (64 G-vectors, segment of at most 64 pairs with one band n): seg holds per segment
// (n - n_lo, first, count) into perm, the chunk's pair indices grouped by n; the B operand Y_n is shared
// by the segment's rows, the A rows are the pairs' P'_m, and the results go to the pairs' own rows.
template <typename T>
__global__ __launch_bounds__(256) void k_paw_mm_n(const T* __restrict__ Yr, const T* __restrict__ Yi, int nproj,
                                                  const double* __restrict__ Pkq, int ldP,
                                                  const int32_t* __restrict__ pm, const int32_t* __restrict__ seg,
                                                  const int32_t* __restrict__ perm, int NGp, T* __restrict__ rre,
                                                  T* __restrict__ rim) {
    typedef typename Mfma<T>::acc acc_t;
    __shared__ T sAr[64][kPawKB + 1], sAi[64][kPawKB + 1];
    __shared__ T sBr[kPawKB][64 + 4], sBi[kPawKB][64 + 4];
    const int g0 = blockIdx.x * 64;
    const int ns = seg[3 * blockIdx.y], f = seg[3 * blockIdx.y + 1], nrows = seg[3 * blockIdx.y + 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // staging roles: A row ar, k ak .. ak+3; B k-row bk, columns bc .. bc+3
    const int ar = tid >> 2, ak = (tid & 3) * 4;
    const int bk = tid >> 4, bc = (tid & 15) * 4;
    const size_t mA = ar < nrows ? (size_t)pm[perm[f + ar]] : 0;
    const size_t yb = (size_t)ns * nproj * NGp;
    acc_t accR[4], accI[4];
#pragma unroll
    for (int y = 0; y < 4; ++y) {
        accR[y] = acc_t{0, 0, 0, 0};
        accI[y] = acc_t{0, 0, 0, 0};
    }
    for (int kb = 0; kb < nproj; kb += kPawKB) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = kb + ak + e;
            double vr = 0.0, vi = 0.0;
            if (k < nproj && ar < nrows) {
                vr = Pkq[2 * (mA * ldP + k)];
                vi = Pkq[2 * (mA * ldP + k) + 1];
            }
            sAr[ar][ak + e] = T(vr);
            sAi[ar][ak + e] = T(vi);
        }
        {
            const int k = kb + bk;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                T vr = T(0), vi = T(0);
                if (k < nproj) {
                    const size_t o = yb + (size_t)k * NGp + g0 + bc + e;
                    vr = Yr[o];
                    vi = Yi[o];
                }
                sBr[bk][bc + e] = vr;
                sBi[bk][bc + e] = vi;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kPawKB; kk += 4) {
            const int kr = kk + (lane >> 4), rc = lane & 15;
            const T a_r = sAr[16 * wave + rc][kr], a_i = sAi[16 * wave + rc][kr];
            const T a_n = -a_i;
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                // (Ar + i Ai)(Br + i Bi) = Ar Br - Ai Bi + i (Ar Bi + Ai Br)
                const T b_r = sBr[kr][16 * y + rc], b_i = sBi[kr][16 * y + rc];
                accR[y] = Mfma<T>::step(a_r, b_r, accR[y]);
                accR[y] = Mfma<T>::step(a_n, b_i, accR[y]);
                accI[y] = Mfma<T>::step(a_r, b_i, accI[y]);
                accI[y] = Mfma<T>::step(a_i, b_r, accI[y]);
            }
        }
    }
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * wave + Mfma<T>::row(lane, r);
            if (row < nrows) {
                const size_t o = (size_t)perm[f + row] * NGp + g0 + 16 * y + (lane & 15);
                rre[o] += accR[y][r];
                rim[o] += accI[y][r];
            }
        }
}

}  // namespace

template <typename T>
hipError_t launch_paw_mfma(const double* Pk, const double* Pkq, int ldP, const int32_t* pn, const int32_t* pm,
                           int npairs, int m_lo, int nslots, const int32_t* proj_off, const int32_t* qoff, int natoms,
                           int nproj, const double* Q, int NG, int NGp, T* Zr, T* Zi, T* rre, T* rim, hipStream_t s) {
    if (!npairs || !nproj) return hipSuccess;
    if (NGp % 64) return hipErrorInvalidValue;
    dim3 gz((unsigned)((NGp + 255) / 256), (unsigned)nproj, (unsigned)((nslots + kZSlots - 1) / kZSlots));
    hipLaunchKernelGGL(k_paw_z<T>, gz, dim3(256), 0, s, Pkq, ldP, m_lo, nslots, proj_off, qoff, natoms, nproj, Q, NG,
                       NGp, Zr, Zi);
    dim3 gm((unsigned)(NGp / 64), (unsigned)((npairs + 63) / 64));
    hipLaunchKernelGGL(k_paw_mm<T>, gm, dim3(256), 0, s, Zr, Zi, nproj, Pk, ldP, pn, pm, npairs, m_lo, NGp, rre, rim);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_paw_yn(const double* Pk, int ldP, int n_lo, int nslots, const int32_t* proj_off, const int32_t* qoff,
                         int natoms, int nproj, const double* Q, int NG, int NGp, T* Yr, T* Yi, hipStream_t s) {
    if (!nslots || !nproj) return hipSuccess;
    dim3 grid((unsigned)((NGp + 255) / 256), (unsigned)nproj, (unsigned)((nslots + kZSlots - 1) / kZSlots));
    hipLaunchKernelGGL(k_paw_yn<T>, grid, dim3(256), 0, s, Pk, ldP, n_lo, nslots, proj_off, qoff, natoms, nproj, Q, NG,
                       NGp, Yr, Yi);
    return hipGetLastError();
}

template hipError_t launch_paw_yn<float>(const double*, int, int, int, const int32_t*, const int32_t*, int, int,
                                         const double*, int, int, float*, float*, hipStream_t);
template hipError_t launch_paw_yn<double>(const double*, int, int, int, const int32_t*, const int32_t*, int, int,
                                          const double*, int, int, double*, double*, hipStream_t);

template <typename T>
hipError_t launch_paw_mfma_n(const T* Yr, const T* Yi, int nproj, const double* Pkq, int ldP, const int32_t* pm,
                             const int32_t* seg, int nseg, const int32_t* perm, int NGp, T* rre, T* rim,
                             hipStream_t s) {
    if (!nseg || !nproj) return hipSuccess;
    if (NGp % 64) return hipErrorInvalidValue;
    dim3 grid((unsigned)(NGp / 64), (unsigned)nseg);
    hipLaunchKernelGGL(k_paw_mm_n<T>, grid, dim3(256), 0, s, Yr, Yi, nproj, Pkq, ldP, pm, seg, perm, NGp, rre, rim);
    return hipGetLastError();
}

template hipError_t launch_paw_mfma_n<float>(const float*, const float*, int, const double*, int, const int32_t*,
                                             const int32_t*, int, const int32_t*, int, float*, float*, hipStream_t);
template hipError_t launch_paw_mfma_n<double>(const double*, const double*, int, const double*, int, const int32_t*,
                                              const int32_t*, int, const int32_t*, int, double*, double*,
                                              hipStream_t);

template hipError_t launch_paw_mfma<float>(const double*, const double*, int, const int32_t*, const int32_t*, int,
                                           int, int, const int32_t*, const int32_t*, int, int, const double*, int,
                                           int, float*, float*, float*, float*, hipStream_t);
template hipError_t launch_paw_mfma<double>(const double*, const double*, int, const int32_t*, const int32_t*, int,
                                            int, int, const int32_t*, const int32_t*, int, int, const double*, int,
                                            int, double*, double*, double*, double*, hipStream_t);

}  // namespace rpa
