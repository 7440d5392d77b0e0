// Dense stages of the chi0 / E_c path:
//   PAW correction of the pair densities (Eq. n_G_2, Table 1 steps 7-9),
//   optical-limit row at q = 0 (Eq. n_q0, Eq. nabla, Eq. Q_q0, step 10),
//   real transition weights (Eq. chi0, Eq. A_iw),
//   grouped complex rank-k update of chi0 (Eq. zher_multi, step 11) on FP64 MFMA,
//   E_c(q) from a blocked FP64 Cholesky factorisation of 1 - K (Eq. rpa, step 13).
//
// Matrices of the rank-k update and of the factorisation are planar (separate
// real and imaginary arrays), row-major, with a padded leading dimension that is
// a multiple of the 64-wide tile.
#include "internal.hpp"

namespace rpa {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ cplx<double> ld_c128(const double* p, size_t i) { return mk(p[2 * i], p[2 * i + 1]); }

// ------------------------------------------------------------------- PAW
// Y[s][aj][g] = sum_i conj(P_k[n_s][a, i]) Q[qoff_a + i Np_a + j][g]
template <typename T>
__global__ void k_paw_y(const double* __restrict__ Pk, int ldP, const int32_t* __restrict__ nlist,
                        const int32_t* __restrict__ proj_off, const int32_t* __restrict__ qoff, int natoms,
                        int nprojtot, const double* __restrict__ Q, int NG, int NGp, T* __restrict__ Yre,
                        T* __restrict__ Yim) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int aj = blockIdx.y;
    const int s = blockIdx.z;
    if (g >= NGp) return;
    int a = 0;
    while (a + 1 < natoms && proj_off[a + 1] <= aj) ++a;
    const int lo = proj_off[a], np = proj_off[a + 1] - lo, j = aj - lo;
    const size_t n = nlist[s];
    cplx<double> acc = mk(0.0, 0.0);
    if (g < NG) {
        for (int i = 0; i < np; ++i) {
            const cplx<double> p = ld_c128(Pk, n * ldP + lo + i);
            const cplx<double> q = ld_c128(Q, (size_t)(qoff[a] + i * np + j) * NG + g);
            acc = acc + cmulc(p, q);
        }
    }
    const size_t o = ((size_t)s * nprojtot + aj) * NGp + g;
    Yre[o] = T(acc.x);
    Yim[o] = T(acc.y);
}

// rho[p][g] += sum_aj Y[n_p - nlo][aj][g] P_kq[m_p][aj]
constexpr int kPawPairs = 8;
template <typename T>
__global__ __launch_bounds__(256) void k_paw_add(const T* __restrict__ Yre, const T* __restrict__ Yim,
                                                 const int32_t* __restrict__ pn, int nlo,
                                                 const int32_t* __restrict__ pm,
                                                 const double* __restrict__ Pkq, int ldP, int nprojtot, int npairs,
                                                 int NG, int NGp, T* __restrict__ rre, T* __restrict__ rim) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* pr = reinterpret_cast<T*>(smem);
    T* pi = pr + kPawPairs * nprojtot;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int p0 = blockIdx.y * kPawPairs;
    const int np = min(kPawPairs, npairs - p0);
    for (int e = threadIdx.x; e < np * nprojtot; e += blockDim.x) {
        const int pp = e / nprojtot, aj = e - pp * nprojtot;
        const cplx<double> v = ld_c128(Pkq, (size_t)pm[p0 + pp] * ldP + aj);
        pr[e] = T(v.x);
        pi[e] = T(v.y);
    }
    __syncthreads();
    if (g >= NG) return;
    for (int pp = 0; pp < np; ++pp) {
        const size_t yb = (size_t)(pn[p0 + pp] - nlo) * nprojtot * NGp + g;
        T sr = T(0), si = T(0);
        for (int aj = 0; aj < nprojtot; ++aj) {
            const T yr = Yre[yb + (size_t)aj * NGp], yi = Yim[yb + (size_t)aj * NGp];
            const T xr = pr[pp * nprojtot + aj], xi = pi[pp * nprojtot + aj];
            sr += yr * xr - yi * xi;
            si += yr * xi + yi * xr;
        }
        const size_t o = (size_t)(p0 + pp) * NGp + g;
        rre[o] += sr;
        rim[o] += si;
    }
}

// ---------------------------------------------------------------- optical
// rho[p][g0] = [sum_Q conj(Ck_n) Ckq_m wq - i sum_a sum_ij conj(Pk_ni) Dq_ij Pkq_mj] / (e_m - e_n)
template <typename T>
__global__ __launch_bounds__(256) void k_optical_row(const double* __restrict__ Ck, const double* __restrict__ Ckq,
                                                     int nQ, const double* __restrict__ wq,
                                                     const double* __restrict__ Pk, const double* __restrict__ Pkq,
                                                     int ldP, const double* __restrict__ Dq,
                                                     const int32_t* __restrict__ proj_off,
                                                     const int32_t* __restrict__ qoff, int natoms,
                                                     const double* __restrict__ epsk, const double* __restrict__ epskq,
                                                     const int32_t* __restrict__ pn, const int32_t* __restrict__ pm,
                                                     int g0, int NGp, T* __restrict__ rre, T* __restrict__ rim) {
    __shared__ double red[4][256];
    const int p = blockIdx.x;
    const size_t n = pn[p], m = pm[p];
    double mr = 0, mi = 0, dr = 0, di = 0;
    for (int q = threadIdx.x; q < nQ; q += blockDim.x) {
        const cplx<double> c = cmulc(ld_c128(Ck, n * nQ + q), ld_c128(Ckq, m * nQ + q));
        mr += c.x * wq[q];
        mi += c.y * wq[q];
    }
    const int nq2 = qoff[natoms];
    for (int e = threadIdx.x; e < nq2; e += blockDim.x) {
        int a = 0;
        while (a + 1 < natoms && qoff[a + 1] <= e) ++a;
        const int np = proj_off[a + 1] - proj_off[a];
        const int r = e - qoff[a], i = r / np, j = r - i * np;
        const cplx<double> t = cmulc(ld_c128(Pk, n * ldP + proj_off[a] + i), ld_c128(Pkq, m * ldP + proj_off[a] + j));
        dr += t.x * Dq[e];
        di += t.y * Dq[e];
    }
    red[0][threadIdx.x] = mr;
    red[1][threadIdx.x] = mi;
    red[2][threadIdx.x] = dr;
    red[3][threadIdx.x] = di;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 4; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double den = epskq[m] - epsk[n];
        // numerator = mom - i * paw
        const double nr = red[0][0] + red[3][0];
        const double ni = red[1][0] - red[2][0];
        rre[(size_t)p * NGp + g0] = T(nr / den);
        rim[(size_t)p * NGp + g0] = T(ni / den);
    }
}

// Intraband head at q -> 0: term[b] = w (-df/de)_n (qhat.v_n)^2 for the listed bands n = band[b], with the
// band velocity qhat.v_n = sum_Q |C_n(Q)|^2 wq(Q) - i sum_a sum_ij conj(P_ni) Dq_ij P_nj (the diagonal of
// the optical row's numerator); one workgroup per band
__global__ __launch_bounds__(256) void k_band_drude(const double* __restrict__ C, int nQ,
                                                    const double* __restrict__ wq, const double* __restrict__ P,
                                                    int ldP, const double* __restrict__ Dq,
                                                    const int32_t* __restrict__ proj_off,
                                                    const int32_t* __restrict__ qoff, int natoms,
                                                    const int32_t* __restrict__ band, const double* __restrict__ mdf,
                                                    double weight, double* __restrict__ term) {
    __shared__ double red[2][256];
    const int b = blockIdx.x;
    const size_t n = band[b];
    double mr = 0, di = 0;
    for (int q = threadIdx.x; q < nQ; q += blockDim.x) {
        const cplx<double> c = ld_c128(C, n * nQ + q);
        mr += (c.x * c.x + c.y * c.y) * wq[q];
    }
    const int nq2 = natoms > 0 ? qoff[natoms] : 0;
    for (int e = threadIdx.x; e < nq2; e += blockDim.x) {
        int a = 0;
        while (a + 1 < natoms && qoff[a + 1] <= e) ++a;
        const int np = proj_off[a + 1] - proj_off[a];
        const int r = e - qoff[a], i = r / np, j = r - i * np;
        const cplx<double> t = cmulc(ld_c128(P, n * ldP + proj_off[a] + i), ld_c128(P, n * ldP + proj_off[a] + j));
        di += t.y * Dq[e];
    }
    red[0][threadIdx.x] = mr;
    red[1][threadIdx.x] = di;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // real part of (mom - i paw): mom is real (|C|^2 weights), paw = i * di for real antisymmetric D
        const double v = red[0][0] + red[1][0];
        term[b] = weight * mdf[b] * v * v;
    }
}

// chi0_00(w) += -(sum of the terms)/(Omega w^2), one thread per frequency
__global__ void k_add_drude(const double* __restrict__ term, int nterms, const double* __restrict__ omega, int nw,
                            double inv_volume, double* __restrict__ head, long long stride) {
    const int w = threadIdx.x;
    if (w >= nw) return;
    double s = 0;
    for (int b = 0; b < nterms; ++b) s += term[b];
    head[(size_t)w * stride] += -s * inv_volume / (omega[w] * omega[w]);
}

// ---------------------------------------------------------------- weights
// Real frequencies w + i eta: rows w < nw hold Re a, rows nw + w hold Im a, with
// a = prefac (f_n - f_m) [1/(w + i eta + d) - 1/(w + i eta - d)], d = e_n - e_m
__global__ void k_weights_real(const double* __restrict__ epsk, const double* __restrict__ epskq,
                               const double* __restrict__ fk, const double* __restrict__ fkq,
                               const int32_t* __restrict__ pn, const int32_t* __restrict__ pm, int npairs,
                               const double* __restrict__ omega, int nw, double eta, double prefac,
                               double* __restrict__ a, int lda) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= lda) return;
    if (p >= npairs) {
        for (int w = 0; w < 2 * nw; ++w) a[(size_t)w * lda + p] = 0.0;
        return;
    }
    const double d = epsk[pn[p]] - epskq[pm[p]];
    const double df = fk[pn[p]] - fkq[pm[p]];
    for (int w = 0; w < nw; ++w) {
        const double x = omega[w];
        // 1/(x + d + i eta) - 1/(x - d + i eta)
        const double u = x + d, v = x - d, e2 = eta * eta;
        const double du = u * u + e2, dv = v * v + e2;
        const double re = u / du - v / dv;
        const double im = -eta / du + eta / dv;
        a[(size_t)w * lda + p] = prefac * df * re;
        a[(size_t)(nw + w) * lda + p] = prefac * df * im;
    }
}

// Real-frequency intraband head: head[w] += s Re(1/(Omega z^2)), head[nw + w] += s Im(1/(Omega z^2)),
// z = w + i eta, s the sum of the terms
__global__ void k_add_drude_real(const double* __restrict__ term, int nterms, const double* __restrict__ omega,
                                 int nw, double eta, double inv_volume, double* __restrict__ head, long long stride) {
    const int w = threadIdx.x;
    if (w >= nw) return;
    double s = 0;
    for (int b = 0; b < nterms; ++b) s += term[b];
    const double x = omega[w];
    // 1/z^2 = (x^2 - eta^2 - 2 i x eta)/((x^2 - eta^2)^2 + 4 x^2 eta^2)
    const double rr = x * x - eta * eta, ii = -2.0 * x * eta, den = rr * rr + ii * ii;
    head[(size_t)w * stride] += s * inv_volume * rr / den;
    head[(size_t)(nw + w) * stride] += s * inv_volume * ii / den;
}

// out[w] = A_w + i B_w for the Hermitian accumulators A_w (row block w) and B_w (row block nw + w), each
// stored as its lower triangle (real and imaginary planes)
__global__ void k_chi_out_real(const double* __restrict__ Cre, const double* __restrict__ Cim, int ldC,
                               long long sC, int NG, int nw, double* __restrict__ out) {
    const int i = blockIdx.x, w = blockIdx.y;
    const double* ar = Cre + (size_t)w * sC;
    const double* ai = Cim + (size_t)w * sC;
    const double* br = Cre + (size_t)(nw + w) * sC;
    const double* bi = Cim + (size_t)(nw + w) * sC;
    double* o = out + 2 * ((size_t)w * NG * NG + (size_t)i * NG);
    for (int j = threadIdx.x; j < NG; j += blockDim.x) {
        double are, aim, bre, bim;
        if (j <= i) {
            const size_t e = (size_t)i * ldC + j;
            are = ar[e]; aim = ai[e]; bre = br[e]; bim = bi[e];
        } else {
            const size_t e = (size_t)j * ldC + i;
            are = ar[e]; aim = -ai[e]; bre = br[e]; bim = -bi[e];
        }
        // (are + i aim) + i (bre + i bim)
        o[2 * j] = are - bim;
        o[2 * j + 1] = aim + bre;
    }
}

__global__ void k_weights(const double* __restrict__ epsk, const double* __restrict__ epskq,
                          const double* __restrict__ fk, const double* __restrict__ fkq, const int32_t* __restrict__ pn,
                          const int32_t* __restrict__ pm, int npairs, const double* __restrict__ omega, int nw,
                          double prefac, double* __restrict__ a, int lda) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= lda) return;
    if (p >= npairs) {
        for (int w = 0; w < nw; ++w) a[(size_t)w * lda + p] = 0.0;
        return;
    }
    const double d = epsk[pn[p]] - epskq[pm[p]];
    const double df = fk[pn[p]] - fkq[pm[p]];
    for (int w = 0; w < nw; ++w) {
        const double om = omega[w];
        a[(size_t)w * lda + p] = prefac * df * 2.0 * d / (om * om + d * d);
    }
}

// ------------------------------------------------------------ FP64 HERK
// One 64x64 lower tile (I >= J) of one batch entry per workgroup; four waves,
// each a 32x32 quadrant as 2x2 blocks of v_mfma_f64_16x16x4f64.
// Fragment layouts (16x16x4 f64): A lane l holds A[l%16][l/16], B lane l holds
// B[l/16][l%16], D lane l element r holds D[l/16 + 4*r][l%16] (rows interleave
// across the four lane groups, unlike the 16-bit-input MFMAs).
// K-stage of the FP64 rank-k kernel. Stages of 8 (32 KB of LDS, double-buffered) with registers bounded
// for three workgroups per CU hide more latency (48 x 1408^2 at K = 256: 57.7 against 51.9 TFLOP/s for
// stages of 16 at two per CU) and serve the chi0 update and the Cholesky trailing updates (K = 128, once
// per pair of panels). Stages of 16 at two per CU serve K <= 64.
template <int BK> struct HerkF64Cfg;
template <> struct HerkF64Cfg<8> { static constexpr int waves_per_simd = 3; };
template <> struct HerkF64Cfg<16> { static constexpr int waves_per_simd = 2; };

__device__ __forceinline__ void tile_of(int t, int& I, int& J) {
    int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    I = i;
    J = t - i * (i + 1) / 2;
}

// The next K-stage is loaded into registers while the current one runs on the
// MFMA units, and LDS is double-buffered, so one barrier separates the stages.
template <int kHerkBK>
__global__ __launch_bounds__(256, HerkF64Cfg<kHerkBK>::waves_per_simd) void k_herk_f64(HerkArgs h) {
    __shared__ double sAr[2][kHerkBK][kTile], sAi[2][kHerkBK][kTile], sBr[2][kHerkBK][kTile],
        sBi[2][kHerkBK][kTile];
    int I, J;
    tile_of(blockIdx.x, I, J);
    const int b = blockIdx.y;
    const double* Are = h.Are + (size_t)b * h.sA;
    const double* Aim = h.Aim + (size_t)b * h.sA;
    const double* w = h.w ? h.w + (size_t)b * h.sw : nullptr;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int ci = h.colA + I * kTile, cj = h.colA + J * kTile;
    // the accumulators start from C itself: its loads are in flight with those of the first stage, and
    // the epilogue only stores (with a short K, a load of C after the loop would be an exposed round trip)
    double* Cre = h.Cre + (size_t)b * h.sC + (size_t)(h.r0 + I * kTile + wr + (lane >> 4)) * h.ldC +
                  h.r0 + J * kTile + wc + (lane & 15);
    double* Cim = h.Cim + (Cre - h.Cre);
    v4d accR[2][2], accI[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const size_t o = (size_t)(x * 16 + 4 * r) * h.ldC + y * 16;
                accR[x][y][r] = Cre[o];
                accI[x][y][r] = Cim[o];
            }
    constexpr int kPer = kHerkBK * kTile / 256;
    // fetch only issues loads (rows past K are clamped to a valid one and masked in stash), so the loads
    // of the next stage stay in flight while the MFMAs of this one run
    double pr[kPer], pi[kPer], qr[kPer], qi[kPer], pw[kPer];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + 256 * i;
            const int kk = e >> 6, c = e & 63, k = min(k0 + kk, h.K - 1);
            const size_t row = (size_t)k * h.ldA;
            pw[i] = w ? w[k] : h.alpha;
            pr[i] = Are[row + ci + c];
            pi[i] = Aim[row + ci + c];
            qr[i] = Are[row + cj + c];
            qi[i] = Aim[row + cj + c];
        }
    };
    auto stash = [&](int buf, int k0) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int e = threadIdx.x + 256 * i;
            const int kk = e >> 6, c = e & 63;
            const bool ok = k0 + kk < h.K;
            sAr[buf][kk][c] = ok ? pr[i] * pw[i] : 0.0;
            sAi[buf][kk][c] = ok ? pi[i] * pw[i] : 0.0;
            sBr[buf][kk][c] = ok ? qr[i] : 0.0;
            sBi[buf][kk][c] = ok ? qi[i] : 0.0;
        }
    };
    fetch(0);
    stash(0, 0);
    int cur = 0;
    for (int k0 = 0; k0 < h.K; k0 += kHerkBK) {
        __syncthreads();
        const bool more = k0 + kHerkBK < h.K;
        if (more) fetch(k0 + kHerkBK);
#pragma unroll
        for (int kk = 0; kk < kHerkBK; kk += 4) {
            const int kr = kk + (lane >> 4), cc = lane & 15;
            double a_r[2], a_i[2], a_n[2], b_r[2], b_i[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a_r[x] = sAr[cur][kr][wr + x * 16 + cc];
                a_i[x] = sAi[cur][kr][wr + x * 16 + cc];
                a_n[x] = -a_r[x];
                b_r[x] = sBr[cur][kr][wc + x * 16 + cc];
                b_i[x] = sBi[cur][kr][wc + x * 16 + cc];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    accR[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r[x], b_r[y], accR[x][y], 0, 0, 0);
                    accR[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i[x], b_i[y], accR[x][y], 0, 0, 0);
                    accI[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i[x], b_r[y], accI[x][y], 0, 0, 0);
                    accI[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_n[x], b_i[y], accI[x][y], 0, 0, 0);
                }
        }
        if (more) stash(cur ^ 1, k0 + kHerkBK);
        cur ^= 1;
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const size_t o = (size_t)(x * 16 + 4 * r) * h.ldC + y * 16;
                Cre[o] = accR[x][y][r];
                Cim[o] = accI[x][y][r];
            }
}

// ------------------------------------------------------- E_c: 1 - K setup
__global__ void k_trace_k(const double* __restrict__ Cre, int ldC, long long sC, int NG,
                          const double* __restrict__ vsqrt, double* __restrict__ trk) {
    __shared__ double red[256];
    const int w = blockIdx.x;
    double s = 0;
    for (int i = threadIdx.x; i < NG; i += blockDim.x) s += vsqrt[i] * vsqrt[i] * Cre[(size_t)w * sC + (size_t)i * ldC + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) trk[w] = red[0];
}

__global__ void k_trace_full(const double* __restrict__ chi, int NG, const double* __restrict__ vsqrt,
                             double* __restrict__ trk) {
    __shared__ double red[256];
    const int w = blockIdx.x;
    double s = 0;
    for (int i = threadIdx.x; i < NG; i += blockDim.x)
        s += vsqrt[i] * vsqrt[i] * chi[2 * ((size_t)w * NG * NG + (size_t)i * NG + i)];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = blockDim.x / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) trk[w] = red[0];
}

// lower triangle (row i, cols j <= i) := -v_i v_j chi_ij, zero outside NG
__global__ void k_negk(double* __restrict__ Cre, double* __restrict__ Cim, int ldC, long long sC, int NG,
                       const double* __restrict__ vsqrt) {
    const int i = blockIdx.x, w = blockIdx.y;
    double* rr = Cre + (size_t)w * sC + (size_t)i * ldC;
    double* ri = Cim + (size_t)w * sC + (size_t)i * ldC;
    const double vi = i < NG ? vsqrt[i] : 0.0;
    // the padding is assigned, not scaled: whatever it held (NaN included) must not reach the factorisation
    for (int j = threadIdx.x; j <= i; j += blockDim.x) {
        const bool in = i < NG && j < NG;
        const double s = in ? -vi * vsqrt[j] : 0.0;
        rr[j] = in ? rr[j] * s : 0.0;
        ri[j] = in ? ri[j] * s : 0.0;
    }
}

__global__ void k_negk_full(const double* __restrict__ chi, int NG, double* __restrict__ Cre,
                            double* __restrict__ Cim, int ldC, long long sC, const double* __restrict__ vsqrt) {
    const int i = blockIdx.x, w = blockIdx.y;
    double* rr = Cre + (size_t)w * sC + (size_t)i * ldC;
    double* ri = Cim + (size_t)w * sC + (size_t)i * ldC;
    for (int j = threadIdx.x; j <= i; j += blockDim.x) {
        double re = 0, im = 0;
        if (i < NG && j < NG) {
            const double s = -vsqrt[i] * vsqrt[j];
            const size_t o = 2 * ((size_t)w * NG * NG + (size_t)i * NG + j);
            re = chi[o] * s;
            im = chi[o + 1] * s;
        }
        rr[j] = re;
        ri[j] = im;
    }
}

__global__ void k_weighted_sum(const double* __restrict__ x, const double* __restrict__ w, int n,
                               double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += w[j] * x[j];
    *out = s;
}

__device__ __forceinline__ float hash_unit(unsigned long long i) {
    unsigned long long z = i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (float)((z >> 40) * (1.0 / 16777216.0)) * 2.0f - 1.0f;
}

__global__ void k_fill_pattern(float* __restrict__ f, size_t nf, double* __restrict__ d, size_t nd) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += (size_t)gridDim.x * blockDim.x)
        f[i] = hash_unit(i);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += (size_t)gridDim.x * blockDim.x)
        d[i] = -1e-3 * (1.5 + hash_unit(i + nf));
}

__global__ void k_zero_d(double* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}
__global__ void k_zero_i(int* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// ------------------------------------------------------ blocked Cholesky
// The factorised matrix is 1 + A with A = -K held in C; the identity is never
// formed: pivot j is 1 + A_jj and contributes log1p(A_jj) to ln det(1 - K),
// which keeps ln det accurate when K is small (large frequencies).
//
// Panel: factor the 64x64 diagonal block at j0 in LDS, accumulate its log-det,
// and store the inverse of its lower-triangular factor for the row solve.
//
// Both the factorisation and the inversion are right-looking and keep their
// columns unscaled (the pivot of column c is s_c = sqrt(1 + A_cc), so
// L_rc L_jc^* = A_rc A_jc^* / (1 + A_cc)); the scaling is applied once when the
// results are written. Lane j owns column j and wave v of eight walks the rows
// r = v (mod 8): A[r][c] is a broadcast read and A[r][j] a contiguous one. Each
// column costs one barrier: the reciprocal of the next pivot is formed during
// the step by the lane that updates it, the rows of a wave are counted
// wave-uniformly, and lanes whose entry of a row is not updated write it to a
// slot of their own instead of branching.
constexpr int kPanelLd = kTile + 1;
constexpr int kPanelWaves = 8;
__global__ __launch_bounds__(64 * kPanelWaves) void k_chol_panel(double* __restrict__ Cre, double* __restrict__ Cim,
                                                                 int ldC, long long sC, int j0,
                                                                 double* __restrict__ Lre, double* __restrict__ Lim,
                                                                 double* __restrict__ logdet, int* __restrict__ fail) {
    constexpr int NW = kPanelWaves;
    // A (lower triangle, diagonal included) and the strict lower triangle of W share one array:
    // W[r][j] (j < r) sits at t[j][r + 1], in the upper part that A leaves free. W's diagonal is 1.
    __shared__ double2 t[kTile][kPanelLd];
    __shared__ double2 sink[kTile];
    __shared__ double pinv[kTile], piv[kTile], lgp[kTile];
    const int w = blockIdx.x, tid = threadIdx.x;
    const int j = tid & (kTile - 1), wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    double* cr = Cre + (size_t)w * sC;
    double* ci = Cim + (size_t)w * sC;
    for (int e = tid; e < kTile * kPanelLd; e += blockDim.x) {
        const int r = e / kPanelLd, c = e - r * kPanelLd;
        t[r][c] = c <= r ? make_double2(cr[(size_t)(j0 + r) * ldC + j0 + c], ci[(size_t)(j0 + r) * ldC + j0 + c])
                         : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (tid == 0) pinv[0] = 1.0 / (1.0 + t[0][0].x);
    __syncthreads();
    // Factor and inverse advance together, one barrier per column c. Column c of A is final once step
    // c - 1 is done, and step c reads nothing else of A, so the two updates of step c touch disjoint
    // entries and can share the interval:
    //   factor  (lanes j > c):  A[r][j] -= A[r][c] conj(A[j][c]) / (1 + A[c][c]),  j <= r;
    //   inverse (lanes j <= c): W[r][j] -= A[r][c] W[c][j] / (1 + A[c][c]),        c < r,
    // with W = I at the start and V = W / s_r at the end. Both read x[r] -= A[r][c] g_j. The pivots' square
    // roots and logarithms wait until the end.
    for (int c = 0; c < kTile - 1; ++c) {
        const double inv = pinv[c];
        const bool fac = j > c;
        // g_j: conj(A[j][c]) for the factor; W[c][j] (1 on the diagonal) for the inverse
        const double2 g = fac ? t[j][c] : (j == c ? make_double2(1.0, 0.0) : t[j][c + 1]);
        const double br = g.x * inv, bi = (fac ? -g.y : g.y) * inv;
        const int rlo = fac ? j : 0;
        // this wave's rows above c: the first, r0, and their number (both wave-uniform)
        const int r0 = c + 1 + ((wv - c - 1) & (NW - 1));
        const int ns = (kTile - r0 + NW - 1) / NW;
        // lane j walks A's column j (t[r][j]) or W's column j (t[j][r + 1])
        const int xs = fac ? kPanelLd : 1;
        const int rb = min(r0, kTile - 1);
        double2* xq = fac ? &t[rb][j] : &t[j][rb + 1];
        const double2* aq = &t[rb][c];
        // all loads of the step first, so their latencies overlap
        double2 arc[kTile / NW], x[kTile / NW];
#pragma unroll
        for (int i = 0; i < kTile / NW; ++i) {
            if (i < ns) {
                arc[i] = aq[i * NW * kPanelLd];
                x[i] = xq[i * NW * xs];
            }
        }
#pragma unroll
        for (int i = 0; i < kTile / NW; ++i) {
            if (i < ns) {
                x[i].x -= arc[i].x * br - arc[i].y * bi;
                x[i].y -= arc[i].x * bi + arc[i].y * br;
                double2* d = r0 + NW * i >= rlo ? &xq[i * NW * xs] : &sink[j];
                *d = x[i];
                // the wave that owns row c + 1: its lane c + 1 now holds the final A[c+1][c+1]
                if (i == 0 && r0 == c + 1 && j == c + 1) pinv[c + 1] = 1.0 / (1.0 + x[0].x);
            }
        }
        __syncthreads();
    }
    if (tid < kTile) {
        const double d = t[tid][tid].x;
        piv[tid] = sqrt(1.0 + d);
        lgp[tid] = (1.0 + d > 0.0) ? log1p(d) : __builtin_nan("");
    }
    __syncthreads();
    double* lr = Lre + (size_t)w * kTile * kTile;
    double* li = Lim + (size_t)w * kTile * kTile;
    for (int e = tid; e < kTile * kTile; e += blockDim.x) {
        const int r = e >> 6, c = e & 63;
        if (c <= r) {
            const double sr = 1.0 / piv[r];
            const double2 wv2 = c == r ? make_double2(1.0, 0.0) : t[c][r + 1];
            lr[e] = wv2.x * sr;
            li[e] = wv2.y * sr;
            // the factor itself replaces the lower triangle of the block
            double xr, xi;
            if (c == r) {
                xr = piv[c];
                xi = 0.0;
            } else {
                const double sc = 1.0 / piv[c];
                xr = t[r][c].x * sc;
                xi = t[r][c].y * sc;
            }
            cr[(size_t)(j0 + r) * ldC + j0 + c] = xr;
            ci[(size_t)(j0 + r) * ldC + j0 + c] = xi;
        } else {
            lr[e] = 0.0;
            li[e] = 0.0;
        }
    }
    if (tid == 0) {
        // pivots in column order; the first one that is not positive marks the failure
        double ldacc = 0.0;
        int bad = 0;
        for (int c = 0; c < kTile; ++c) {
            if (!(1.0 + t[c][c].x > 0.0) && !bad) bad = j0 + c + 1;
            ldacc += lgp[c];
        }
        logdet[w] += ldacc;
        if (bad && !fail[w]) fail[w] = bad;
    }
}

// Row solve of the panel below the diagonal block: X = A21 (L11^-1)^H, written
// transposed (X[c][r], rows contiguous) as the operand of the trailing update.
constexpr int kTrsmRows = 32;
__global__ __launch_bounds__(256) void k_chol_trsm(double* __restrict__ Cre, double* __restrict__ Cim,
                                                   int ldC, long long sC, int j0, int NGp,
                                                   const double* __restrict__ Lre, const double* __restrict__ Lim,
                                                   double* __restrict__ Pre, double* __restrict__ Pim, long long sP) {
    __shared__ double lr[kTile][kTile + 1], li[kTile][kTile + 1];
    __shared__ double ar[kTrsmRows][kTile + 1], ai[kTrsmRows][kTile + 1];
    const int w = blockIdx.y, tid = threadIdx.x;
    const int r0 = j0 + kTile + blockIdx.x * kTrsmRows;
    double* cr = Cre + (size_t)w * sC;
    double* ci = Cim + (size_t)w * sC;
    for (int e = tid; e < kTile * kTile; e += blockDim.x) {
        lr[e >> 6][e & 63] = Lre[(size_t)w * kTile * kTile + e];
        li[e >> 6][e & 63] = Lim[(size_t)w * kTile * kTile + e];
    }
    for (int e = tid; e < kTrsmRows * kTile; e += blockDim.x) {
        const int r = e >> 6, c = e & 63;
        const int row = r0 + r;
        ar[r][c] = row < NGp ? cr[(size_t)row * ldC + j0 + c] : 0.0;
        ai[r][c] = row < NGp ? ci[(size_t)row * ldC + j0 + c] : 0.0;
    }
    __syncthreads();
    double* pr = Pre + (size_t)w * sP;
    double* pi = Pim + (size_t)w * sP;
    for (int e = tid; e < kTrsmRows * kTile; e += blockDim.x) {
        const int r = e % kTrsmRows, c = e / kTrsmRows;
        const int row = r0 + r;
        // X[r][c] = sum_{k<=c} A[r][k] conj(Linv[c][k])
        double xr = 0, xi = 0;
        for (int k = 0; k <= c; ++k) {
            xr += ar[r][k] * lr[c][k] + ai[r][k] * li[c][k];
            xi += ai[r][k] * lr[c][k] - ar[r][k] * li[c][k];
        }
        if (row < NGp) {
            pr[(size_t)c * NGp + row] = xr;
            pi[(size_t)c * NGp + row] = xi;
            // the factor's block column replaces the matrix below the diagonal block
            cr[(size_t)row * ldC + j0 + c] = xr;
            ci[(size_t)row * ldC + j0 + c] = xi;
        }
    }
}

__global__ void k_finalize(const double* __restrict__ logdet, const double* __restrict__ trk,
                           const int* __restrict__ fail, const double* __restrict__ wgt, int nw, double* __restrict__ F,
                           double* __restrict__ ec) {
    if (threadIdx.x != 0) return;
    double e = 0.0;
    for (int w = 0; w < nw; ++w) {
        const double f = fail[w] ? __builtin_nan("") : logdet[w] + trk[w];
        if (F) F[w] = f;
        e += wgt[w] * f;
    }
    *ec = e / (2.0 * kPi);
}

template <typename T>
__global__ void k_rho_out(const T* __restrict__ rre, const T* __restrict__ rim, int NG, int NGp,
                          double* __restrict__ out) {
    const size_t p = blockIdx.y;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < NG; g += gridDim.x * blockDim.x) {
        out[2 * (p * NG + g)] = (double)rre[p * NGp + g];
        out[2 * (p * NG + g) + 1] = (double)rim[p * NGp + g];
    }
}

__global__ void k_chi_out(const double* __restrict__ Cre, const double* __restrict__ Cim, int ldC, long long sC,
                          int NG, int add, double* __restrict__ out) {
    const int i = blockIdx.x, w = blockIdx.y;
    const double* cr = Cre + (size_t)w * sC;
    const double* ci = Cim + (size_t)w * sC;
    double* o = out + 2 * ((size_t)w * NG * NG + (size_t)i * NG);
    for (int j = threadIdx.x; j < NG; j += blockDim.x) {
        double re, im;
        if (j <= i) { re = cr[(size_t)i * ldC + j]; im = ci[(size_t)i * ldC + j]; }
        else { re = cr[(size_t)j * ldC + i]; im = -ci[(size_t)j * ldC + i]; }
        if (add) {
            re += o[2 * j];
            im += o[2 * j + 1];
        }
        o[2 * j] = re;
        o[2 * j + 1] = im;
    }
}

}  // namespace

template <typename T>
hipError_t launch_paw_y(const double* Pk, int ldP, const int32_t* nlist, int nn, const int32_t* proj_off,
                        const int32_t* qoff, int natoms, int nprojtot, const double* Q, int NG, int NGp, T* Yre,
                        T* Yim, hipStream_t s) {
    if (!nn || !nprojtot) return hipSuccess;
    dim3 grid((unsigned)((NGp + 255) / 256), (unsigned)nprojtot, (unsigned)nn);
    hipLaunchKernelGGL(k_paw_y<T>, grid, dim3(256), 0, s, Pk, ldP, nlist, proj_off, qoff, natoms, nprojtot, Q, NG, NGp,
                       Yre, Yim);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_paw_add(const T* Yre, const T* Yim, const int32_t* pn, int nlo, const int32_t* pm, const double* Pkq,
                          int ldP, int nprojtot, int npairs, int NG, int NGp, T* rre, T* rim, hipStream_t s) {
    if (!npairs || !nprojtot) return hipSuccess;
    dim3 grid((unsigned)((NG + 255) / 256), (unsigned)((npairs + kPawPairs - 1) / kPawPairs));
    const size_t lds = 2 * (size_t)kPawPairs * nprojtot * sizeof(T);
    hipLaunchKernelGGL(k_paw_add<T>, grid, dim3(256), lds, s, Yre, Yim, pn, nlo, pm, Pkq, ldP, nprojtot, npairs, NG,
                       NGp, rre, rim);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_optical_row(const double* Ck, const double* Ckq, int nQ, const double* wq, const double* Pk,
                              const double* Pkq, int ldP, const double* Dq, const int32_t* proj_off,
                              const int32_t* qoff, int natoms, const double* epsk, const double* epskq,
                              const int32_t* pn, const int32_t* pm, int npairs, int g0, int NGp, T* rre, T* rim,
                              hipStream_t s) {
    if (!npairs) return hipSuccess;
    hipLaunchKernelGGL(k_optical_row<T>, dim3((unsigned)npairs), dim3(256), 0, s, Ck, Ckq, nQ, wq, Pk, Pkq, ldP, Dq,
                       proj_off, qoff, natoms, epsk, epskq, pn, pm, g0, NGp, rre, rim);
    return hipGetLastError();
}

hipError_t launch_band_drude(const double* C, int nQ, const double* wq, const double* P, int ldP, const double* Dq,
                             const int32_t* proj_off, const int32_t* qoff, int natoms, const int32_t* band,
                             const double* mdf, int nbands, double weight, double* term, hipStream_t s) {
    if (!nbands) return hipSuccess;
    hipLaunchKernelGGL(k_band_drude, dim3((unsigned)nbands), dim3(256), 0, s, C, nQ, wq, P, ldP, Dq, proj_off, qoff,
                       natoms, band, mdf, weight, term);
    return hipGetLastError();
}

hipError_t launch_add_drude(const double* term, int nterms, const double* omega, int nw, double inv_volume,
                            double* head, long long stride, hipStream_t s) {
    if (nw > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_add_drude, dim3(1), dim3(256), 0, s, term, nterms, omega, nw, inv_volume, head, stride);
    return hipGetLastError();
}

hipError_t launch_weights(const double* epsk, const double* epskq, const double* fk, const double* fkq,
                          const int32_t* pn, const int32_t* pm, int npairs, const double* omega, int nw, double prefac,
                          double* a, int lda, hipStream_t s) {
    if (!lda) return hipSuccess;
    hipLaunchKernelGGL(k_weights, dim3((unsigned)((lda + 255) / 256)), dim3(256), 0, s, epsk, epskq, fk, fkq, pn, pm,
                       npairs, omega, nw, prefac, a, lda);
    return hipGetLastError();
}

hipError_t launch_weights_real(const double* epsk, const double* epskq, const double* fk, const double* fkq,
                               const int32_t* pn, const int32_t* pm, int npairs, const double* omega, int nw,
                               double eta, double prefac, double* a, int lda, hipStream_t s) {
    if (!lda) return hipSuccess;
    hipLaunchKernelGGL(k_weights_real, dim3((unsigned)((lda + 255) / 256)), dim3(256), 0, s, epsk, epskq, fk, fkq, pn,
                       pm, npairs, omega, nw, eta, prefac, a, lda);
    return hipGetLastError();
}

hipError_t launch_add_drude_real(const double* term, int nterms, const double* omega, int nw, double eta,
                                 double inv_volume, double* head, long long stride, hipStream_t s) {
    if (nw > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_add_drude_real, dim3(1), dim3(256), 0, s, term, nterms, omega, nw, eta, inv_volume, head,
                       stride);
    return hipGetLastError();
}

hipError_t launch_chi_out_real(const double* Cre, const double* Cim, int ldC, int NG, int nw, double* out,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_chi_out_real, dim3((unsigned)NG, (unsigned)nw), dim3(256), 0, s, Cre, Cim, ldC,
                       (long long)ldC * ldC, NG, nw, out);
    return hipGetLastError();
}

hipError_t launch_herk_f64(const HerkArgs& h, hipStream_t s) {
    if (h.nT <= 0 || h.nbatch <= 0 || h.K <= 0) return hipSuccess;
    const unsigned ntiles = (unsigned)(h.nT * (h.nT + 1) / 2);
    if (h.K > kTile)
        hipLaunchKernelGGL(k_herk_f64<8>, dim3(ntiles, (unsigned)h.nbatch), dim3(256), 0, s, h);
    else
        hipLaunchKernelGGL(k_herk_f64<16>, dim3(ntiles, (unsigned)h.nbatch), dim3(256), 0, s, h);
    return hipGetLastError();
}

hipError_t launch_build_negk(double* Cre, double* Cim, int ldC, int NG, int NGp, int nw, const double* vsqrt,
                             double* trk, hipStream_t s) {
    const long long sC = (long long)ldC * ldC;
    hipLaunchKernelGGL(k_trace_k, dim3((unsigned)nw), dim3(256), 0, s, Cre, ldC, sC, NG, vsqrt, trk);
    hipLaunchKernelGGL(k_negk, dim3((unsigned)NGp, (unsigned)nw), dim3(256), 0, s, Cre, Cim, ldC, sC, NG, vsqrt);
    return hipGetLastError();
}

hipError_t launch_build_negk_from_full(const double* chi, int NG, double* Cre, double* Cim, int NGp, int nw,
                                       const double* vsqrt, double* trk, hipStream_t s) {
    const long long sC = (long long)NGp * NGp;
    hipLaunchKernelGGL(k_trace_full, dim3((unsigned)nw), dim3(256), 0, s, chi, NG, vsqrt, trk);
    hipLaunchKernelGGL(k_negk_full, dim3((unsigned)NGp, (unsigned)nw), dim3(256), 0, s, chi, NG, Cre, Cim, NGp, sC,
                       vsqrt);
    return hipGetLastError();
}

hipError_t launch_chol_panel(double* Cre, double* Cim, int ldC, int j0, int nw, double* Lre, double* Lim,
                             double* logdet, int* fail, hipStream_t s) {
    hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)nw), dim3(64 * kPanelWaves), 0, s, Cre, Cim, ldC,
                       (long long)ldC * ldC, j0, Lre, Lim, logdet, fail);
    return hipGetLastError();
}

hipError_t launch_chol_trsm(double* Cre, double* Cim, int ldC, int j0, int NGp, int nw, const double* Lre,
                            const double* Lim, double* Pre, double* Pim, long long sP, hipStream_t s) {
    const int rows = NGp - j0 - kTile;
    if (rows <= 0) return hipSuccess;
    dim3 grid((unsigned)((rows + kTrsmRows - 1) / kTrsmRows), (unsigned)nw);
    hipLaunchKernelGGL(k_chol_trsm, grid, dim3(256), 0, s, Cre, Cim, ldC, (long long)ldC * ldC, j0, NGp, Lre, Lim, Pre,
                       Pim, sP);
    return hipGetLastError();
}

hipError_t launch_finalize(const double* logdet, const double* trk, const int* fail, const double* wgt, int nw,
                           double* F, double* ec, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, logdet, trk, fail, wgt, nw, F, ec);
    return hipGetLastError();
}

hipError_t launch_zero(double* d, int nd, int* iv, int ni, hipStream_t s) {
    if (nd) hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(256), 0, s, d, nd);
    if (ni) hipLaunchKernelGGL(k_zero_i, dim3(1), dim3(256), 0, s, iv, ni);
    return hipGetLastError();
}

hipError_t launch_weighted_sum(const double* x, const double* w, int n, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_weighted_sum, dim3(1), dim3(64), 0, s, x, w, n, out);
    return hipGetLastError();
}

hipError_t launch_fill_pattern(float* f, size_t nf, double* d, size_t nd, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_pattern, dim3(1024), dim3(256), 0, s, f, nf, d, nd);
    return hipGetLastError();
}

hipError_t launch_chi_out(const double* Cre, const double* Cim, int ldC, int NG, int nw, int add, double* out,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_chi_out, dim3((unsigned)NG, (unsigned)nw), dim3(256), 0, s, Cre, Cim, ldC,
                       (long long)ldC * ldC, NG, add, out);
    return hipGetLastError();
}

// Coefficients of a state set unfolded with time reversal (Eq. trans_wfs): the complex conjugate, element by
// element (the plane-wave labels are transformed on the host).
__global__ __launch_bounds__(256) void k_conj_copy(const double* __restrict__ in, size_t n, double* __restrict__ out) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double2 v = reinterpret_cast<const double2*>(in)[i];
        reinterpret_cast<double2*>(out)[i] = make_double2(v.x, -v.y);
    }
}

// Projections at k from those at k1 (Table 1 step 7): output column c = (atom a, projector i) reads the
// block of atom b(a), P_k[n][c] = ph_c sum_j D[row_c + j] P_k1[n][src_c + j], conjugated with time
// reversal; tab[3c .. 3c+2] = (src_c, Np, row_c), ph = (cos, sin) of k1.L_a per column.
__global__ __launch_bounds__(256) void k_rotate_proj(const double* __restrict__ Pin, int nb, int nproj,
                                                     const int32_t* __restrict__ tab, const double* __restrict__ D,
                                                     const double* __restrict__ ph, int tr,
                                                     double* __restrict__ Pout) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)nb * nproj) return;
    const int n = (int)(idx / nproj), c = (int)(idx % nproj);
    const int src = tab[3 * c], np = tab[3 * c + 1], row = tab[3 * c + 2];
    const double* p = Pin + 2 * ((size_t)n * nproj + src);
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < np; ++j) {
        const double d = D[row + j];
        sr += d * p[2 * j];
        si += d * p[2 * j + 1];
    }
    const double cr = ph[2 * c], ci = ph[2 * c + 1];
    const double outr = cr * sr - ci * si, outi = cr * si + ci * sr;
    Pout[2 * idx] = outr;
    Pout[2 * idx + 1] = tr ? -outi : outi;
}

hipError_t launch_conj_copy(const double* in, size_t n, double* out, hipStream_t s) {
    if (!n) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_conj_copy, dim3((unsigned)blocks), dim3(256), 0, s, in, n, out);
    return hipGetLastError();
}

hipError_t launch_rotate_proj(const double* Pin, int nb, int nproj, const int32_t* tab, const double* D,
                              const double* ph, int tr, double* Pout, hipStream_t s) {
    const size_t n = (size_t)nb * nproj;
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_rotate_proj, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Pin, nb, nproj, tab, D, ph,
                       tr, Pout);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_rho_out(const T* rre, const T* rim, int npairs, int NG, int NGp, double* out, hipStream_t s) {
    if (!npairs) return hipSuccess;
    hipLaunchKernelGGL(k_rho_out<T>, dim3((unsigned)((NG + 255) / 256), (unsigned)npairs), dim3(256), 0, s, rre, rim,
                       NG, NGp, out);
    return hipGetLastError();
}

#define RPA_INST(T)                                                                                                  \
    template hipError_t launch_rho_out<T>(const T*, const T*, int, int, int, double*, hipStream_t);                  \
    template hipError_t launch_paw_y<T>(const double*, int, const int32_t*, int, const int32_t*, const int32_t*, int, \
                                        int, const double*, int, int, T*, T*, hipStream_t);                          \
    template hipError_t launch_paw_add<T>(const T*, const T*, const int32_t*, int, const int32_t*, const double*,    \
                                          int, int, int, int, int, T*, T*, hipStream_t);                              \
    template hipError_t launch_optical_row<T>(const double*, const double*, int, const double*, const double*,       \
                                              const double*, int, const double*, const int32_t*, const int32_t*,     \
                                              int, const double*, const double*, const int32_t*, const int32_t*,     \
                                              int, int, int, T*, T*, hipStream_t);
RPA_INST(double)
RPA_INST(float)
#undef RPA_INST

}  // namespace rpa
