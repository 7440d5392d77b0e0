// Adjoint of E_c(q) with respect to eigenvalues, plane-wave coefficients and
// PAW projections (the paper has no adjoint; this differentiates Eq. rpa with
// Eq. chi0, Eq. n_G_2, Eq. fft, Eq. get_wfs and Eq. n_q0).
//
// With K = V chi0 V (V = diag v^1/2) and F = ln det(1 - K) + Tr K,
//   dF = Tr[W dchi0],  W(w) = V [1 - (1 - K)^-1] V,
// so for chi0 = sum_p a_p rho_p rho_p^H:
//   dE/da_p(w) = c_w rho_p^H W rho_p,   rho_bar_p = sum_w c_w 2 a_p(w) W rho_p,
// c_w = dE_up W_w / 2 pi. rho_bar then flows back through the optical row,
// the PAW term and the pruned FFT of conj(phi_n) phi_m (whose adjoint is the
// inverse transform followed by a product with the other orbital) to the
// coefficients. Complex gradients follow dE = Re sum conj(grad) d(value).
#include "internal.hpp"

namespace rpa {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ cplx<double> ldc(const double* p, size_t i) { return mk(p[2 * i], p[2 * i + 1]); }

// ------------------------------------------------------------------ GEMM
// C[b] = beta C[b] + alpha op(A[b]) op(B[b]), planar FP64, 64x64 tiles of
// v_mfma_f64_16x16x4f64 (D lane l element r holds row l/16 + 4r, column l%16).
// K-stage of the complex GEMM: 8 (34 KB of LDS, double-buffered) with registers bounded for three
// workgroups per CU, which hides more latency than stages of 16 at two per CU (11-15 % faster on the
// panel-solve, look-ahead and adjoint shapes)
constexpr int kGB = 8;

// The next K-stage is loaded into registers while the current one runs on the MFMA units (the loads carry
// no arithmetic, so they stay in flight), LDS is double-buffered, and with beta the whole C block of a
// row of sub-tiles is read before any of it is written.
__global__ __launch_bounds__(256, 3) void k_gemm_c64(GemmArgs g) {
    // rows padded by two doubles: operands contiguous along k are staged down a column, 16 rows apart,
    // and the padding spreads those 16 writes over distinct banks
    constexpr int kLd = kTile + 2;
    __shared__ double sAr[2][kGB][kLd], sAi[2][kGB][kLd], sBr[2][kGB][kLd], sBi[2][kGB][kLd];
    const int I = blockIdx.x, J = blockIdx.y, b = blockIdx.z;
    if (g.lower && J > I) return;  // the whole tile lies above the diagonal
    // with triangular factors every k below the tile's first row or column contributes zero
    const int kbeg = g.ktri ? max(I, J) * kTile : 0;
    const double* Ar = g.Ar + (size_t)b * g.sA;
    const double* Ai = g.Ai + (size_t)b * g.sA;
    const double* Br = g.Br + (size_t)b * g.sB;
    const double* Bi = g.Bi + (size_t)b * g.sB;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const double sa = g.conjA ? -1.0 : 1.0, sb = g.conjB ? -1.0 : 1.0;
    v4d accR[2][2], accI[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) {
            accR[x][y] = v4d{0, 0, 0, 0};
            accI[x][y] = v4d{0, 0, 0, 0};
        }
    // element e of a stage: the index order follows the contiguous direction of each operand
    auto a_at = [&](int e, int& kk, int& c) {
        if (g.aI == 1) { kk = e >> 6; c = e & 63; } else { c = e / kGB; kk = e % kGB; }
    };
    auto b_at = [&](int e, int& kk, int& c) {
        if (g.bJ == 1) { kk = e >> 6; c = e & 63; } else { c = e / kGB; kk = e % kGB; }
    };
    constexpr int kPer = kGB * kTile / 256;
    double pr[kPer], pi[kPer], qr[kPer], qi[kPer];
    // indices past M, N or K are clamped to valid elements here and masked in stash
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            int kk, c;
            a_at(e, kk, c);
            size_t o = (size_t)min(I * kTile + c, g.M - 1) * g.aI + (size_t)min(k0 + kk, g.K - 1) * g.aK;
            pr[u] = Ar[o];
            pi[u] = Ai[o];
            b_at(e, kk, c);
            o = (size_t)min(k0 + kk, g.K - 1) * g.bK + (size_t)min(J * kTile + c, g.N - 1) * g.bJ;
            qr[u] = Br[o];
            qi[u] = Bi[o];
        }
    };
    auto stash = [&](int buf, int k0) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = tid + 256 * u;
            int kk, c;
            a_at(e, kk, c);
            bool ok = I * kTile + c < g.M && k0 + kk < g.K;
            sAr[buf][kk][c] = ok ? pr[u] : 0.0;
            sAi[buf][kk][c] = ok ? sa * pi[u] : 0.0;
            b_at(e, kk, c);
            ok = J * kTile + c < g.N && k0 + kk < g.K;
            sBr[buf][kk][c] = ok ? qr[u] : 0.0;
            sBi[buf][kk][c] = ok ? sb * qi[u] : 0.0;
        }
    };
    if (kbeg < g.K) {
        fetch(kbeg);
        stash(0, kbeg);
    }
    int cur = 0;
    for (int k0 = kbeg; k0 < g.K; k0 += kGB) {
        __syncthreads();
        const bool more = k0 + kGB < g.K;
        if (more) fetch(k0 + kGB);
#pragma unroll
        for (int kk = 0; kk < kGB; kk += 4) {
            const int kr = kk + (lane >> 4), cc = lane & 15;
            double a_r[2], a_i[2], a_n[2], b_r[2], b_i[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a_r[x] = sAr[cur][kr][wr + x * 16 + cc];
                a_i[x] = sAi[cur][kr][wr + x * 16 + cc];
                a_n[x] = -a_i[x];
                b_r[x] = sBr[cur][kr][wc + x * 16 + cc];
                b_i[x] = sBi[cur][kr][wc + x * 16 + cc];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    // (ar + i ai)(br + i bi) = ar br - ai bi + i (ar bi + ai br)
                    accR[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r[x], b_r[y], accR[x][y], 0, 0, 0);
                    accR[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_n[x], b_i[y], accR[x][y], 0, 0, 0);
                    accI[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r[x], b_i[y], accI[x][y], 0, 0, 0);
                    accI[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i[x], b_r[y], accI[x][y], 0, 0, 0);
                }
        }
        if (more) stash(cur ^ 1, k0 + kGB);
        cur ^= 1;
    }
    double* Cr = g.Cr + (size_t)b * g.sC;
    double* Ci = g.Ci + (size_t)b * g.sC;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        double cr[2][4], ci[2][4];
        if (g.beta) {
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = I * kTile + wr + x * 16 + (lane >> 4) + 4 * r;
                    const int j = J * kTile + wc + y * 16 + (lane & 15);
                    const size_t o = (i < g.M && j < g.N) ? (size_t)i * g.ldC + j : 0;
                    cr[y][r] = Cr[o];
                    ci[y][r] = Ci[o];
                }
        }
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I * kTile + wr + x * 16 + (lane >> 4) + 4 * r;
                const int j = J * kTile + wc + y * 16 + (lane & 15);
                if (i < g.M && j < g.N) {
                    const size_t o = (size_t)i * g.ldC + j;
                    const double vr = g.alpha * accR[x][y][r], vi = g.alpha * accI[x][y][r];
                    if (g.beta) {
                        Cr[o] = cr[y][r] + vr;
                        Ci[o] = ci[y][r] + vi;
                    } else {
                        Cr[o] = vr;
                        Ci[o] = vi;
                    }
                }
            }
    }
}

// Short-K form (K <= 64) for the latency-bound GEMMs of the Cholesky chain (the panel solve and the
// look-ahead column): 32x32 tiles, each wave one 16x16 block, and every operand value of the whole K
// loaded from memory straight into the MFMA operand registers at once (no LDS, no barrier), so that
// a workgroup waits for memory once instead of once per K-stage.
constexpr int kShortK = 64;
__global__ __launch_bounds__(256) void k_gemm_c64_k64(GemmArgs g) {
    if (g.lower && blockIdx.y > blockIdx.x) return;   // the tile lies wholly above the diagonal
    const int b = blockIdx.z, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i0 = blockIdx.x * 32 + (wave >> 1) * 16, j0 = blockIdx.y * 32 + (wave & 1) * 16;
    const double* Ar = g.Ar + (size_t)b * g.sA;
    const double* Ai = g.Ai + (size_t)b * g.sA;
    const double* Br = g.Br + (size_t)b * g.sB;
    const double* Bi = g.Bi + (size_t)b * g.sB;
    double* Cr = g.Cr + (size_t)b * g.sC;
    double* Ci = g.Ci + (size_t)b * g.sC;
    const double sa = g.conjA ? -1.0 : 1.0, sb = g.conjB ? -1.0 : 1.0;
    // operand layouts of v_mfma_f64_16x16x4f64: A lane l holds A[l%16][l/16], B lane l holds B[l/16][l%16];
    // indices past M, N or K are clamped to valid elements and their values masked below
    const int cc = lane & 15, kq = lane >> 4;
    const size_t ia = (size_t)min(i0 + cc, g.M - 1) * g.aI, jb = (size_t)min(j0 + cc, g.N - 1) * g.bJ;
    double ar[kShortK / 4], ai[kShortK / 4], br[kShortK / 4], bi[kShortK / 4];
#pragma unroll
    for (int s = 0; s < kShortK / 4; ++s) {
        const size_t k = (size_t)min(4 * s + kq, g.K - 1);
        ar[s] = Ar[ia + k * g.aK];
        ai[s] = Ai[ia + k * g.aK];
        br[s] = Br[k * g.bK + jb];
        bi[s] = Bi[k * g.bK + jb];
    }
    // D lane l element r holds row l/16 + 4r, column l%16; with beta C is read along with the operands
    const int jc = j0 + cc;
    double cr[4] = {0, 0, 0, 0}, ci[4] = {0, 0, 0, 0};
    if (g.beta) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = i0 + kq + 4 * r;
            const size_t o = (i < g.M && jc < g.N) ? (size_t)i * g.ldC + jc : 0;
            cr[r] = Cr[o];
            ci[r] = Ci[o];
        }
    }
    v4d accR = {0, 0, 0, 0}, accI = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < kShortK / 4; ++s) {
        if (4 * s >= g.K) break;
        const bool ok = 4 * s + kq < g.K;
        const double a_r = ok ? ar[s] : 0.0, a_i = ok ? sa * ai[s] : 0.0;
        const double b_r = ok ? br[s] : 0.0, b_i = ok ? sb * bi[s] : 0.0;
        // (ar + i ai)(br + i bi) = ar br - ai bi + i (ar bi + ai br)
        accR = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r, b_r, accR, 0, 0, 0);
        accR = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_i, b_i, accR, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f64_16x16x4f64(a_r, b_i, accI, 0, 0, 0);
        accI = __builtin_amdgcn_mfma_f64_16x16x4f64(a_i, b_r, accI, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + kq + 4 * r;
        if (i < g.M && jc < g.N) {
            const size_t o = (size_t)i * g.ldC + jc;
            Cr[o] = cr[r] + g.alpha * accR[r];
            Ci[o] = ci[r] + g.alpha * accI[r];
        }
    }
}

// identity in rows [0, n) of a [nb][ld][ld] planar batch (zero elsewhere)
__global__ void k_identity(double* __restrict__ Xr, double* __restrict__ Xi, int n, int ld) {
    const int i = blockIdx.x, b = blockIdx.y;
    double* xr = Xr + ((size_t)b * ld + i) * ld;
    double* xi = Xi + ((size_t)b * ld + i) * ld;
    for (int j = threadIdx.x; j < ld; j += blockDim.x) {
        xr[j] = (i == j && i < n) ? 1.0 : 0.0;
        xi[j] = 0.0;
    }
}

// W = V (1 - Minv) V in place, zero outside NG, from the lower triangle of the Hermitian Minv: row block i
// reads its entries j <= i and writes them and their mirrors (j, i) (the upper part of row j, which row
// block j does not read); c_w = dE_up W_w / 2 pi
__global__ void k_build_w(double* __restrict__ Mr, double* __restrict__ Mi, int NG, int NGp,
                          const double* __restrict__ vs) {
    const int i = blockIdx.x, b = blockIdx.y;
    double* mr = Mr + (size_t)b * NGp * NGp;
    double* mi = Mi + (size_t)b * NGp * NGp;
    for (int j = threadIdx.x; j <= i; j += blockDim.x) {
        double r = 0, im = 0;
        if (i < NG && j < NG) {
            const double s = vs[i] * vs[j];
            r = s * ((i == j ? 1.0 : 0.0) - mr[(size_t)i * NGp + j]);
            im = -s * mi[(size_t)i * NGp + j];
        }
        mr[(size_t)i * NGp + j] = r;
        mi[(size_t)i * NGp + j] = im;
        mr[(size_t)j * NGp + i] = r;
        mi[(size_t)j * NGp + i] = -im;
    }
}

__global__ void k_freq_coeffs(const double* __restrict__ dE, const double* __restrict__ ow, int nw,
                              double* __restrict__ cw) {
    const int w = threadIdx.x;
    if (w < nw) cw[w] = dE[0] * ow[w] / (2.0 * kPi);
}

// All frequencies at once, from Y [w][pair][NGp] (stride sY between frequencies): per pair p,
// g_p += sum_w c_w 2 a_p(w) Y_p(w) and dEda[w][p] = c_w Re(rho_p^H Y_p(w)), with Y_p(w) = W(w) rho_p. The
// sphere goes in segments of 256 kGwPer entries, whose rho_p and g_p a thread keeps in registers over the
// frequencies; the dot products of the segments add up in LDS (nw <= kGwMaxW).
constexpr int kGwPer = 16;
constexpr int kGwMaxW = 256;
__global__ __launch_bounds__(256) void k_grad_weights_all(const double* __restrict__ rr, const double* __restrict__ ri,
                                                          const double* __restrict__ yr, const double* __restrict__ yi,
                                                          size_t sY, int NG, int NGp, const double* __restrict__ a,
                                                          int lda, int nw, const double* __restrict__ cw,
                                                          double* __restrict__ gr, double* __restrict__ gi,
                                                          double* __restrict__ dEda) {
    __shared__ double red[256];
    __shared__ double sdot[kGwMaxW];
    const size_t p = blockIdx.x;
    for (int w = threadIdx.x; w < nw; w += blockDim.x) sdot[w] = 0.0;
    for (int base = 0; base < NG; base += 256 * kGwPer) {
        double xr[kGwPer], xi[kGwPer], hr[kGwPer], hi[kGwPer];
#pragma unroll
        for (int e = 0; e < kGwPer; ++e) {
            const int i = base + threadIdx.x + 256 * e;
            xr[e] = i < NG ? rr[p * NGp + i] : 0.0;
            xi[e] = i < NG ? ri[p * NGp + i] : 0.0;
            hr[e] = 0.0;
            hi[e] = 0.0;
        }
        for (int w = 0; w < nw; ++w) {
            const double f = 2.0 * cw[w] * a[(size_t)w * lda + p];
            const double* ywr = yr + (size_t)w * sY + p * NGp;
            const double* ywi = yi + (size_t)w * sY + p * NGp;
            double dot = 0.0;
#pragma unroll
            for (int e = 0; e < kGwPer; ++e) {
                const int i = base + threadIdx.x + 256 * e;
                if (i < NG) {
                    const double y_r = ywr[i], y_i = ywi[i];
                    dot += xr[e] * y_r + xi[e] * y_i;
                    hr[e] += f * y_r;
                    hi[e] += f * y_i;
                }
            }
            red[threadIdx.x] = dot;
            __syncthreads();
            for (int k = blockDim.x / 2; k > 0; k >>= 1) {
                if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
                __syncthreads();
            }
            if (threadIdx.x == 0) sdot[w] += red[0];
            __syncthreads();
        }
#pragma unroll
        for (int e = 0; e < kGwPer; ++e) {
            const int i = base + threadIdx.x + 256 * e;
            if (i < NG) {
                gr[p * NGp + i] += hr[e];
                gi[p * NGp + i] += hi[e];
            }
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < nw; w += blockDim.x) dEda[(size_t)w * lda + p] = cw[w] * sdot[w];
}

// u_p = sum_w dE/da_p(w) da_p(w)/d(e_n - e_m)   (energy gradient per pair, n side +, m side -)
__global__ void k_pair_eps(const double* __restrict__ dEda, int lda, int nw, const double* __restrict__ epsk,
                           const double* __restrict__ epskq, const double* __restrict__ fk,
                           const double* __restrict__ fkq, const int32_t* __restrict__ pn,
                           const int32_t* __restrict__ pm, int npairs, const double* __restrict__ omega, double prefac,
                           double* __restrict__ u) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const double d = epsk[pn[p]] - epskq[pm[p]];
    const double df = fk[pn[p]] - fkq[pm[p]];
    double s = 0.0;
    for (int w = 0; w < nw; ++w) {
        const double o2 = omega[w] * omega[w];
        const double den = o2 + d * d;
        s += dEda[(size_t)w * lda + p] * prefac * df * 2.0 * (o2 - d * d) / (den * den);
    }
    u[p] = s;
}

// optical row: head_p = num_p/(e_m - e_n); g_num = g_p(0)/(e_m - e_n); energy term added to u_p;
// g_p(0) cleared (the pseudo and PAW values at G = 0 were replaced)
__global__ void k_optical_adj(const double* __restrict__ rr, const double* __restrict__ ri, double* __restrict__ gr,
                              double* __restrict__ gi, int g0, int NGp, const double* __restrict__ epsk,
                              const double* __restrict__ epskq, const int32_t* __restrict__ pn,
                              const int32_t* __restrict__ pm, int npairs, double* __restrict__ u,
                              double* __restrict__ gnum) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const size_t o = (size_t)p * NGp + g0;
    const double den = epskq[pm[p]] - epsk[pn[p]];
    const double g_r = gr[o], g_i = gi[o];
    // Re(conj(g0) head) / (e_m - e_n) goes to e_n with +, to e_m with -
    u[p] += (g_r * rr[o] + g_i * ri[o]) / den;
    gnum[2 * p] = g_r / den;
    gnum[2 * p + 1] = g_i / den;
    gr[o] = 0.0;
    gi[o] = 0.0;
}

// U_m(G, a i) = sum_j P_kq[m][a j] Q[a, i, j](G) for bands m in [mlo, mlo + nm)
__global__ void k_paw_u(const double* __restrict__ Pkq, int ldP, int mlo, const int32_t* __restrict__ proj_off,
                        const int32_t* __restrict__ qoff, int natoms, int nproj, const double* __restrict__ Q, int NG,
                        int NGp, double* __restrict__ Ur, double* __restrict__ Ui) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int ai = blockIdx.y;
    const int s = blockIdx.z;
    if (g >= NGp) return;
    int a = 0;
    while (a + 1 < natoms && proj_off[a + 1] <= ai) ++a;
    const int lo = proj_off[a], np = proj_off[a + 1] - lo, i = ai - lo;
    const size_t m = (size_t)(mlo + s);
    cplx<double> acc = mk(0.0, 0.0);
    if (g < NG)
        for (int j = 0; j < np; ++j) acc = acc + ldc(Pkq, m * ldP + lo + j) * ldc(Q, (size_t)(qoff[a] + i * np + j) * NG + g);
    const size_t o = ((size_t)s * nproj + ai) * NGp + g;
    Ur[o] = acc.x;
    Ui[o] = acc.y;
}

// per pair p and projector column c: Zm[p][c] = sum_G g_p(G) conj(Y_n(G, c)),
// Zn[p][c] = sum_G conj(g_p(G)) U_m(G, c)
constexpr int kZc = 16;
__global__ __launch_bounds__(256) void k_paw_adj(const double* __restrict__ gr, const double* __restrict__ gi, int NG,
                                                 int NGp, const double* __restrict__ Yr, const double* __restrict__ Yi,
                                                 int nlo, const double* __restrict__ Ur, const double* __restrict__ Ui,
                                                 int mlo, int nproj, const int32_t* __restrict__ pn,
                                                 const int32_t* __restrict__ pm, double* __restrict__ Zm,
                                                 double* __restrict__ Zn) {
    __shared__ double red[4][kZc][65];
    const size_t p = blockIdx.x;
    const int c0 = blockIdx.y * kZc;
    const int nc = min(kZc, nproj - c0);
    const size_t ys = (size_t)(pn[p] - nlo) * nproj * NGp, us = (size_t)(pm[p] - mlo) * nproj * NGp;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double zmr[kZc], zmi[kZc], znr[kZc], zni[kZc];
    for (int c = 0; c < kZc; ++c) zmr[c] = zmi[c] = znr[c] = zni[c] = 0.0;
    for (int g = threadIdx.x; g < NG; g += blockDim.x) {
        const double g_r = gr[p * NGp + g], g_i = gi[p * NGp + g];
        for (int c = 0; c < nc; ++c) {
            const size_t yo = ys + (size_t)(c0 + c) * NGp + g, uo = us + (size_t)(c0 + c) * NGp + g;
            const double y_r = Yr[yo], y_i = Yi[yo], u_r = Ur[uo], u_i = Ui[uo];
            // g conj(Y)
            zmr[c] += g_r * y_r + g_i * y_i;
            zmi[c] += g_i * y_r - g_r * y_i;
            // conj(g) U
            znr[c] += g_r * u_r + g_i * u_i;
            zni[c] += g_r * u_i - g_i * u_r;
        }
    }
    // wave-level then block-level reduction
    for (int c = 0; c < nc; ++c) {
        double v[4] = {zmr[c], zmi[c], znr[c], zni[c]};
        for (int q = 0; q < 4; ++q) {
            double x = v[q];
            for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
            if (lane == 0) red[q][c][wv] = x;
        }
    }
    __syncthreads();
    if (threadIdx.x < nc) {
        const int c = threadIdx.x;
        double s[4];
        for (int q = 0; q < 4; ++q) s[q] = red[q][c][0] + red[q][c][1] + red[q][c][2] + red[q][c][3];
        const size_t o = 2 * (p * nproj + c0 + c);
        Zm[o] = s[0];
        Zm[o + 1] = s[1];
        Zn[o] = s[2];
        Zn[o + 1] = s[3];
    }
}

// Owner-band reductions over a CSR list of pairs (entries are pair indices).
// dP_k[n][c] += sum_{p in n} Zn[p][c] (+ optical: sum_j conj(gp) D_cj P_kq[m][j]),
// dP_kq[m][c] += sum_{p in m} Zm[p][c] (+ optical: sum_i gp P_k[n][i] D_ic), gp = i g_num
__global__ void k_paw_reduce(const double* __restrict__ Z, const int32_t* __restrict__ start,
                             const int32_t* __restrict__ list, int nproj, double* __restrict__ dP, int band0,
                             const double* __restrict__ gnum, const double* __restrict__ Pother,
                             const int32_t* __restrict__ other, const double* __restrict__ Dq,
                             const int32_t* __restrict__ proj_off, const int32_t* __restrict__ qoff, int natoms,
                             int side) {
    const int b = blockIdx.x;
    const int c = blockIdx.y * blockDim.x + threadIdx.x;
    if (c >= nproj) return;
    double sr = 0, si = 0;
    int a = 0;
    while (a + 1 < natoms && proj_off[a + 1] <= c) ++a;
    const int lo = proj_off[a], np = proj_off[a + 1] - lo, ci = c - lo;
    for (int e = start[b]; e < start[b + 1]; ++e) {
        const int p = list[e];
        sr += Z[2 * ((size_t)p * nproj + c)];
        si += Z[2 * ((size_t)p * nproj + c) + 1];
        if (gnum) {
            // gp = i g_num
            const double gpr = -gnum[2 * p + 1], gpi = gnum[2 * p];
            const size_t ob = (size_t)other[p] * nproj;
            for (int j = 0; j < np; ++j) {
                if (side == 0) {
                    // n side: conj(gp) D[c][j] P_kq[m][j]
                    const double d = Dq[qoff[a] + ci * np + j];
                    const double pr = Pother[2 * (ob + lo + j)], pi = Pother[2 * (ob + lo + j) + 1];
                    sr += d * (gpr * pr + gpi * pi);
                    si += d * (gpr * pi - gpi * pr);
                } else {
                    // m side: gp P_k[n][j] D[j][c]
                    const double d = Dq[qoff[a] + j * np + ci];
                    const double pr = Pother[2 * (ob + lo + j)], pi = Pother[2 * (ob + lo + j) + 1];
                    sr += d * (gpr * pr - gpi * pi);
                    si += d * (gpr * pi + gpi * pr);
                }
            }
        }
    }
    const size_t o = 2 * ((size_t)(band0 + b) * nproj + c);
    dP[o] += sr;
    dP[o + 1] += si;
}

// dE/de_n += sum_{p in n} u_p, dE/de_m -= sum_{p in m} u_p
__global__ void k_eps_reduce(const double* __restrict__ u, const int32_t* __restrict__ start,
                             const int32_t* __restrict__ list, int nbands, double sign, double* __restrict__ de) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbands) return;
    double s = 0;
    for (int e = start[b]; e < start[b + 1]; ++e) s += u[list[e]];
    de[b] += sign * s;
}

// optical momentum part in coefficient space:
// dC_kq[m](Q) += w_Q sum_{p in m} g_num_p C_k[n_p](Q);  dC_k[n](Q) += w_Q sum_{p in n} conj(g_num_p) C_kq[m_p](Q)
__global__ void k_optical_c(const double* __restrict__ gnum, const int32_t* __restrict__ start,
                            const int32_t* __restrict__ list, const int32_t* __restrict__ other,
                            const double* __restrict__ Cother, int nQ, const double* __restrict__ wq, int side,
                            double* __restrict__ dC) {
    const int b = blockIdx.y;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nQ) return;
    double sr = 0, si = 0;
    for (int e = start[b]; e < start[b + 1]; ++e) {
        const int p = list[e];
        const double gr = gnum[2 * p], gi = side == 0 ? -gnum[2 * p + 1] : gnum[2 * p + 1];
        const double cr = Cother[2 * ((size_t)other[p] * nQ + q)], ci = Cother[2 * ((size_t)other[p] * nQ + q) + 1];
        sr += gr * cr - gi * ci;
        si += gr * ci + gi * cr;
    }
    dC[2 * ((size_t)b * nQ + q)] += wq[q] * sr;
    dC[2 * ((size_t)b * nQ + q) + 1] += wq[q] * si;
}

template <int DIR, typename T, class Addr>
__device__ cplx<T>* stages(cplx<T>* src, cplx<T>* dst, const FftPlan& plan, int N, int nlines, bool line_fast,
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

// adjoint of the z pass and the gather: T'[p][z][c] = sum_kz e^{+2 pi i z kz/N3} g_p(G(kz, c)) / N
__global__ __launch_bounds__(256) void k_zadj(const double* __restrict__ gr, const double* __restrict__ gi, int NGp,
                                              PairGeom g, int CB, const int32_t* __restrict__ col_start,
                                              const int32_t* __restrict__ col_g, const int32_t* __restrict__ col_kz,
                                              const cplx<double>* __restrict__ tw3g, cplx<double>* __restrict__ tadj) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N3 = g.N3, ncols = g.ncols;
    cplx<double>* tw3 = reinterpret_cast<cplx<double>*>(smem);
    cplx<double>* A = tw3 + N3;
    cplx<double>* B = A + (size_t)CB * N3;
    const size_t p = blockIdx.x;
    const int c0 = blockIdx.y * CB;
    const int nc = min(CB, ncols - c0);
    for (int t = threadIdx.x; t < N3; t += blockDim.x) tw3[t] = tw3g[t];
    for (int f = threadIdx.x; f < N3 * CB; f += blockDim.x) A[f] = mk(0.0, 0.0);
    __syncthreads();
    const double invN = 1.0 / ((double)g.N1 * g.N2 * N3);
    for (int i = col_start[c0] + threadIdx.x; i < col_start[c0 + nc]; i += blockDim.x) {
        const int gi_ = col_g[i], kz = col_kz[i] >> 16, c = (col_kz[i] & 0xffff) - c0;
        A[kz * CB + c] = mk(gr[p * NGp + gi_] * invN, gi[p * NGp + gi_] * invN);
    }
    __syncthreads();
    auto az = [CB](int l, int e) { return e * CB + l; };
    cplx<double>* rz = stages<1>(A, B, g.p3, N3, nc, true, az, tw3);
    for (int f = threadIdx.x; f < N3 * nc; f += blockDim.x) {
        const int z = f / nc, c = f - z * nc;
        tadj[(p * N3 + z) * ncols + c0 + c] = rz[z * CB + c];
    }
}

// owner-band accumulation over the band's pairs on one z-plane:
//   side 1 (owner m): phibar_kq[m] += phi_k[n] xbar_p
//   side 0 (owner n): phibar_k[n]  += phi_kq[m] conj(xbar_p)
// xbar_p = inverse y (kept columns) and inverse x transforms of T'_p on this plane.
__global__ __launch_bounds__(256) void k_xyadj(const cplx<double>* __restrict__ tadj, PairGeom g,
                                               const int32_t* __restrict__ start, const int32_t* __restrict__ list,
                                               const int32_t* __restrict__ other, const cplx<double>* __restrict__ phio,
                                               int band0, int side, const int32_t* __restrict__ kxg,
                                               const int32_t* __restrict__ kyg, const cplx<double>* __restrict__ tw1g,
                                               const cplx<double>* __restrict__ tw2g, cplx<double>* __restrict__ phibar) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N1 = g.N1, N2 = g.N2, N3 = g.N3, K1 = g.K1, K2 = g.K2;
    const int plane = N1 * N2;
    cplx<double>* tw1 = reinterpret_cast<cplx<double>*>(smem);
    cplx<double>* tw2 = tw1 + N1;
    cplx<double>* A = tw2 + N2;
    cplx<double>* B = A + plane;
    int* kx = reinterpret_cast<int*>(B + plane);
    int* ky = kx + K1;
    const int b = blockIdx.x, z = blockIdx.y;
    const size_t vol = (size_t)plane * N3;
    for (int t = threadIdx.x; t < N1; t += blockDim.x) tw1[t] = tw1g[t];
    for (int t = threadIdx.x; t < N2; t += blockDim.x) tw2[t] = tw2g[t];
    for (int t = threadIdx.x; t < K1; t += blockDim.x) kx[t] = kxg[t];
    for (int t = threadIdx.x; t < K2; t += blockDim.x) ky[t] = kyg[t];
    constexpr int kPer = 16;  // plane elements per thread kept in registers (plane <= 4096)
    cplx<double> acc[kPer];
    for (int e = 0; e < kPer; ++e) acc[e] = mk(0.0, 0.0);
    const int kk = K1 * K2;
    for (int e = start[b]; e < start[b + 1]; ++e) {
        const int p = list[e];
        __syncthreads();
        for (int f = threadIdx.x; f < plane; f += blockDim.x) A[f] = mk(0.0, 0.0);
        __syncthreads();
        for (int f = threadIdx.x; f < kk; f += blockDim.x) {
            const int iy = f / K1, ix = f - iy * K1;
            A[ky[iy] * N1 + kx[ix]] = tadj[((size_t)p * N3 + z) * kk + f];
        }
        __syncthreads();
        auto ay = [=](int l, int e2) { return e2 * N1 + kx[l]; };
        cplx<double>* ry = stages<1>(A, B, g.p2, N2, K1, true, ay, tw2);
        cplx<double>* oy = (ry == A) ? B : A;
        // inverse x on every line; lines untouched by the y pass are zero in both buffers
        for (int f = threadIdx.x; f < plane; f += blockDim.x) {
            const int x = f % N1;
            bool kept = false;
            for (int i = 0; i < K1; ++i) kept |= (kx[i] == x);
            if (!kept) ry[f] = mk(0.0, 0.0);
        }
        __syncthreads();
        auto ax = [N1](int l, int e2) { return l * N1 + e2; };
        cplx<double>* rx = stages<1>(ry, oy, g.p1, N1, N2, false, ax, tw1);
        const size_t ob = (size_t)other[p] * vol + (size_t)z * plane;
        for (int q = 0; q < kPer; ++q) {
            const int f = threadIdx.x + q * blockDim.x;
            if (f < plane) {
                const cplx<double> xb = rx[f];
                const cplx<double> ph = phio[ob + f];
                acc[q] = acc[q] + (side == 1 ? ph * xb : ph * conj(xb));
            }
        }
    }
    const size_t out = (size_t)(band0 + b) * vol + (size_t)z * plane;
    for (int q = 0; q < kPer; ++q) {
        const int f = threadIdx.x + q * blockDim.x;
        if (f < plane) phibar[out + f] = phibar[out + f] + acc[q];
    }
}

// dC[b][Q] += phibar_hat[b][map[Q]]
__global__ void k_gather_c(const cplx<double>* __restrict__ ph, size_t vol, const int32_t* __restrict__ map, int nQ,
                           double* __restrict__ dC) {
    const size_t b = blockIdx.y;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < nQ; q += gridDim.x * blockDim.x) {
        const cplx<double> v = ph[b * vol + map[q]];
        dC[2 * (b * nQ + q)] += v.x;
        dC[2 * (b * nQ + q) + 1] += v.y;
    }
}

__global__ void k_zero(double* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0.0;
}

}  // namespace

hipError_t launch_gemm_c64(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0 || g.nbatch <= 0) return hipSuccess;
    if (g.K <= 0 && g.beta) return hipSuccess;
    dim3 grid((unsigned)((g.M + kTile - 1) / kTile), (unsigned)((g.N + kTile - 1) / kTile), (unsigned)g.nbatch);
    hipLaunchKernelGGL(k_gemm_c64, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_gemm_c64_shortk(const GemmArgs& g, hipStream_t s) {
    if (g.K < 1 || g.K > kShortK) return launch_gemm_c64(g, s);
    if (g.M <= 0 || g.N <= 0 || g.nbatch <= 0) return hipSuccess;
    dim3 grid((unsigned)((g.M + 31) / 32), (unsigned)((g.N + 31) / 32), (unsigned)g.nbatch);
    hipLaunchKernelGGL(k_gemm_c64_k64, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_identity(double* Xr, double* Xi, int n, int ld, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_identity, dim3((unsigned)ld, (unsigned)nb), dim3(256), 0, s, Xr, Xi, n, ld);
    return hipGetLastError();
}

hipError_t launch_build_w(double* Mr, double* Mi, int NG, int NGp, int nw, const double* vs, hipStream_t s) {
    hipLaunchKernelGGL(k_build_w, dim3((unsigned)NGp, (unsigned)nw), dim3(256), 0, s, Mr, Mi, NG, NGp, vs);
    return hipGetLastError();
}

hipError_t launch_freq_coeffs(const double* dE, const double* ow, int nw, double* cw, hipStream_t s) {
    hipLaunchKernelGGL(k_freq_coeffs, dim3(1), dim3(64), 0, s, dE, ow, nw, cw);
    return hipGetLastError();
}

hipError_t launch_grad_weights_all(const double* rr, const double* ri, const double* yr, const double* yi, size_t sY,
                                   int NG, int NGp, const double* a, int lda, int nw, const double* cw, double* gr,
                                   double* gi, double* dEda, int npairs, hipStream_t s) {
    if (!npairs) return hipSuccess;
    if (nw > kGwMaxW) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_grad_weights_all, dim3((unsigned)npairs), dim3(256), 0, s, rr, ri, yr, yi, sY, NG, NGp, a, lda,
                       nw, cw, gr, gi, dEda);
    return hipGetLastError();
}

hipError_t launch_pair_eps(const double* dEda, int lda, int nw, const double* epsk, const double* epskq,
                           const double* fk, const double* fkq, const int32_t* pn, const int32_t* pm, int npairs,
                           const double* omega, double prefac, double* u, hipStream_t s) {
    if (!npairs) return hipSuccess;
    hipLaunchKernelGGL(k_pair_eps, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, dEda, lda, nw, epsk, epskq,
                       fk, fkq, pn, pm, npairs, omega, prefac, u);
    return hipGetLastError();
}

hipError_t launch_optical_adj(const double* rr, const double* ri, double* gr, double* gi, int g0, int NGp,
                              const double* epsk, const double* epskq, const int32_t* pn, const int32_t* pm,
                              int npairs, double* u, double* gnum, hipStream_t s) {
    if (!npairs) return hipSuccess;
    hipLaunchKernelGGL(k_optical_adj, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s, rr, ri, gr, gi, g0, NGp,
                       epsk, epskq, pn, pm, npairs, u, gnum);
    return hipGetLastError();
}

hipError_t launch_paw_u(const double* Pkq, int ldP, int mlo, int nm, const int32_t* proj_off, const int32_t* qoff,
                        int natoms, int nproj, const double* Q, int NG, int NGp, double* Ur, double* Ui,
                        hipStream_t s) {
    if (!nm || !nproj) return hipSuccess;
    dim3 grid((unsigned)((NGp + 255) / 256), (unsigned)nproj, (unsigned)nm);
    hipLaunchKernelGGL(k_paw_u, grid, dim3(256), 0, s, Pkq, ldP, mlo, proj_off, qoff, natoms, nproj, Q, NG, NGp, Ur, Ui);
    return hipGetLastError();
}

hipError_t launch_paw_adj(const double* gr, const double* gi, int NG, int NGp, const double* Yr, const double* Yi,
                          int nlo, const double* Ur, const double* Ui, int mlo, int nproj, const int32_t* pn,
                          const int32_t* pm, int npairs, double* Zm, double* Zn, hipStream_t s) {
    if (!npairs || !nproj) return hipSuccess;
    dim3 grid((unsigned)npairs, (unsigned)((nproj + kZc - 1) / kZc));
    hipLaunchKernelGGL(k_paw_adj, grid, dim3(256), 0, s, gr, gi, NG, NGp, Yr, Yi, nlo, Ur, Ui, mlo, nproj, pn, pm, Zm,
                       Zn);
    return hipGetLastError();
}

hipError_t launch_paw_reduce(const double* Z, const int32_t* start, const int32_t* list, int nb, int nproj, double* dP,
                             int band0, const double* gnum, const double* Pother, const int32_t* other,
                             const double* Dq, const int32_t* proj_off, const int32_t* qoff, int natoms, int side,
                             hipStream_t s) {
    if (!nb || !nproj) return hipSuccess;
    dim3 grid((unsigned)nb, (unsigned)((nproj + 63) / 64));
    hipLaunchKernelGGL(k_paw_reduce, grid, dim3(64), 0, s, Z, start, list, nproj, dP, band0, gnum, Pother, other, Dq,
                       proj_off, qoff, natoms, side);
    return hipGetLastError();
}

hipError_t launch_eps_reduce(const double* u, const int32_t* start, const int32_t* list, int nbands, double sign,
                             double* de, hipStream_t s) {
    if (!nbands) return hipSuccess;
    hipLaunchKernelGGL(k_eps_reduce, dim3((unsigned)((nbands + 255) / 256)), dim3(256), 0, s, u, start, list, nbands,
                       sign, de);
    return hipGetLastError();
}

hipError_t launch_optical_c(const double* gnum, const int32_t* start, const int32_t* list, const int32_t* other,
                            const double* Cother, int nQ, const double* wq, int side, int nb, double* dC,
                            hipStream_t s) {
    if (!nb) return hipSuccess;
    dim3 grid((unsigned)((nQ + 255) / 256), (unsigned)nb);
    hipLaunchKernelGGL(k_optical_c, grid, dim3(256), 0, s, gnum, start, list, other, Cother, nQ, wq, side, dC);
    return hipGetLastError();
}

hipError_t launch_zadj(const double* gr, const double* gi, int NGp, int npairs, const PairGeom& g,
                       const int32_t* col_start, const int32_t* col_g, const int32_t* col_kz, const cplx<double>* tw3,
                       cplx<double>* tadj, hipStream_t s) {
    if (!npairs) return hipSuccess;
    const size_t per = 64 * 1024 / sizeof(cplx<double>);
    int CB = (int)((per - g.N3) / (2 * (size_t)g.N3));
    if (CB > g.ncols) CB = g.ncols;
    if (CB < 1) return hipErrorInvalidValue;
    const size_t lds = ((size_t)g.N3 + 2 * (size_t)CB * g.N3) * sizeof(cplx<double>);
    dim3 grid((unsigned)npairs, (unsigned)((g.ncols + CB - 1) / CB));
    hipLaunchKernelGGL(k_zadj, grid, dim3(256), lds, s, gr, gi, NGp, g, CB, col_start, col_g, col_kz, tw3, tadj);
    return hipGetLastError();
}

hipError_t launch_xyadj(const cplx<double>* tadj, const PairGeom& g, const int32_t* start, const int32_t* list,
                        const int32_t* other, const cplx<double>* phio, int band0, int nb, int side,
                        const int32_t* kx, const int32_t* ky, const cplx<double>* tw1, const cplx<double>* tw2,
                        cplx<double>* phibar, hipStream_t s) {
    if (!nb) return hipSuccess;
    const size_t plane = (size_t)g.N1 * g.N2;
    if (plane > 16 * 256) return hipErrorInvalidValue;
    const size_t lds = (g.N1 + g.N2 + 2 * plane) * sizeof(cplx<double>) + (g.K1 + g.K2) * sizeof(int);
    dim3 grid((unsigned)nb, (unsigned)g.N3);
    hipLaunchKernelGGL(k_xyadj, grid, dim3(256), lds, s, tadj, g, start, list, other, phio, band0, side, kx, ky, tw1,
                       tw2, phibar);
    return hipGetLastError();
}

hipError_t launch_gather_c(const cplx<double>* ph, size_t vol, const int32_t* map, int nQ, int nb, double* dC,
                           hipStream_t s) {
    if (!nb || !nQ) return hipSuccess;
    hipLaunchKernelGGL(k_gather_c, dim3((unsigned)((nQ + 255) / 256), (unsigned)nb), dim3(256), 0, s, ph, vol, map, nQ,
                       dC);
    return hipGetLastError();
}

hipError_t launch_zero_d(double* p, size_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace rpa
