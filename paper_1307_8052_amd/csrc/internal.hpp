// Internal interfaces between the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft.hpp"

namespace rpa {

// Tile edge of the rank-k update and of the Cholesky blocks; the padded
// G dimension NGp is a multiple of it.
constexpr int kTile = 64;

// Workgroup size of every FFT-stage kernel.
constexpr int kFftThreads = 256;

// Geometry of the pruned pair-density transform for one q.
struct PairGeom {
    int N1, N2, N3;       // grid
    int K1, K2;           // kept Miller ranges along a1 and a2 (the sphere's extent)
    int ncols;            // K1*K2 columns (m1, m2) of the sphere's bounding box
    int NG, NGp;          // sphere size and its padded size
    FftPlan p1, p2, p3;
    int x0, y0;           // grid index of the first kept x / y frequency (the kept sets wrap modulo N)
    int nzc;              // columns that hold sphere entries (the only ones transformed along z)
    int z0, K3;           // grid index of the sphere's first z frequency and its z extent
};

// ----------------------------------------------------------------- FFT stages
template <typename T>
hipError_t launch_fill_zero(cplx<T>* p, size_t n, hipStream_t s);

template <typename T>
hipError_t launch_orb_scatter(const double* C, int nbands, int nQ, const int32_t* map, size_t vol,
                              cplx<T>* phi, hipStream_t s);

// In-place batched 1-D inverse transforms along one axis of [nb][N3][N2][N1] arrays.
template <typename T>
hipError_t launch_fft_axis(cplx<T>* data, int nb, int N1, int N2, int N3, int axis, const FftPlan& plan,
                           const cplx<T>* tw, int dir, hipStream_t s);

template <typename T>
hipError_t launch_pair_xy(const cplx<T>* phik, const cplx<T>* phikq, const int32_t* pn, const int32_t* pm,
                          int npairs, const PairGeom& g, const int32_t* kx_grid, const int32_t* ky_grid,
                          const cplx<T>* tw1, const cplx<T>* tw2, cplx<T>* tbuf, hipStream_t s);

// Register-resident variants of the two pair kernels (same tbuf layout and
// output): the xy kernel when N1 == N2 has a compiled line length, the z kernel
// when N3 has one; each can pair with the other's LDS-pass counterpart.
template <typename T>
bool pair_xy_reg_supported(const PairGeom& g);
template <typename T>
bool pair_z_reg_supported(const PairGeom& g);
template <typename T>
hipError_t launch_pair_xy_reg(const cplx<T>* phik, const cplx<T>* phikq, const int32_t* pn, const int32_t* pm,
                              int npairs, const PairGeom& g, cplx<T>* tbuf, hipStream_t s);
// In-place transforms of nb grids [nb][N3][N2][N1] (dir = +1 inverse without
// 1/N, -1 forward) with register-resident lines: along z, or along x and y;
// hipErrorNotSupported where the register kernels do not cover the axis. Along z,
// cols (DEVICE, ncols offsets y * N1 + x into a plane) restricts the transform to
// those columns (the others must be zero); NULL transforms all of them.
template <typename T>
hipError_t launch_grid_fft_z_reg(cplx<T>* data, int nb, int N1, int N2, int N3, int dir, const int32_t* cols,
                                 int ncols, hipStream_t s);
template <typename T>
hipError_t launch_grid_fft_xy_reg(cplx<T>* data, int nb, int N1, int N2, int N3, int dir, hipStream_t s);
template <typename T>
// zcol: the box column of each of the g.nzc columns that hold sphere entries; col_start and the column
// bits of col_kz index that list
hipError_t launch_pair_z_reg(const cplx<T>* tbuf, int npairs, const PairGeom& g, const int32_t* zcol,
                             const int32_t* col_start, const int32_t* col_g, const int32_t* col_kz, T* rho_re,
                             T* rho_im, hipStream_t s);
// The z kernel for N3 = 4 M (M a compiled line length) by quads of lanes, keeping only the sphere's z window
// [z0, z0 + K3) in LDS; same arguments and output as launch_pair_z_reg.
template <typename T>
bool pair_z_quad_supported(const PairGeom& g);
template <typename T>
hipError_t launch_pair_z_quad(const cplx<T>* tbuf, int npairs, const PairGeom& g, const int32_t* zcol,
                              const int32_t* col_start, const int32_t* col_g, const int32_t* col_kz, T* rho_re,
                              T* rho_im, hipStream_t s);
template <typename T>
hipError_t launch_pair_z_gather(const cplx<T>* tbuf, int npairs, const PairGeom& g, const int32_t* zcol,
                                const int32_t* col_start, const int32_t* col_g, const int32_t* col_kz,
                                const cplx<T>* tw3, T* rho_re, T* rho_im, hipStream_t s);

// ------------------------------------------------------------ linear algebra
template <typename T>
hipError_t launch_paw_y(const double* Pk, int ldP, const int32_t* nlist, int nn, const int32_t* proj_off,
                        const int32_t* qoff, int natoms, int nprojtot, const double* Q, int NG, int NGp,
                        T* Yre, T* Yim, hipStream_t s);

template <typename T>
hipError_t launch_paw_add(const T* Yre, const T* Yim, const int32_t* pn, int nlo, const int32_t* pm,
                          const double* Pkq, int ldP, int nprojtot, int npairs, int NG, int NGp, T* rho_re,
                          T* rho_im, hipStream_t s);
// Intraband head at q -> 0: term[b] = weight (-df/de)[b] (qhat.v_n)^2 for n = band[b] (band velocity from
// the coefficients, the table wq = qhat.(k + G_Q) and the PAW nabla table Dq), then
// head[w * stride] += -(sum of terms) inv_volume / omega[w]^2 (nw <= 256)
hipError_t launch_band_drude(const double* C, int nQ, const double* wq, const double* P, int ldP, const double* Dq,
                             const int32_t* proj_off, const int32_t* qoff, int natoms, const int32_t* band,
                             const double* mdf, int nbands, double weight, double* term, hipStream_t s);
hipError_t launch_add_drude(const double* term, int nterms, const double* omega, int nw, double inv_volume,
                            double* head, long long stride, hipStream_t s);

// Real frequencies w + i eta (2 nw weight rows: Re a for w < nw, Im a for nw + w; the chi0 of the call is
// A_w + i B_w with Hermitian A_w, B_w accumulated from those rows)
hipError_t launch_weights_real(const double* epsk, const double* epskq, const double* fk, const double* fkq,
                               const int32_t* pn, const int32_t* pm, int npairs, const double* omega, int nw,
                               double eta, double prefac, double* a, int lda, hipStream_t s);
hipError_t launch_add_drude_real(const double* term, int nterms, const double* omega, int nw, double eta,
                                 double inv_volume, double* head, long long stride, hipStream_t s);
hipError_t launch_chi_out_real(const double* Cre, const double* Cim, int ldC, int NG, int nw, double* out,
                               hipStream_t s);

// PAW term as an MFMA GEMM (k_paw.hip): Z_m = Q P'_m for m = m_lo .. m_lo + nslots - 1 into Zr/Zi
// [nslots][nproj][NGp], then rho[p] += conj(P_k[pn[p]]) Z_{pm[p]} for the npairs pairs (pm within the
// slots); NGp a multiple of 64
// Y_n for n = n_lo .. n_lo + nslots - 1 into Yr/Yi [nslots][nproj][NGp] (eight bands per thread)
template <typename T>
hipError_t launch_paw_yn(const double* Pk, int ldP, int n_lo, int nslots, const int32_t* proj_off, const int32_t* qoff,
                         int natoms, int nproj, const double* Q, int NG, int NGp, T* Yr, T* Yi, hipStream_t s);
// The n-factorised MFMA form: rho[perm[f + r]] += P_kq[pm[perm[f + r]]] . Y[n] for the nseg segments
// (n - n_lo, f, count <= 64) of seg, with Y [n - n_lo][nproj][NGp] from launch_paw_y; NGp a multiple of 64
template <typename T>
hipError_t launch_paw_mfma_n(const T* Yr, const T* Yi, int nproj, const double* Pkq, int ldP, const int32_t* pm,
                             const int32_t* seg, int nseg, const int32_t* perm, int NGp, T* rre, T* rim,
                             hipStream_t s);
template <typename T>
hipError_t launch_paw_mfma(const double* Pk, const double* Pkq, int ldP, const int32_t* pn, const int32_t* pm,
                           int npairs, int m_lo, int nslots, const int32_t* proj_off, const int32_t* qoff, int natoms,
                           int nproj, const double* Q, int NG, int NGp, T* Zr, T* Zi, T* rre, T* rim, hipStream_t s);

template <typename T>
hipError_t launch_optical_row(const double* Ck, const double* Ckq, int nQ, const double* wq, const double* Pk,
                              const double* Pkq, int ldP, const double* Dq, const int32_t* proj_off,
                              const int32_t* qoff, int natoms, const double* epsk, const double* epskq,
                              const int32_t* pn, const int32_t* pm, int npairs, int g0, int NGp, T* rho_re,
                              T* rho_im, hipStream_t s);

hipError_t launch_weights(const double* epsk, const double* epskq, const double* fk, const double* fkq,
                          const int32_t* pn, const int32_t* pm, int npairs, const double* omega, int nw,
                          double prefac, double* a, int lda, hipStream_t s);

// C[b] (lower tiles of the nT x nT block region at (r0, r0)) +=
//   sum_k w[b][k] A[b][k][c0 + i] conj(A[b][k][c0 + j]); w == nullptr means alpha.
struct HerkArgs {
    const double* Are; const double* Aim; long long sA; int ldA; int colA; int K;
    const double* w; long long sw; double alpha;
    double* Cre; double* Cim; long long sC; int ldC; int r0;
    int nT; int nbatch;
};
hipError_t launch_herk_f64(const HerkArgs& h, hipStream_t s);

// Split-precision rank-k update (FP32 operands, hi/lo BF16 or FP16 products on
// MFMA, FP32 accumulation, FP64 output accumulation).
struct HerkSplitArgs {
    const float* Are; const float* Aim; int ldA; int K;
    const double* w; int lda;
    double* Cre; double* Cim; long long sC; int ldC;
    int nT; int nw;
    int fp16;            // 0 = BF16, 1 = FP16 (scaled)
    const float* wscale; // FP16: [nw] scales of X_w and [nw] the scale of rho (nullptr for BF16)
};
hipError_t launch_herk_split(const HerkSplitArgs& h, hipStream_t s);
// FP16 operand scales from the chunk's rho (n = K * ld elements per part) and weights; `part`
// holds 256 floats of scratch.
hipError_t launch_split_scales(const float* rre, const float* rim, size_t n, const double* a, int lda, int K, int nw,
                               float* scales, float* part, hipStream_t s);

// Large-tile split update: operands pre-packed K-blocked ([K/32][NGq][32]) by
// launch_pack_split; NGq = NGp rounded up to 128; 128x128 lower tiles.
struct HerkSplit2Args {
    const float* Xre; const float* Xim; const unsigned short* B[4]; int NGq; int K;
    const double* w; int lda;
    double* Cre; double* Cim; long long sC; int ldC;
    int ntiles; int nw; int fp16; const float* scales;
    int overwrite;       // variants 4 and 5: C = the update instead of C += it (a fresh accumulator)
};
hipError_t launch_pack_split(const float* rre, const float* rim, int K, int ldr, int NGq, const float* scales, int nw,
                             int fp16, float* Xre, float* Xim, unsigned short* const B[4], hipStream_t s);
// pipelined = 1: double-buffered, branch-free K loop (same operands and result)
// 64 x 128 tiles (ntiles = sum over 64-row blocks I of I/2 + 1), FP32 partial sums
// added into FP64 every 8 K-steps; four waves of 64 x 32, or eight of 32 x 32
hipError_t launch_herk_split4(const HerkSplit2Args& h, int eight_waves, hipStream_t s);


// -K = -v_i v_j chi_ij on the lower triangle (in place, planar), zero padding,
// and Tr K per frequency.
hipError_t launch_build_negk(double* Cre, double* Cim, int ldC, int NG, int NGp, int nw,
                             const double* vsqrt, double* trk, hipStream_t s);
hipError_t launch_build_negk_from_full(const double* chi, int NG, double* Cre, double* Cim, int NGp, int nw,
                                       const double* vsqrt, double* trk, hipStream_t s);

hipError_t launch_chol_panel(double* Cre, double* Cim, int ldC, int j0, int nw, double* Lre, double* Lim,
                             double* logdet, int* fail, hipStream_t s);
// Both also write the factor L (lower triangle, diagonal real) back into C.
// Pre/Pim: the solved panel of each matrix, P[c][r] at c * NGp + r; one matrix every sP doubles.
hipError_t launch_chol_trsm(double* Cre, double* Cim, int ldC, int j0, int NGp, int nw,
                            const double* Lre, const double* Lim, double* Pre, double* Pim, long long sP,
                            hipStream_t s);
hipError_t launch_finalize(const double* logdet, const double* trk, const int* fail, const double* wgt, int nw,
                           double* F, double* ec, hipStream_t s);

hipError_t launch_zero(double* d, int nd, int* iv, int ni, hipStream_t s);
// out[0] = sum_j w[j] x[j]
hipError_t launch_weighted_sum(const double* x, const double* w, int n, double* out, hipStream_t s);
// deterministic pseudo-random fill in [-1, 1) (tuning inputs)
hipError_t launch_fill_pattern(float* f, size_t nf, double* d, size_t nd, hipStream_t s);

// planar (re, im) [npairs][NGp] of type T -> interleaved complex128 [npairs][NG]
template <typename T>
hipError_t launch_rho_out(const T* rre, const T* rim, int npairs, int NG, int NGp, double* out, hipStream_t s);

hipError_t launch_conj_copy(const double* in, size_t n, double* out, hipStream_t s);
hipError_t launch_rotate_proj(const double* Pin, int nb, int nproj, const int32_t* tab, const double* D,
                              const double* ph, int tr, double* Pout, hipStream_t s);
hipError_t launch_chi_out(const double* Cre, const double* Cim, int ldC, int NG, int nw, int add, double* out,
                          hipStream_t s);

// ------------------------------------------------------------------ adjoint
// C[b] = beta C[b] + alpha op(A[b]) op(B[b]); A(i,k) at i*aI + k*aK, B(k,j) at
// k*bK + j*bJ, C(i,j) at i*ldC + j; conj flags conjugate an operand; beta 0 or 1.
struct GemmArgs {
    int M, N, K, nbatch;
    const double* Ar; const double* Ai; long long sA; long long aI, aK; int conjA;
    const double* Br; const double* Bi; long long sB; long long bK, bJ; int conjB;
    double* Cr; double* Ci; long long sC; long long ldC; double alpha; int beta;
    int lower;           // only entries i >= j of C are needed (a hint: tiles wholly above may be skipped)
    int ktri;            // A[i][k] = 0 for k < i and B[k][j] = 0 for k < j (both lower-triangular factors of a
                         // product L^H L): the K loop of a tile starts at its first row or column
};
hipError_t launch_gemm_c64(const GemmArgs& g, hipStream_t s);
// The same product for 1 <= K <= 64 in one round trip to memory (latency-bound shapes of the Cholesky
// chain); other K go to launch_gemm_c64.
hipError_t launch_gemm_c64_shortk(const GemmArgs& g, hipStream_t s);
hipError_t launch_identity(double* Xr, double* Xi, int n, int ld, int nb, hipStream_t s);
hipError_t launch_build_w(double* Mr, double* Mi, int NG, int NGp, int nw, const double* vs, hipStream_t s);
hipError_t launch_freq_coeffs(const double* dE, const double* ow, int nw, double* cw, hipStream_t s);
// all nw frequencies in one launch, Y [w] at yr/yi + w sY (nw <= 256)
hipError_t launch_grad_weights_all(const double* rr, const double* ri, const double* yr, const double* yi, size_t sY,
                                   int NG, int NGp, const double* a, int lda, int nw, const double* cw, double* gr,
                                   double* gi, double* dEda, int npairs, hipStream_t s);

hipError_t launch_pair_eps(const double* dEda, int lda, int nw, const double* epsk, const double* epskq,
                           const double* fk, const double* fkq, const int32_t* pn, const int32_t* pm, int npairs,
                           const double* omega, double prefac, double* u, hipStream_t s);
hipError_t launch_optical_adj(const double* rr, const double* ri, double* gr, double* gi, int g0, int NGp,
                              const double* epsk, const double* epskq, const int32_t* pn, const int32_t* pm,
                              int npairs, double* u, double* gnum, hipStream_t s);
hipError_t launch_paw_u(const double* Pkq, int ldP, int mlo, int nm, const int32_t* proj_off, const int32_t* qoff,
                        int natoms, int nproj, const double* Q, int NG, int NGp, double* Ur, double* Ui, hipStream_t s);
hipError_t launch_paw_adj(const double* gr, const double* gi, int NG, int NGp, const double* Yr, const double* Yi,
                          int nlo, const double* Ur, const double* Ui, int mlo, int nproj, const int32_t* pn,
                          const int32_t* pm, int npairs, double* Zm, double* Zn, hipStream_t s);
hipError_t launch_paw_reduce(const double* Z, const int32_t* start, const int32_t* list, int nb, int nproj, double* dP,
                             int band0, const double* gnum, const double* Pother, const int32_t* other,
                             const double* Dq, const int32_t* proj_off, const int32_t* qoff, int natoms, int side,
                             hipStream_t s);
hipError_t launch_eps_reduce(const double* u, const int32_t* start, const int32_t* list, int nbands, double sign,
                             double* de, hipStream_t s);
hipError_t launch_optical_c(const double* gnum, const int32_t* start, const int32_t* list, const int32_t* other,
                            const double* Cother, int nQ, const double* wq, int side, int nb, double* dC,
                            hipStream_t s);
hipError_t launch_zadj(const double* gr, const double* gi, int NGp, int npairs, const PairGeom& g,
                       const int32_t* col_start, const int32_t* col_g, const int32_t* col_kz, const cplx<double>* tw3,
                       cplx<double>* tadj, hipStream_t s);
hipError_t launch_xyadj(const cplx<double>* tadj, const PairGeom& g, const int32_t* start, const int32_t* list,
                        const int32_t* other, const cplx<double>* phio, int band0, int nb, int side,
                        const int32_t* kx, const int32_t* ky, const cplx<double>* tw1, const cplx<double>* tw2,
                        cplx<double>* phibar, hipStream_t s);
// Register form of the x-y adjoint for square grids of a register length divisible by 4 (FP64): seg holds
// per segment (owner, first, end into list, slot); owners with several segments write partial
// [slot][N3][N1 N2], which launch_xyadj_reduce adds into phibar (own[j]: such an owner, its slots
// [ostart[j], ostart[j + 1])).
bool xyadj_reg_supported(const PairGeom& g);
hipError_t launch_xyadj_reg(const cplx<double>* tadj, const PairGeom& g, const int32_t* seg, int nseg,
                            const int32_t* list, const int32_t* other, const cplx<double>* phio, int band0, int side,
                            cplx<double>* phibar, cplx<double>* partial, hipStream_t s);
hipError_t launch_xyadj_reduce(const cplx<double>* partial, size_t vol, const int32_t* own, const int32_t* ostart,
                               int nown, int band0, cplx<double>* phibar, hipStream_t s);
hipError_t launch_gather_c(const cplx<double>* ph, size_t vol, const int32_t* map, int nQ, int nb, double* dC,
                           hipStream_t s);
hipError_t launch_zero_d(double* p, size_t n, hipStream_t s);

}  // namespace rpa
