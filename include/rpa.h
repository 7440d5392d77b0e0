/*
 * rpa.h - C ABI of the MI355X (gfx950) library for the RPA correlation energy
 * in the projector augmented wave method: the non-interacting response
 * function chi0(q; G, G'; i w) and E_c(q).
 *
 * Method: J. Yan, L. Li, C. O'Grady, "Graphics Processing Unit Acceleration
 * of the Random Phase Approximation in the Projector Augmented Wave Method",
 * arXiv 1307.8052. Equation names below are that paper's labels.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Hartree atomic units. Cell rows A[i] are the lattice vectors a_i (bohr);
 *    reciprocal rows b_j satisfy a_i . b_j = 2 pi delta_ij; a Miller triple m
 *    is G = m1 b1 + m2 b2 + m3 b3 and sits at grid position m mod N.
 *  - complex128 arrays are interleaved (re, im) doubles, row-major.
 *  - Pointers marked DEVICE are caller-owned device memory on the context's
 *    device; pointers marked HOST are caller-owned host memory read during
 *    the call only. The library never frees or keeps caller pointers.
 *  - `stream` is a hipStream_t (NULL = the default stream). Device work is
 *    stream-ordered and asynchronous; host arrays are consumed before return.
 *  - Every call validates on the host before any launch and returns an
 *    rpa_status; nothing aborts or throws across the ABI. A failed kernel
 *    launch or an earlier asynchronous fault is reported as RPA_ERR_HIP.
 *    rpa_last_error() gives a per-thread detail string for the last failure.
 *  - Calls on one context are not re-entrant: one host thread at a time. All
 *    calls on a context share its device workspaces, so calls issued on
 *    different streams must be ordered by the caller (e.g. with events).
 */
#ifndef RPA_MI355X_H
#define RPA_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rpa_ctx rpa_ctx;

typedef enum {
    RPA_OK = 0,
    RPA_ERR_INPUT = -1,       /* bad value: NULL pointer, non-monotone eps/f, q+G = 0 off the optical limit */
    RPA_ERR_SHAPE = -2,       /* inconsistent sizes (bands, projector offsets, Miller ranges) */
    RPA_ERR_ALIAS = -3,       /* grid too small for an alias-free pair product on the G-sphere */
    RPA_ERR_NOMEM = -4,       /* device allocation failed or workspace cap below the minimum */
    RPA_ERR_NOT_PD = -5,      /* 1 - v^1/2 chi0 v^1/2 not positive definite at some frequency */
    RPA_ERR_HIP = -6,         /* HIP runtime error */
    RPA_ERR_UNSUPPORTED = -7  /* grid length not a product of 2, 3, 5 or too large for LDS staging */
} rpa_status;

typedef enum {
    RPA_FP64 = 0,        /* FP64 FFTs, FP64 MFMA rank-k update */
    RPA_SPLIT_BF16 = 1,  /* FP32 FFTs; rank-k update on BF16 MFMA with hi/lo split, FP32 accumulate */
    RPA_SPLIT_FP16 = 2   /* FP32 FFTs; rank-k update on FP16 MFMA with hi/lo split, FP32 accumulate */
} rpa_precision;

/* Unit cell and FFT grid. n[i] is the number of grid points along a_i; each
 * must be >= 2 and a product of the primes 2, 3 and 5. */
typedef struct {
    double A[3][3];
    int n[3];
} rpa_cell;

/* One state set at k (or at k+q) - Eq. get_wfs and Eq. n_G_2.
 *  C        DEVICE complex128 [nbands][nQ]: plane-wave coefficients C_n(Q) of the
 *           periodic part; psi~_n(r) = e^{ik.r} sum_Q C_n(Q) e^{i G_Q.r}, no
 *           1/sqrt(Omega). The states are expected orthonormal in the PAW sense
 *           (Sec. 2.2: sum_Q C_n^* C_m + sum_a sum_ij conj(P_ni) S^a_ij P_mj =
 *           delta_nm with S^a_ij = Q^a_ij(0)); the library does not check it.
 *  miller   HOST int32 [nQ][3]: Miller index of each Q; every |m_i| < n[i]/2.
 *  eps      HOST [nbands]: Kohn-Sham eigenvalues (Ha), ascending.
 *  f        HOST [nbands]: occupations in [0, 2] (spin included), non-increasing.
 *  proj_off HOST int32 [natoms+1]: projector offsets; atom a owns columns
 *           proj_off[a] .. proj_off[a+1]-1 of P.
 *  P        DEVICE complex128 [nbands][proj_off[natoms]]: P^a_ni = <p~^a_i|psi~_n>.
 *  kpt      Cartesian k (bohr^-1); enters only the optical-limit momentum.
 *  weight   Brillouin-zone weight w_k of this k-point (1/N_k).
 *  dfde     HOST [nbands] -df/d eps >= 0 of every band (partially occupied,
 *           e.g. Fermi-smeared, bands), or NULL. When set, an optical q-point
 *           gets the intraband (n = m) head of chi0 at q -> 0:
 *             chi0_00(i w) += -(1/Omega) w_k sum_n (-df/de)_n (qhat.v_n)^2 / w^2,
 *           with the band velocity qhat.v_n the n = m element of Eq. n_q0's
 *           numerator (momentum plus the PAW nabla term of Eq. nabla).
 *           Not supported by rpa_ec_backward (RPA_ERR_UNSUPPORTED).
 *  sym      HOST pointer to a symmetry operation (rpa_symop), or NULL. When
 *           set, C, miller, P, eps, f and dfde are those of a k-point k1 of the
 *           irreducible zone, and the set used is the one unfolded to
 *           kpt = (-1)^s T k1 + G0 (weight: that of kpt). Not supported by
 *           rpa_ec_backward (RPA_ERR_UNSUPPORTED).
 * A spin-polarised system is passed as one state set per spin channel
 * (occupations in [0, 1]); chi0 is their sum (the spin index of Eq. chi0). */
typedef struct rpa_symop rpa_symop;
typedef struct {
    int nbands;
    int nQ;
    const int32_t* miller;
    const void* C;
    const double* eps;
    const double* f;
    int natoms;
    const int32_t* proj_off;
    const void* P;
    double kpt[3];
    double weight;
    const double* dfde;
    const rpa_symop* sym;
} rpa_states;

/* A point operation of the crystal carrying a state set of the irreducible
 * zone at k1 to k = (-1)^s T k1 + G0 of the full zone - Eq. kmap, Eq.
 * trans_wfs (psi_nk(r) = psi_nk1(T^-1 r), complex conjugated with time
 * reversal) and Table 1 steps 4 and 7 (projections at k from rotated
 * projector functions).
 *  rot           U, integer, det +-1: T maps fractional real-space
 *                coordinates x -> U x (r = sum_i x_i a_i); the Cartesian
 *                matrix A^T U A^-T must be orthogonal (RPA_ERR_INPUT).
 *  time_reversal s: 1 = the states are also complex conjugated.
 *  gshift        G0 in Miller units (reduces k to the caller's zone).
 *  kibz          Cartesian k1 (the Bloch phase of atoms mapped across a
 *                lattice vector).
 *  atom_map      HOST int32 [natoms]: b(a), the atom with T^-1 R_a = R_b + L_a;
 *                atoms a and b carry the same number of projectors.
 *  atom_shift    HOST int32 [natoms][3]: L_a in lattice units.
 *  proj_rot      HOST double [sum_a Np_a^2]: D^a, row-major (i, j), the
 *                rotation of atom a's projector functions,
 *                p^a_i(T y) = sum_j D^a_ij p^a_j(y) (real projector
 *                functions). NULL allowed only when natoms = 0.
 * The library unfolds in reciprocal space: the periodic part is
 * u_k(r) = e^{-i G0.r} [conj] u_k1(T^-1 r), whose coefficient at Miller
 * (-1)^s U^-T m - g0 is C_k1(m) (conjugated with time reversal) - the grid
 * function that the remap r -> T^-1 r of the transformed orbital gives, with
 * no pass over the grid - and rotates the projections,
 *   P^a_k,i = e^{i k1.L_a} sum_j D^a_ij P^b_k1,j   (conjugated with time reversal).
 * The transformed Miller indices must fit the grid (RPA_ERR_ALIAS otherwise). */
struct rpa_symop {
    int32_t rot[3][3];
    int32_t time_reversal;
    int32_t gshift[3];
    double kibz[3];
    const int32_t* atom_map;
    const int32_t* atom_shift;
    const double* proj_rot;
};

/* One q-point - Eq. rpa_c, Eq. n_G_2, Eq. n_q0.
 *  q        Cartesian q (bohr^-1).
 *  optical  1: q -> 0 limit along qhat (q must be 0). Row G = 0 of every pair
 *           density is replaced by Eq. n_q0 and v^1/2 at G = 0 is sqrt(4 pi).
 *           Eq. n_q0 divides by eps_m - eps_n: a transition with equal
 *           eigenvalues is RPA_ERR_INPUT.
 *  NG, gmiller  HOST int32 [NG][3]: the G-sphere (any order; chi0 comes out in
 *           this order). rpa_gsphere() produces the canonical one.
 *  Qpaw     DEVICE complex128 [sum_a Np_a^2][NG]: Q^a_ij(q+G), row
 *           qoff_a + i*Np_a + j with qoff_a = sum_{b<a} Np_b^2.
 *  Dpaw     HOST double [3][sum_a Np_a^2]: PAW nabla correction D^a_ij
 *           (Eq. Q_q0) per Cartesian direction; read only when optical = 1.
 *  weight   w_q, used by rpa_ec_batched to form sum_q w_q E_c(q).          */
typedef struct {
    double q[3];
    int optical;
    double qhat[3];
    int NG;
    const int32_t* gmiller;
    const void* Qpaw;
    const double* Dpaw;
    double weight;
} rpa_qspec;

/* Imaginary-frequency quadrature (HOST): nodes omega[nw] > 0 and weights of
 * d omega, so that E_c(q) = sum_i weight_i F(omega_i) / 2 pi (Eq. rpa). */
typedef struct {
    int nw;
    const double* omega;
    const double* weight;
} rpa_freq;

/* Create a context on HIP device `device` for one cell and grid. The context
 * owns device workspaces (grown on demand up to workspace_cap_bytes; 0 means
 * no cap) and caches. Errors: RPA_ERR_INPUT (NULL out or cell),
 * RPA_ERR_UNSUPPORTED (grid), RPA_ERR_HIP. */
int rpa_create(rpa_ctx** out, const rpa_cell* cell, int device, size_t workspace_cap_bytes);

/* Release every resource of the context (after synchronizing its device). */
int rpa_destroy(rpa_ctx* ctx);

/* The chi G-sphere {G : |q+G|^2/2 <= ecut} (Sec. 2.1), ordered by |q+G|^2,
 * then (m1, m2, m3) lexicographically. Host only. Writes up to `capacity`
 * triples to miller_out (HOST int32 [capacity][3], may be NULL) and the
 * count to *ng_out; RPA_ERR_SHAPE if capacity is too small (count still set). */
int rpa_gsphere(const rpa_cell* cell, const double q[3], double ecut, int32_t* miller_out,
                int capacity, int* ng_out);

/* Pair densities rho_nm(q+G) (Eq. n_G_2 with Eq. fft; Eq. n_q0 row when
 * optical) for an explicit pair list: n from set k, m from set kq.
 *  pair_n, pair_m HOST int32 [npairs].
 *  rho_out DEVICE complex128 [npairs][NG].
 * Computed in the precision's FFT type (FP64 or FP32) and widened. */
int rpa_pair_density(rpa_ctx* ctx, const rpa_states* k, const rpa_states* kq, const rpa_qspec* qs,
                     int npairs, const int32_t* pair_n, const int32_t* pair_m, rpa_precision prec,
                     void* rho_out, void* stream);

/* chi0_GG'(q, i w) of Eq. chi0 summed over nk (k, k+q) state-set pairs, grouped
 * as in Eq. zher_multi: pairs (n, m) with f_n - f_m > 1e-8 carry the real
 * weight a_nm(w) = (w_k/Omega)(f_n - f_m) 2 (e_n - e_m)/(w^2 + (e_n - e_m)^2)
 * (resonant and anti-resonant terms of each transition paired).
 *  k, kq    HOST arrays of nk state sets (kq[i] may equal k[i]).
 *  chi0_out DEVICE complex128 [nw][NG][NG], full Hermitian, gmiller order. */
int rpa_chi0(rpa_ctx* ctx, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs,
             const rpa_freq* fr, rpa_precision prec, void* chi0_out, void* stream);

/* rpa_chi0, added into chi0_inout instead of overwriting it: the k sum of
 * Eq. chi0 over calls, e.g. one k-point (or one group of k-points) at a time
 * with only that group's orbitals resident. Same arguments and layout as
 * rpa_chi0; chi0_inout DEVICE complex128 [nw][NG][NG] must hold a full
 * Hermitian matrix per frequency (zeros before the first call). */
int rpa_chi0_add(rpa_ctx* ctx, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs,
                 const rpa_freq* fr, rpa_precision prec, void* chi0_inout, void* stream);

/* chi0_GG'(q, w + i eta) at real frequencies (Sec. 5: the response function
 * of TDDFT, GW and BSE), summed over nk state-set pairs as rpa_chi0: Eq. chi0
 * with i w -> w + i eta and the two orderings of each transition paired as on
 * the imaginary axis, so every pair carries the complex weight
 *   a_nm(w) = (w_k/Omega)(f_n - f_m)[1/(w + i eta + e_n - e_m) - 1/(w + i eta - e_n + e_m)]
 * (at w = 0, eta = w' this is the imaginary-axis weight at i w'). chi0(w) is
 * not Hermitian; it is computed as A_w + i B_w from two Hermitian grouped
 * updates with the real weights Re a and Im a. Optical q-points carry the
 * same head as rpa_chi0 (Eq. n_q0), and sets with dfde the intraband head
 * (1/Omega) w_k sum_n (-df/de)_n (qhat.v_n)^2 / (w + i eta)^2.
 *  omega    HOST [nw] real frequencies (Ha, any sign), 1 <= nw <= 256.
 *  eta      broadening (Ha), > 0.
 *  chi0_out DEVICE complex128 [nw][NG][NG] (full matrices, gmiller order).
 * RPA_ERR_INPUT for a bad frequency list or eta. */
int rpa_chi0_real(rpa_ctx* ctx, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs,
                  const double* omega, int nw, double eta, rpa_precision prec, void* chi0_out, void* stream);

/* E_c(q) from a given chi0 (Eq. rpa, Table 1 step 13):
 * F(w) = ln det(1 - K) + Tr K with K = v^1/2 chi0 v^1/2, v^1/2_G = sqrt(4 pi)/|q+G|,
 * ln det from an FP64 Cholesky factorisation; E_c = sum_i weight_i F(w_i)/2 pi.
 *  chi0   DEVICE complex128 [nw][NG][NG] (lower triangle read).
 *  ec_dev DEVICE double [1]; F_dev DEVICE double [nw] or NULL.
 * A non-positive pivot is reported on the next synchronizing call of this
 * context as RPA_ERR_NOT_PD via rpa_check(); the returned values are then NaN. */
int rpa_ec_from_chi0(rpa_ctx* ctx, const rpa_qspec* qs, const rpa_freq* fr, const void* chi0,
                     double* ec_dev, double* F_dev, void* stream);

/* chi0 then E_c(q) in one call, without materialising the output chi0. */
int rpa_ec(rpa_ctx* ctx, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs,
           const rpa_freq* fr, rpa_precision prec, double* ec_dev, double* F_dev, void* stream);

/* rpa_ec for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, kernels and results as rpa_ec, but every device workspace
 * (orbitals, pair transforms, pair densities, weights, PAW and split
 * operands, the chi0 accumulator, the Cholesky buffers and the uploaded host
 * tables) is carved out of one static device array of 128 MiB per GPU, set
 * up by rpa_create and held until the process ends. The call makes no
 * hipMalloc, hipFree, pinned-host or library allocation; host tables are
 * copied from ordinary host memory with hipMemcpyAsync.
 *  - A problem whose workspaces exceed 128 MiB is rejected with
 *    RPA_ERR_NOMEM before any kernel runs (rpa_last_error names the buffer
 *    and the bytes needed). Small spheres and band counts fit: e.g. NG ~ 120
 *    with 64 states on a 16^3 grid takes a few MiB, while NG ~ 1500 with 16
 *    frequencies needs 600 MiB for chi0 alone and does not.
 *  - Every call on a GPU shares that GPU's array, which keeps the last call's
 *    contents; the kernels clear what must start at zero. Calls that overlap
 *    on one GPU (different streams or host threads, any context) race: order
 *    them. rpa_check reports a non-positive pivot of the last call, as for
 *    rpa_ec, until another call on the same GPU reuses the array.
 *  - The stage profiler records nothing during this call. */
int rpa_ec_noalloc(rpa_ctx* ctx, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs,
                   const rpa_freq* fr, rpa_precision prec, double* ec_dev, double* F_dev, void* stream);

/* E_c(q) for nq q-points that share the same (k, k+q) state-set pairs (as with
 * Gamma-only sampling) - Eq. rpa_c's q sum. Orbitals are built once; each q
 * has its own G-sphere, PAW table and chi0. Outputs: ec_dev DEVICE double
 * [nq + 1] holds E_c(q_j) and, at index nq, sum_j w_qj E_c(q_j); F_dev DEVICE
 * double [nq][nw] or NULL.
 * use_graph = 1: the whole launch sequence is captured once into a hipGraph
 * (with buffers owned by that graph) and replayed by later calls whose host
 * inputs (sizes, Miller lists, eigenvalues, occupations, frequencies, q, PAW
 * nabla table) and device pointers are unchanged; device array contents may
 * change between replays. Replays must use the same stream; a call with other
 * inputs re-captures. */
int rpa_ec_batched(rpa_ctx* ctx, const rpa_states* k, const rpa_states* kq, int nk, int nq, const rpa_qspec* qs,
                   const rpa_freq* fr, rpa_precision prec, double* ec_dev, double* F_dev, int use_graph,
                   void* stream);

/* rpa_ec_batched with a (k, k+q) state-set list of its own for every q-point
 * (a k-mesh, where the k+q sets differ from q to q) - Eq. rpa_c's q sum over
 * Eq. chi0's k sum. q-point j uses k[j][0 .. nk[j]-1] and kq[j][0 .. nk[j]-1]
 * (HOST arrays of HOST pointers; the sets follow the rpa_states rules, and a
 * set listed under several q-points is read by each of them). Outputs, graph
 * capture and replay as for rpa_ec_batched (the per-q lists are part of the
 * replay key). The jobs of all q-points share one planning pass, one upload
 * and the batched factorisation of every (q, w) matrix. Errors: as
 * rpa_ec_batched; RPA_ERR_INPUT for nk[j] <= 0 or a NULL list. */
int rpa_ec_batched_sets(rpa_ctx* ctx, int nq, const rpa_states* const* k, const rpa_states* const* kq, const int* nk,
                        const rpa_qspec* qs, const rpa_freq* fr, rpa_precision prec, double* ec_dev, double* F_dev,
                        int use_graph, void* stream);

/* Gradient of E_c(q) (FP64 path) with respect to the inputs of nk (k, k+q)
 * state-set pairs (Eq. chi0's k sum): given the upstream derivative dEc
 * (DEVICE double [1], e.g. 1.0), writes for pair i, at the offset that is the
 * sum of the sizes of pairs 0 .. i-1,
 *  deps_k  DEVICE double [sum_i nbands_k_i]            dE/d eps_n at k_i
 *  dC_k    DEVICE complex128 [sum_i nbands_k_i nQ_k_i] dE/dRe C + i dE/dIm C
 *  dP_k    DEVICE complex128 [sum_i nbands_k_i nproj]  (may be NULL without PAW atoms)
 * and the same for the k+q sets (deps_kq, dC_kq, dP_kq, sized by the kq
 * sets; may be NULL when every kq[i] is the same set as k[i]). When kq[i] is
 * the same set as k[i] (same C, P and Miller pointers) both roles of pair i
 * are summed into its k slot and its kq slot is left untouched; a set listed
 * in several pairs gets one gradient per listing (their sum is its total).
 * Occupations are held fixed; C and P are free variables (no
 * re-orthonormalisation). E_c(q) is written to ec_dev.
 * chi0 of all pairs, its Cholesky factor and W(w) = v^1/2 [(1 - K)^-1 - 1]
 * v^1/2 are formed once; then every pair's densities are recomputed chunk by
 * chunk and rho_bar = sum_w c_w 2 a(w) W(w) rho is taken back through the
 * optical row, the PAW term, the pruned pair FFT and the orbital FFT.
 * RPA_ERR_UNSUPPORTED if N1*N2 > 4096, for more than 64 frequencies, for sets
 * with -df/de at an optical q-point and for sets with a symmetry operation. */
int rpa_ec_backward(rpa_ctx* ctx, const rpa_states* k, const rpa_states* kq, int nk, const rpa_qspec* qs,
                    const rpa_freq* fr, const double* dEc, double* ec_dev, double* deps_k, void* dC_k, void* dP_k,
                    double* deps_kq, void* dC_kq, void* dP_kq, void* stream);

/* Rank-k kernel choice of the split precisions per padded sphere size
 * (NG rounded up to 64):
 *   1 = 64x64 tiles staged from FP32 rho, FP32 partial sums added into FP64
 *       every 8 K-steps;
 *   4 = pipelined 64x128 tiles from the K-blocked pre-split rho, FP32 partial
 *       sums added into FP64 every 8 K-steps;
 *   5 = variant 4 with eight waves per workgroup, two per SIMD (bit-identical
 *       to 4).
 * Without an entry, NG >= 385 uses variant 5, smaller spheres variant 1
 * (rpa_set_autotune: calls record an entry per size bucket).
 *  rpa_autotune     times the variants on synthetic operands of the given
 *                   shape on `stream` (synchronizes) and records the fastest.
 *  rpa_tune_set/get force / read the choice (FP64 has variant 0 only;
 *                   RPA_ERR_INPUT for another variant).
 *  rpa_tune_cache_io saves (save = 1) or loads a text table at `path`. */
int rpa_autotune(rpa_ctx* ctx, rpa_precision prec, int NG, int npairs, int nw, void* stream);

/* Grid-transform kernels (Eq. get_wfs, Eq. fft) for this context: path 0
 * (default) runs register-resident lines along z when N3 is one of the
 * compiled line lengths (8, 10, 12, 16, 20, 24, 32, 40, 48, and 64 in the split
 * precisions), and along x and y when N1 == N2 is one of them, and LDS radix
 * passes for the other axes (a 40 x 40 x 160 grid runs x and y in registers and
 * z through LDS); path 1 always runs the LDS radix passes. Both give the same
 * result up to rounding order. RPA_ERR_INPUT for another value. */
int rpa_set_pair_path(rpa_ctx* ctx, int path);

/* Split precisions: with enable = 1 (the default) the first call whose
 * sphere falls in a new size bucket (NG padded to 64, rounded up to 128 up
 * to 2048 and to 256 beyond) times the rank-k variants on synthetic operands
 * of that bucket (one chunk of the call's pairs, its frequencies; the call
 * synchronizes its stream once) and records the fastest for the bucket, as
 * rpa_autotune does. Not under graph capture and not in rpa_ec_noalloc, which
 * use the recorded or default variant. enable = 0 keeps the defaults and
 * rpa_tune_set choices. */
int rpa_set_autotune(rpa_ctx* ctx, int enable);

/* Upper bound on the pairs of one chunk (the K of one grouped rank-k update,
 * Eq. zher_multi's group). 0 (default): the chunk is as large as the workspace
 * budget allows (up to 6 GiB of per-chunk buffers, a quarter of the cap when
 * one is set). A smaller bound lowers the per-chunk memory and splits a
 * q-point's sum into more updates; chi0 is the same up to rounding order.
 * RPA_ERR_INPUT if max_pairs < 0. */
int rpa_set_chunk_pairs(rpa_ctx* ctx, int max_pairs);

/* The PAW correction (Eq. n_G_2) runs on MFMA in one of two factorised forms:
 * per band n (Y_n = conj(P_n) Q, then rho_p += P'_m . Y_n for the pairs of
 * each n), chosen by default where the pairs span fewer bands n than bands m
 * and Y fits 2 GiB (an eighth of the cap when one is set), or per band m
 * (Z_m = Q P'_m, then rho_p += conj(P_n) . Z_m), in passes over consecutive
 * pairs whose bands m fit a Z buffer of that size. max_bands > 0 selects the
 * per-m form with at most max_bands bands m per pass; 0 (default) restores
 * the automatic choice. Pair densities of one form do not depend on the
 * bound or the chunking; the two forms agree to rounding.
 * RPA_ERR_INPUT if max_bands < 0. */
int rpa_set_paw_window(rpa_ctx* ctx, int max_bands);
int rpa_tune_set(rpa_ctx* ctx, rpa_precision prec, int NG, int variant);
int rpa_tune_get(rpa_ctx* ctx, rpa_precision prec, int NG, int* variant);
int rpa_tune_cache_io(rpa_ctx* ctx, const char* path, int save);

/* Synchronize `stream` and report device-side failures of earlier calls on
 * this context (RPA_ERR_NOT_PD with the frequency index in rpa_last_error). */
int rpa_check(rpa_ctx* ctx, void* stream);

/* Stage profiler. rpa_profile(ctx, 1) clears the totals and starts recording a
 * pair of HIP events on the launch stream around every kernel group of the
 * calls that follow (0 stops). rpa_profile_get() synchronizes on the recorded
 * events and returns the summed elapsed milliseconds and the number of timed
 * groups of one stage: "orbitals", "pair_xy", "pair_z_gather", "paw",
 * "optical", "weights", "split_pack" (the split precisions' hi/lo packing and
 * FP16 scales ahead of each rank-k update), "herk" (the rank-k update kernel of
 * chi0 alone, one launch per pair chunk and frequency set), "cholesky" (the
 * whole E_c stage), and for rpa_ec_backward "adjoint_inverse" ((1 - K)^-1 from
 * the Cholesky factor and W(omega)), "adjoint_gemm" (the products W(omega) rho
 * of a pair chunk: one batched launch for all frequencies where their products
 * fit 8 GiB and NG <= 4096, else one per frequency), "adjoint_pairs" (the z and x-y adjoint
 * transforms with the orbital products) or "adjoint_rest" (weights, energies,
 * PAW and optical adjoints, the coefficient transforms).
 * RPA_ERR_INPUT for an unknown stage name. */
int rpa_profile(rpa_ctx* ctx, int enable);
int rpa_profile_get(rpa_ctx* ctx, const char* stage, double* ms, long long* launches);

/* Static text for a status code. */
const char* rpa_status_string(int status);

/* Detail of the last failure on the calling thread (never NULL). */
const char* rpa_last_error(const rpa_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RPA_MI355X_H */
