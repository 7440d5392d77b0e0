"""FP64 reference implementation of the chi0 / E_c path, step by step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings taken where the paper is silent or ambiguous
----------------------------------------------------
R1  Units: Hartree atomic units. Omega = |det A|.
R2  chi G-sphere (Sec. 2.1, text after Eq. rpa_c; Table 1 step 6):
    S_q = {G : |q+G|^2/2 <= Ecut}; ordered by |q+G|^2, then (m1, m2, m3)
    lexicographically. E_c does not depend on the order.
R3  Orbitals (Eq. get_wfs): periodic parts phi_n(r) = sum_Q C_n(Q) e^{i G_Q.r}
    with no 1/sqrt(Omega); the coefficients are orthonormal, so that
    <psi_n|psi_n'> = delta at q = 0, G = 0 (Sec. 2.2, optical-limit text) and
    Omega cancels from the pair density.
R4  Pair density by FFT (Eq. fft, Eq. n_G): the Bloch phases e^{-ik.r},
    e^{i(k+q).r} and e^{-iq.r} cancel, so
    n~_nm(G) = (1/N) sum_j conj(phi_n(r_j)) phi'_m(r_j) e^{-i G.r_j},
    i.e. numpy's forward fftn divided by the number of grid points.
R5  k+q states: the caller passes the k and k+q state sets explicitly; with a
    single Gamma point both are the same set.
R6  PAW term (Eq. n_G_2): <psi~_n|p~_i> = conj(P_ni); Q is a dense table
    [sum_a Np_a^2][NG] with row off_a + i*Np_a + j.
R7  Weights (Eq. chi0, Eq. A_iw): occupations f in [0, 2] include spin; the
    resonant and anti-resonant orderings of each transition are paired (time
    reversal), which turns (f_n - f_m)/(i w + e_n - e_m) into its real part
    times 2, so ZHER/ZHERK see real weights:
        a_nm(w) = (w_k/Omega) (f_n - f_m) 2 (e_n - e_m) / (w^2 + (e_n - e_m)^2),
    over the pairs with f_n - f_m > delta_f (delta_f = 1e-8). Every a <= 0.
R8  Brillouin-zone sum (Eq. chi0) carries w_k (1/N_k); the q sum (Eq. rpa_c)
    carries w_q with sum w_q = 1.
R9  Coulomb (Sec. 2.2): v_G(q) = 4 pi/|q+G|^2; K = v^1/2 chi0 v^1/2, which has
    the same determinant as 1 - v chi0.
R10 Optical limit (Eq. n_q0, Eq. nabla, Eq. Q_q0): at q = 0 the G = 0 element
    of every pair density is replaced by
        [sum_Q C_n^*(Q) C_m(Q) qhat.(k+G_Q) - i qhat.sum_a sum_ij conj(P_ni) D^a_ij P_mj] / (e_m - e_n)
    and v^1/2 at G = 0 is sqrt(4 pi) (the |q| of v and of n cancel). The
    pseudo part uses the exact plane-wave momentum (the paper's GPU form).
R11 Frequency grid (Sec. 2.1): Gauss-Legendre nodes t on [-1, 1],
    x = (t+1)/2, w = w0 x/(1-x), d w = w0/(1-x)^2 dx, w0 = 1 Ha.
R12 Spin (Sec. 2.2: the spin index is implicit in Eq. chi0): a spin-polarised
    system is passed as one state set per spin channel, occupations in [0, 1];
    chi0 is the sum over the sets.
R14 Real frequencies (Sec. 5: chi0 on the real axis for TDDFT, GW and BSE): Eq.
    chi0 with i w -> w + i eta, the two orderings of each transition paired as
    in R7:
        a_nm(w) = (w_k/Omega)(f_n - f_m)[1/(w + i eta + e_n - e_m) - 1/(w + i eta - (e_n - e_m))],
    complex, so chi0(w) = sum a rho rho^H is not Hermitian; at w = 0,
    eta = w' it is R7's weight at i w'. The intraband head of R13 becomes
    +(1/Omega) sum w_k (-df/de)(qhat.v)^2 / (w + i eta)^2.
R13 Intraband head at q -> 0 (the paper's systems are insulators or need no
    such term; for partially occupied bands the n = m terms of Eq. chi0 do not
    vanish as q -> 0): with -df/de of every band supplied, the head gets
        -(1/Omega) sum_sets w_k sum_n (-df/de)_n (qhat.v_n)^2 / w^2,
    qhat.v_n the diagonal of Eq. n_q0's numerator (the band velocity). This is
    the small-q limit of the n = m terms of Eq. chi0 summed over a
    time-reversal-symmetric k set (the imaginary O(q^2) part is a total
    derivative over the Brillouin zone and drops out).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

FOUR_PI = 4.0 * np.pi
TWO_PI = 2.0 * np.pi


# ---------------------------------------------------------------------------
# geometry (R1, R2)
# ---------------------------------------------------------------------------
def reciprocal_rows(A):
    """Rows b_i of the reciprocal lattice: a_i . b_j = 2 pi delta_ij."""
    return TWO_PI * np.linalg.inv(np.asarray(A, dtype=np.float64)).T


def cartesian(miller, B, shift=(0.0, 0.0, 0.0)):
    """shift + m1 b1 + m2 b2 + m3 b3, summed left to right per component."""
    m = np.asarray(miller, dtype=np.float64)
    out = np.empty(m.shape[:-1] + (3,))
    for c in range(3):
        out[..., c] = ((shift[c] + m[..., 0] * B[0, c]) + m[..., 1] * B[1, c]) + m[..., 2] * B[2, c]
    return out


def sq_norm(v):
    return (v[..., 0] * v[..., 0] + v[..., 1] * v[..., 1]) + v[..., 2] * v[..., 2]


def gsphere(A, q, ecut):
    """The chi sphere of Sec. 2.1: every G with |q+G|^2/2 <= ecut (R2).

    Brute force over a Miller box that provably contains the sphere.
    """
    A = np.asarray(A, dtype=np.float64)
    B = reciprocal_rows(A)
    gmax = np.sqrt(2.0 * ecut) + float(np.linalg.norm(q))
    # |m_i| = |(q+G).a_i - q.a_i| / 2pi <= (|q+G| + |q|) |a_i| / 2pi
    mmax = np.floor(gmax * np.linalg.norm(A, axis=1) / TWO_PI).astype(int) + 1
    axes = [np.arange(-M, M + 1) for M in mmax]
    m = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    k2 = sq_norm(cartesian(m, B, q))
    keep = 0.5 * k2 <= ecut
    m, k2 = m[keep], k2[keep]
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], k2))
    return np.ascontiguousarray(m[order].astype(np.int32))


def grid_index(miller, grid):
    """Grid position of a Miller index on an N-point axis: m mod N."""
    return tuple(np.mod(np.asarray(miller)[:, c], grid[c]) for c in range(3))


# ---------------------------------------------------------------------------
# orbitals (Eq. get_wfs, Table 1 step 3; R3)
# ---------------------------------------------------------------------------
def orbitals(C, miller, grid):
    """phi_n(r_j) = sum_Q C_n(Q) exp(i G_Q . r_j) on the grid r_j = sum_i (j_i/N_i) a_i.

    The sum over Q is an unnormalised inverse DFT: place C at m mod N, then
    N * ifftn. Returns complex128 [nb, N1, N2, N3].
    """
    C = np.asarray(C)
    nb = C.shape[0]
    box = np.zeros((nb,) + tuple(grid), dtype=np.complex128)
    i1, i2, i3 = grid_index(miller, grid)
    box[:, i1, i2, i3] = C
    ntot = grid[0] * grid[1] * grid[2]
    return sfft.ifftn(box, axes=(1, 2, 3), workers=-1) * ntot


# ---------------------------------------------------------------------------
# pair set and weights (Eq. chi0, Eq. A_iw; R7)
# ---------------------------------------------------------------------------
def pair_list(f_k, f_kq, delta_f=1e-8):
    """All (n, m) with f_n(k) - f_m(k+q) > delta_f, n-major then m ascending."""
    f_k = np.asarray(f_k)
    f_kq = np.asarray(f_kq)
    n_idx, m_idx = np.nonzero(f_k[:, None] - f_kq[None, :] > delta_f)
    return n_idx.astype(np.int64), m_idx.astype(np.int64)


def transition_weights_real(eps_k, eps_kq, f_k, f_kq, pairs, w_k, volume, omega, eta):
    """Complex weights at real frequencies (R14):
    a_nm(w) = (w_k/Omega)(f_n - f_m)[1/(w + i eta + e_n - e_m) - 1/(w + i eta - (e_n - e_m))]; [P, nw]."""
    n, m = pairs
    d = (np.asarray(eps_k)[n] - np.asarray(eps_kq)[m])[:, None]
    df = (np.asarray(f_k)[n] - np.asarray(f_kq)[m])[:, None]
    z = np.asarray(omega, dtype=np.float64)[None, :] + 1j * eta
    return (w_k / volume) * df * (1.0 / (z + d) - 1.0 / (z - d))


def transition_weights(eps_k, eps_kq, f_k, f_kq, pairs, w_k, volume, omega):
    """a_nm(w) = (w_k/Omega)(f_n - f_m) 2 (e_n - e_m)/(w^2 + (e_n - e_m)^2)  (R7); [P, nw]."""
    n, m = pairs
    d = np.asarray(eps_k)[n] - np.asarray(eps_kq)[m]
    df = np.asarray(f_k)[n] - np.asarray(f_kq)[m]
    w = np.asarray(omega)[None, :]
    return (w_k / volume) * df[:, None] * 2.0 * d[:, None] / (w * w + d[:, None] ** 2)


# ---------------------------------------------------------------------------
# pair densities (Eq. n_G, Eq. fft, Eq. n_G_2; Table 1 steps 5-9)
# ---------------------------------------------------------------------------
def pseudo_pair_density(phi_k, phi_kq, pairs, gmiller, grid, batch=64):
    """n~_nm(G) = fftn(conj(phi_n) phi'_m)[G] / N  (R4); complex128 [P, NG]."""
    n_idx, m_idx = pairs
    P = n_idx.size
    ntot = grid[0] * grid[1] * grid[2]
    i1, i2, i3 = grid_index(gmiller, grid)
    out = np.empty((P, len(gmiller)), dtype=np.complex128)
    for s in range(0, P, batch):
        e = min(P, s + batch)
        prod = np.conj(phi_k[n_idx[s:e]]) * phi_kq[m_idx[s:e]]
        spec = sfft.fftn(prod, axes=(1, 2, 3), workers=-1)
        out[s:e] = spec[:, i1, i2, i3] / ntot
    return out


def pseudo_pair_density_pw(C_k, miller_k, C_kq, miller_kq, pairs, gmiller):
    """Plane-wave convolution n~_nm(G) = sum_Q C_n^*(Q) C'_m(Q + G).

    Same quantity as :func:`pseudo_pair_density` whenever the grid is alias
    free; evaluated without any grid, one G at a time.
    """
    n_idx, m_idx = pairs
    lut = {tuple(v): i for i, v in enumerate(np.asarray(miller_kq).tolist())}
    out = np.zeros((n_idx.size, len(gmiller)), dtype=np.complex128)
    Ck = np.asarray(C_k)
    Ckq = np.asarray(C_kq)
    mk = np.asarray(miller_k)
    for g, G in enumerate(np.asarray(gmiller).tolist()):
        src, dst = [], []
        for iq, Q in enumerate(mk.tolist()):
            j = lut.get((Q[0] + G[0], Q[1] + G[1], Q[2] + G[2]))
            if j is not None:
                src.append(iq)
                dst.append(j)
        if not src:
            continue
        src = np.asarray(src)
        dst = np.asarray(dst)
        out[:, g] = np.einsum("pq,pq->p", np.conj(Ck[n_idx][:, src]), Ckq[m_idx][:, dst])
    return out


def paw_correction(P_k, P_kq, pairs, Qtab, offsets):
    """sum_a sum_ij conj(P^a_ni) P'^a_mj Q^a_ij(q+G), literally per atom (Eq. n_G_2; R6)."""
    n_idx, m_idx = pairs
    out = np.zeros((n_idx.size, Qtab.shape[1]), dtype=np.complex128)
    qoff = 0
    for a in range(len(offsets) - 1):
        lo, hi = offsets[a], offsets[a + 1]
        npj = hi - lo
        Qa = Qtab[qoff:qoff + npj * npj].reshape(npj, npj, -1)
        qoff += npj * npj
        Pn = np.conj(P_k[n_idx][:, lo:hi])
        Pm = P_kq[m_idx][:, lo:hi]
        out += np.einsum("pi,pj,ijg->pg", Pn, Pm, Qa)
    return out


def momentum_pw(C_k, miller_k, kpt, A, pairs, qhat):
    """qhat . sum_Q C_n^*(Q) C_m(Q) (k + G_Q): the plane-wave form of -i qhat.<psi~_n|nabla|psi~_m>."""
    n_idx, m_idx = pairs
    B = reciprocal_rows(A)
    kG = cartesian(miller_k, B, kpt)
    proj = kG @ np.asarray(qhat, dtype=np.float64)
    return np.einsum("pq,pq->p", np.conj(C_k[n_idx]) * proj[None, :], C_k[m_idx])


def optical_head(C_k, miller_k, kpt, A, P_k, Dtab, offsets, eps, pairs, qhat):
    """n_{q->0}(G=0) of Eq. n_q0 with Eq. nabla and Eq. Q_q0 (R10); [P] complex."""
    n_idx, m_idx = pairs
    pseudo = momentum_pw(C_k, miller_k, kpt, A, pairs, qhat)
    Dq = np.tensordot(np.asarray(qhat, dtype=np.float64), Dtab, axes=(0, 0))  # [sum Np^2]
    paw = np.zeros(n_idx.size, dtype=np.complex128)
    qoff = 0
    for a in range(len(offsets) - 1):
        lo, hi = offsets[a], offsets[a + 1]
        npj = hi - lo
        Da = Dq[qoff:qoff + npj * npj].reshape(npj, npj)
        qoff += npj * npj
        paw += np.einsum("pi,ij,pj->p", np.conj(P_k[n_idx][:, lo:hi]), Da, P_k[m_idx][:, lo:hi])
    de = np.asarray(eps)[m_idx] - np.asarray(eps)[n_idx]
    return (pseudo - 1j * paw) / de


def band_velocity(C_k, miller_k, kpt, A, P_k, Dtab, offsets, qhat):
    """qhat . v_n of every band: the n = m element of Eq. n_q0's numerator,
    sum_Q |C_n(Q)|^2 qhat.(k+G_Q) - i qhat.sum_a sum_ij conj(P_ni) D^a_ij P_nj (R13); real [nb]."""
    nb = np.asarray(C_k).shape[0]
    idx = np.arange(nb)
    pseudo = momentum_pw(C_k, miller_k, kpt, A, (idx, idx), qhat)
    paw = np.zeros(nb, dtype=np.complex128)
    if len(offsets) > 1:
        Dq = np.tensordot(np.asarray(qhat, dtype=np.float64), Dtab, axes=(0, 0))
        qoff = 0
        for a in range(len(offsets) - 1):
            lo, hi = offsets[a], offsets[a + 1]
            npj = hi - lo
            Da = Dq[qoff:qoff + npj * npj].reshape(npj, npj)
            qoff += npj * npj
            Pa = np.asarray(P_k)[:, lo:hi]
            paw += np.einsum("ni,ij,nj->n", np.conj(Pa), Da, Pa)
    return np.real(pseudo - 1j * paw)


def intraband_head(sets, A, Dtab, offsets, qhat, omega):
    """The intraband addition to chi0_00 at q -> 0 (R13):
    -(1/Omega) sum_sets w_k sum_n (-df/de)_n (qhat.v_n)^2 / w^2 over the sets that carry -df/de; [nw]."""
    volume = abs(np.linalg.det(A))
    s = 0.0
    for st in sets:
        mdf = getattr(st, "dfde", None)
        if mdf is None:
            continue
        v = band_velocity(st.C, st.miller, st.kpt, A, st.P, Dtab, offsets, qhat)
        s += st.weight * float(np.sum(np.asarray(mdf) * v * v))
    w = np.asarray(omega, dtype=np.float64)
    return -(s / volume) / (w * w)


# ---------------------------------------------------------------------------
# chi0 (Eq. zher, Eq. zher_multi; Table 1 step 11)
# ---------------------------------------------------------------------------
def chi0_rank1(rho, a):
    """chi0(w) = sum_p a_p(w) n_p n_p^H, one rank-1 update per pair (Eq. zher)."""
    P, NG = rho.shape
    nw = a.shape[1]
    chi = np.zeros((nw, NG, NG), dtype=np.complex128)
    for p in range(P):
        outer = np.outer(rho[p], np.conj(rho[p]))
        for w in range(nw):
            chi[w] += a[p, w] * outer
    return chi


def chi0_grouped(rho, a, group=None):
    """chi0(w) = sum over groups u of n(u) diag(a(u,w)) n(u)^H (Eq. zher_multi)."""
    P, NG = rho.shape
    nw = a.shape[1]
    group = P if group is None else group
    chi = np.zeros((nw, NG, NG), dtype=np.complex128)
    for s in range(0, P, group):
        X = rho[s:s + group]
        for w in range(nw):
            chi[w] += (X.T * a[s:s + group, w][None, :]) @ np.conj(X)
    return chi


# ---------------------------------------------------------------------------
# Coulomb and the integrand (Eq. rpa, Eq. rpa_c; R9)
# ---------------------------------------------------------------------------
def coulomb_sqrt(A, q, gmiller, optical=False):
    """v^1/2_G = sqrt(4 pi)/|q+G|; sqrt(4 pi) at G = 0 in the optical limit (R10)."""
    B = reciprocal_rows(A)
    k = np.sqrt(sq_norm(cartesian(gmiller, B, q)))
    out = np.empty_like(k)
    zero = k == 0.0
    if np.any(zero) and not optical:
        raise ValueError("q + G = 0 outside the optical limit")
    out[~zero] = np.sqrt(FOUR_PI) / k[~zero]
    out[zero] = np.sqrt(FOUR_PI)
    return out


def kernel_matrix(chi, vsqrt):
    return vsqrt[None, :, None] * chi * vsqrt[None, None, :]


def integrand(chi, vsqrt):
    """F(w) = Tr[ln(1 - K) + K] = sum_l [ln(1 - lambda_l) + lambda_l] over the eigenvalues
    lambda of K (Eq. rpa), with ln(1 - lambda) evaluated as log1p(-lambda) so that the
    cancellation against lambda at large w keeps absolute accuracy."""
    K = kernel_matrix(chi, vsqrt)
    F = np.empty(K.shape[0])
    for w in range(K.shape[0]):
        lam = np.linalg.eigvalsh(K[w])
        F[w] = np.sum(np.log1p(-lam) + lam)
    return F


integrand_eigen = integrand


def logdet_one_minus(K):
    """ln det(1 - K) for Hermitian K with 1 - K positive definite, by the textbook (unblocked,
    right-looking) Cholesky factorisation of 1 + A, A = -K, that never forms the identity: each pivot
    is 1 + A_jj and contributes log1p(A_jj) to the log-determinant."""
    A = -np.array(K, dtype=np.complex128, copy=True)
    n = A.shape[0]
    total = 0.0
    for j in range(n):
        d = float(np.real(A[j, j]))
        if not 1.0 + d > 0.0:
            raise np.linalg.LinAlgError(f"pivot {j} not positive")
        total += np.log1p(d)
        col = A[j + 1:, j] / np.sqrt(1.0 + d)
        A[j + 1:, j + 1:] -= np.outer(col, np.conj(col))
    return total


def integrand_cholesky(chi, vsqrt):
    """F(w) = ln det(1 - K) + Tr K with ln det from the Cholesky factor of 1 - K."""
    K = kernel_matrix(chi, vsqrt)
    F = np.empty(K.shape[0])
    for w in range(K.shape[0]):
        F[w] = logdet_one_minus(K[w]) + float(np.real(np.trace(K[w])))
    return F


def integrand_slogdet(chi, vsqrt):
    K = kernel_matrix(chi, vsqrt)
    NG = K.shape[1]
    F = np.empty(K.shape[0])
    for w in range(K.shape[0]):
        sign, ld = np.linalg.slogdet(np.eye(NG) - K[w])
        F[w] = ld + np.real(np.trace(K[w]))
    return F


def ec_from_integrand(F, omega_weight):
    """E_c(q) = int_0^inf dw/2pi F(w) ~= sum_i W_i F(w_i) / 2pi (Eq. rpa)."""
    return float(np.dot(np.asarray(omega_weight), np.asarray(F)) / TWO_PI)


# ---------------------------------------------------------------------------
# quadrature (Sec. 2.1; R11)
# ---------------------------------------------------------------------------
def gauss_legendre(n):
    """Gauss-Legendre nodes and weights on [-1, 1] by Golub-Welsch (eigen-decomposition
    of the Jacobi matrix of the Legendre recurrence)."""
    k = np.arange(1, n)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    J = np.diag(beta, 1) + np.diag(beta, -1)
    t, V = np.linalg.eigh(J)
    w = 2.0 * V[0, :] ** 2
    return t, w


def frequency_grid(n, w0=1.0):
    t, w = gauss_legendre(n)
    x = 0.5 * (t + 1.0)
    return w0 * x / (1.0 - x), 0.5 * w * w0 / (1.0 - x) ** 2


# ---------------------------------------------------------------------------
# end to end for one q (Table 1 steps 3-13)
# ---------------------------------------------------------------------------
def pair_densities(A, grid, sk, skq, gmiller, Qtab, offsets, optical=False, qhat=None,
                   Dtab=None, delta_f=1e-8, phi=None):
    """rho_nm(q+G) for one (k, k+q) state set pair: steps 3-10. Returns (pairs, rho)."""
    pairs = pair_list(sk.f, skq.f, delta_f)
    if phi is None:
        phi_k = orbitals(sk.C, sk.miller, grid)
        phi_kq = phi_k if skq is sk else orbitals(skq.C, skq.miller, grid)
    else:
        phi_k, phi_kq = phi
    rho = pseudo_pair_density(phi_k, phi_kq, pairs, gmiller, grid)
    rho += paw_correction(sk.P, skq.P, pairs, Qtab, offsets)
    if optical:
        zero = np.nonzero(np.all(np.asarray(gmiller) == 0, axis=1))[0]
        if zero.size:
            rho[:, zero[0]] = optical_head(sk.C, sk.miller, sk.kpt, A, sk.P, Dtab, offsets,
                                           sk.eps, pairs, qhat)
    return pairs, rho


def chi0_q(A, grid, ksets, kqsets, gmiller, Qtab, offsets, omega, optical=False, qhat=None,
           Dtab=None, delta_f=1e-8):
    """chi0(q, i w) summed over k (Eq. chi0); complex128 [nw, NG, NG]."""
    volume = abs(np.linalg.det(A))
    chi = np.zeros((len(omega), len(gmiller), len(gmiller)), dtype=np.complex128)
    for sk, skq in zip(ksets, kqsets):
        pairs, rho = pair_densities(A, grid, sk, skq, gmiller, Qtab, offsets, optical, qhat,
                                    Dtab, delta_f)
        a = transition_weights(sk.eps, skq.eps, sk.f, skq.f, pairs, sk.weight, volume, omega)
        chi += chi0_grouped(rho, a)
    if optical and any(getattr(s, "dfde", None) is not None for s in ksets):
        zero = np.nonzero(np.all(np.asarray(gmiller) == 0, axis=1))[0]
        if zero.size:
            chi[:, zero[0], zero[0]] += intraband_head(ksets, A, Dtab, offsets, qhat, omega)
    return chi


def chi0_q_real(A, grid, ksets, kqsets, gmiller, Qtab, offsets, omega, eta, optical=False, qhat=None,
                Dtab=None, delta_f=1e-8):
    """chi0(q, w + i eta) at real frequencies (R14), summed over k; complex128 [nw, NG, NG], not Hermitian."""
    volume = abs(np.linalg.det(A))
    chi = np.zeros((len(omega), len(gmiller), len(gmiller)), dtype=np.complex128)
    for sk, skq in zip(ksets, kqsets):
        pairs, rho = pair_densities(A, grid, sk, skq, gmiller, Qtab, offsets, optical, qhat,
                                    Dtab, delta_f)
        a = transition_weights_real(sk.eps, skq.eps, sk.f, skq.f, pairs, sk.weight, volume, omega, eta)
        for w in range(len(omega)):
            chi[w] += (rho.T * a[:, w][None, :]) @ np.conj(rho)
    if optical and any(getattr(s, "dfde", None) is not None for s in ksets):
        zero = np.nonzero(np.all(np.asarray(gmiller) == 0, axis=1))[0]
        if zero.size:
            # R13's -s/w^2 on the imaginary axis is s/(i w)^2; at w + i eta it is s/(w + i eta)^2
            s_over = -intraband_head(ksets, A, Dtab, offsets, qhat, np.ones(1))[0]
            z = np.asarray(omega, dtype=np.float64) + 1j * eta
            chi[:, zero[0], zero[0]] += s_over / (z * z)
    return chi


def ec_q(A, grid, ksets, kqsets, gmiller, Qtab, offsets, q, omega, omega_weight,
         optical=False, qhat=None, Dtab=None, delta_f=1e-8):
    """E_c(q) and F(w) (Eq. rpa, Table 1 step 13)."""
    chi = chi0_q(A, grid, ksets, kqsets, gmiller, Qtab, offsets, omega, optical, qhat, Dtab,
                 delta_f)
    vs = coulomb_sqrt(A, q, gmiller, optical)
    F = integrand(chi, vs)
    return ec_from_integrand(F, omega_weight), F, chi


def two_level_ec(delta, b):
    """Closed form of int_0^inf dw/2pi [ln(1 + c) - c], c = b delta/(w^2 + delta^2):
    (1/2)[sqrt(delta^2 + b delta) - delta - b/2], written without the cancellation of its three terms
    at small b/delta: with x = b/delta, sqrt(1+x) - 1 - x/2 = -(x^2/4)/(sqrt(1+x) + 1 + x/2)."""
    x = b / delta
    return -0.125 * delta * x * x / (np.sqrt(1.0 + x) + 1.0 + 0.5 * x)
