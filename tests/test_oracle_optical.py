"""Pins of the oracle's optical-limit head (Eq. n_q0 with Eq. nabla) against a model where the
q -> 0 limit of the pair density can be taken directly.

Model: a local-potential Hamiltonian on a fixed plane-wave basis at Gamma,
    H_GG'(k) = |k+G|^2/2 delta_GG' + V(G - G'),  V(-G) = V(G)^*  (V real in space).
Its eigenvectors at k and k+q, with the phases of the k+q states fixed by parallel transport, give the
G = 0 pair density <u_nk|u_m,k+q> directly; divided by |q| it tends to the head of Eq. n_q0 (first-order
k.p perturbation theory: d_k H = k + G in this basis). A central difference in q makes the error O(|q|^2).

PAW part: an exact toy of the PAW transformation in the same basis. With projector functions p~_i, their
duals phi~_i (<phi~_i|p~_k> = delta_ik) and augmentation functions chi_j chosen so that d/dx chi_j lies in the
span of the projectors, the all-electron states psi = psi~ + sum_j chi_j <p~_j|psi~> satisfy
    <psi_n|d/dx|psi_m> = <psi~_n|d/dx|psi~_m> + sum_ij conj(P_ni) D_ij P_mj,
    D_ij = <phi_i|d/dx|phi_j> - <phi~_i|d/dx|phi~_j>,  phi_i = phi~_i + chi_i,
which is Eq. nabla's decomposition with no completeness error. Taking the all-electron states as the
eigenvectors of the model Hamiltonian, the head computed from the pseudo coefficients, P and D must equal
the all-electron head, which the k.p pin ties to the pair density itself. All functions are real in space,
so D is real antisymmetric, as the library's table expects.
"""
import numpy as np
import pytest

import oracle
import synth


def _basis(L=5.0, ecut=6.0):
    A = np.diag([L, L * 1.1, L * 1.2])
    miller = synth.wavefunction_sphere(A, np.zeros(3), ecut)
    return A, miller


def _potential(rng, A, miller, strength=0.6):
    """V(G - G') with V(-G) = conj(V(G)): a real local potential, smooth in G."""
    B = oracle.reciprocal_rows(A)
    diff = miller[:, None, :] - miller[None, :, :]
    keys = {}
    NQ = len(miller)
    V = np.zeros((NQ, NQ), dtype=np.complex128)
    for i in range(NQ):
        for j in range(NQ):
            d = tuple(diff[i, j])
            if d == (0, 0, 0):
                continue
            if d not in keys:
                neg = (-d[0], -d[1], -d[2])
                if neg in keys:
                    keys[d] = np.conj(keys[neg])
                else:
                    g = oracle.cartesian(np.array([d]), B)[0]
                    amp = strength * np.exp(-0.25 * float(g @ g))
                    keys[d] = amp * (rng.standard_normal() + 1j * rng.standard_normal())
            V[i, j] = keys[d]
    return V


def _eig(A, miller, V, k):
    B = oracle.reciprocal_rows(A)
    kg = oracle.cartesian(miller, B, k)
    H = np.diag(0.5 * oracle.sq_norm(kg)).astype(np.complex128) + V
    e, U = np.linalg.eigh(H)
    return e, U.T.copy()          # rows = states


def _transported(U0, U1):
    """Phases of the rows of U1 so that <u_m(k)|u_m(k+q)> is real and positive."""
    ov = np.einsum("mq,mq->m", np.conj(U0), U1)
    return U1 * (np.abs(ov) / ov)[:, None]


def _kp_head(A, miller, V, qhat, nb, t=1e-4):
    """lim_{q->0} <u_nk|u_m,k+q>/|q| along qhat by a central difference, for the nb lowest states."""
    k0 = np.zeros(3)
    e0, U0 = _eig(A, miller, V, k0)
    _, Up = _eig(A, miller, V, k0 + t * qhat)
    _, Um = _eig(A, miller, V, k0 - t * qhat)
    Up = _transported(U0, Up)[:nb]
    Um = _transported(U0, Um)[:nb]
    Mp = np.conj(U0[:nb]) @ Up.T
    Mm = np.conj(U0[:nb]) @ Um.T
    return (Mp - Mm) / (2 * t), e0[:nb], U0[:nb]


def _pairs(nb):
    n = np.array([i for i in range(nb) for j in range(nb) if i != j])
    m = np.array([j for i in range(nb) for j in range(nb) if i != j])
    return n, m


def test_pseudo_head_is_the_kp_limit_of_the_pair_density():
    """No projectors: the head of Eq. n_q0 equals lim <u_nk|u_m,k+q>/|q| (conjugation, the momentum and the
    sign of the energy denominator are all fixed by this)."""
    rng = np.random.default_rng(21)
    A, miller = _basis()
    V = _potential(rng, A, miller)
    qhat = np.array([1.0, 0.0, 0.0])
    nb = 6
    dM, eps, C = _kp_head(A, miller, V, qhat, nb)
    assert np.min(np.diff(eps)) > 1e-3
    pairs = _pairs(nb)
    empty = np.zeros((nb, 0), dtype=np.complex128)
    head = oracle.optical_head(C, miller, np.zeros(3), A, empty, np.zeros((3, 0)), np.array([0]), eps, pairs, qhat)
    ref = dM[pairs]
    assert np.max(np.abs(ref)) > 1e-2
    assert np.max(np.abs(head - ref)) < 1e-6 * np.max(np.abs(ref))


def _paw_toy(rng, A, miller, nproj, scale=0.8):
    """Real-space-real projector, dual and augmentation functions (coefficient columns) on the basis."""
    B = oracle.reciprocal_rows(A)
    G = oracle.cartesian(miller, B)
    gx = G[:, 0]
    index = {tuple(m): i for i, m in enumerate(miller.tolist())}
    neg = np.array([index[(-m[0], -m[1], -m[2])] for m in miller.tolist()])

    def real_fn(c):
        # f(-G) = conj(f(G)): a real function in space
        return 0.5 * (c + np.conj(c[neg]))

    env = np.exp(-0.15 * oracle.sq_norm(G))
    p = np.zeros((len(miller), nproj), dtype=np.complex128)
    for i in range(nproj):
        c = (rng.standard_normal(len(miller)) + 1j * rng.standard_normal(len(miller))) * env
        c[np.abs(gx) < 1e-12] = 0.0          # no G_x = 0 component, so that d/dx can be inverted on it
        p[:, i] = real_fn(c)
    p /= np.linalg.norm(p, axis=0)[None, :]
    phit = p @ np.linalg.inv(p.conj().T @ p)                  # duals: phit^H p = 1
    cmat = scale * rng.standard_normal((nproj, nproj))        # d/dx chi_j = sum_k p_k c_kj
    chi = np.zeros_like(p)
    nz = np.abs(gx) > 1e-12
    chi[nz] = (p @ cmat)[nz] / (1j * gx[nz, None])
    return p, phit, chi


def _dx(f, g, gx):
    """<f|d/dx|g> for coefficient vectors on the basis (d/dx multiplies by i G_x)."""
    return np.conj(f) @ (1j * gx * g)


def test_paw_head_equals_the_all_electron_head():
    """The head assembled from the pseudo coefficients, P and D (Eq. n_q0 with Eq. nabla) equals the head of
    the all-electron states, which in turn is the k.p limit of their pair density. A wrong sign of the PAW
    term, a conjugate on the wrong side or a transposed D fails it."""
    rng = np.random.default_rng(33)
    A, miller = _basis()
    V = _potential(rng, A, miller)
    qhat = np.array([1.0, 0.0, 0.0])
    nb, npj = 6, 4
    dM, eps, C_ae = _kp_head(A, miller, V, qhat, nb)
    p, phit, chi = _paw_toy(rng, A, miller, npj)
    B = oracle.reciprocal_rows(A)
    gx = oracle.cartesian(miller, B)[:, 0]
    # pseudo states: c_ae = (1 + chi p^H) c~  ->  c~ = c_ae - chi (1 + p^H chi)^-1 p^H c_ae
    T = np.eye(npj) + p.conj().T @ chi
    Ct = (C_ae.T - chi @ np.linalg.solve(T, p.conj().T @ C_ae.T)).T
    P = Ct @ np.conj(p)                          # P_ni = <p~_i|psi~_n>
    assert np.max(np.abs(Ct + P @ chi.T - C_ae)) < 1e-12
    phi = phit + chi
    D = np.array([[_dx(phi[:, i], phi[:, j], gx) - _dx(phit[:, i], phit[:, j], gx) for j in range(npj)]
                  for i in range(npj)])
    assert np.max(np.abs(D.imag)) < 1e-12 and np.max(np.abs(D + D.T)) < 1e-12
    Dtab = np.zeros((3, npj * npj))
    Dtab[0] = D.real.reshape(-1)
    Dtab[1] = rng.standard_normal(npj * npj)     # other directions do not enter along x
    pairs = _pairs(nb)
    off = np.array([0, npj])
    head = oracle.optical_head(Ct, miller, np.zeros(3), A, P, Dtab, off, eps, pairs, qhat)
    pseudo_only = oracle.optical_head(Ct, miller, np.zeros(3), A, P, np.zeros((3, npj * npj)), off, eps, pairs, qhat)
    ref = dM[pairs]
    # the PAW part must matter here for the pin to mean anything
    assert np.max(np.abs(pseudo_only - ref)) > 1e-2 * np.max(np.abs(ref))
    assert np.max(np.abs(head - ref)) < 1e-6 * np.max(np.abs(ref))
