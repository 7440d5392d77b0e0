"""Pin of the oracle's intraband head at q -> 0 (reading R13) against the n = m terms of Eq. chi0 at small q.

Model: the local-potential Hamiltonian of test_oracle_optical, with two k-points k0 and -k0 (weights 1/2;
the potential is real, so the spectrum is time-reversal symmetric) and Fermi-smeared occupations that leave
two bands partly filled. At a finite q along qhat, the n = m terms of Eq. chi0 at G = G' = 0,
    (1/Omega) sum_k w_k sum_n (f(e_nk) - f(e_n,k+q)) / (i w + e_nk - e_n,k+q) |<u_nk|u_n,k+q>|^2,
times v(q) = 4 pi/|q|^2, tend (real part, Richardson-extrapolated in q) to 4 pi times the oracle's head
    -(1/Omega) sum_k w_k sum_n (-df/de)_n (qhat.v_n)^2 / w^2,
with the band velocity taken from the coefficients (the diagonal of Eq. n_q0's numerator). A factor of 2,
a missing 1/w^2, the sign, the weights or a velocity from the wrong momentum fail it.
"""
import dataclasses

import numpy as np

import oracle
import synth
from test_oracle_optical import _basis, _eig, _potential


@dataclasses.dataclass
class _Set:
    kpt: np.ndarray
    weight: float
    miller: np.ndarray
    C: np.ndarray
    eps: np.ndarray
    f: np.ndarray
    P: np.ndarray
    dfde: np.ndarray


def test_intraband_head_is_the_small_q_limit():
    rng = np.random.default_rng(5)
    A, miller = _basis()
    V = _potential(rng, A, miller)
    B = oracle.reciprocal_rows(A)
    k0 = 0.11 * B[0] + 0.07 * B[1] + 0.05 * B[2]
    qhat = np.array([0.8, 0.6, 0.0])
    nb = 6
    e0, U0 = _eig(A, miller, V, k0)
    assert np.min(np.diff(e0[:nb + 1])) > 1e-3
    mu, T = 0.5 * (e0[2] + e0[3]), 0.4 * (e0[3] - e0[2])

    def occ(e):
        return 2.0 / (1.0 + np.exp((e - mu) / T))

    def mdf(e):
        f = occ(e)
        return f * (2.0 - f) / (2.0 * T)

    sets = []
    for k in (k0, -k0):
        e, U = _eig(A, miller, V, k)
        sets.append(_Set(kpt=k, weight=0.5, miller=miller, C=U[:nb], eps=e[:nb], f=occ(e[:nb]),
                         P=np.zeros((nb, 0), dtype=np.complex128), dfde=mdf(e[:nb])))
    assert np.allclose(sets[0].eps, sets[1].eps, atol=1e-12)
    assert np.min(np.abs(sets[0].f - np.round(sets[0].f / 2) * 2)) < 1.0  # some band partly filled
    omega = np.array([0.2, 0.7, 2.0])
    vol = abs(np.linalg.det(A))
    head = oracle.intraband_head(sets, A, np.zeros((3, 0)), np.array([0]), qhat, omega)
    assert np.all(head < 0)

    def finite_q(t):
        acc = np.zeros(omega.size, dtype=np.complex128)
        for s in sets:
            e1, U1 = _eig(A, miller, V, s.kpt + t * qhat)
            ov = np.abs(np.einsum("nq,nq->n", np.conj(s.C), U1[:nb])) ** 2
            d = s.eps - e1[:nb]
            df = occ(s.eps) - occ(e1[:nb])
            for iw, w in enumerate(omega):
                acc[iw] += s.weight / vol * np.sum(df / (1j * w + d) * ov)
        return 4 * np.pi / t ** 2 * acc.real

    t = 2e-3
    lim = (4 * finite_q(t / 2) - finite_q(t)) / 3
    ref = 4 * np.pi * head
    assert np.max(np.abs(lim - ref)) < 1e-5 * np.max(np.abs(ref)), (lim, ref)


def test_intraband_head_enters_chi0_only_at_the_optical_head():
    """In chi0 the term is added to the G = G' = 0 element of the optical q-point and nowhere else."""
    w = synth.tiny(grid=(10, 10, 10), n_occ=3, n_unocc=5, optical=True, target_ng=12, fermi_T=0.05)
    s = w.kpoints[0]
    assert s.dfde is not None and np.max(s.dfde) > 0.1
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(w.paw, w.A, qp.q, gm)
    D = synth.paw_d_table(w.paw)
    chi = oracle.chi0_q(w.A, w.grid, [s], [s], gm, Q, w.paw.offsets, w.omega, optical=True, qhat=qp.qhat, Dtab=D)
    s0 = dataclasses.replace(s, dfde=None)
    chi0 = oracle.chi0_q(w.A, w.grid, [s0], [s0], gm, Q, w.paw.offsets, w.omega, optical=True, qhat=qp.qhat,
                         Dtab=D)
    g0 = int(np.nonzero(np.all(gm == 0, axis=1))[0][0])
    diff = chi - chi0
    head = oracle.intraband_head([s], w.A, D, w.paw.offsets, qp.qhat, w.omega)
    assert np.allclose(diff[:, g0, g0], head, rtol=1e-12, atol=0)
    diff[:, g0, g0] = 0
    assert np.max(np.abs(diff)) == 0.0
