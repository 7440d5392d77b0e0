"""Pins of the oracle's chi0 at real frequencies (reading R14: Eq. chi0 with i w -> w + i eta, the two
orderings of each transition paired as on the imaginary axis).

1. Analytic continuation: at w = 0 and eta = w' the real-frequency chi0 is the imaginary-axis chi0 at i w'
   (whose weights are pinned by the closed forms of the imaginary-axis tests), for every element.
2. chi0(-w) = chi0(w)^H (the weights at -w are the conjugates).
3. Absorption: Im chi0_GG(w) <= 0 on the diagonal for w > 0 (and >= 0 for w < 0).
4. One transition: chi0 = a(w) rho rho^H with a(w) written out here from the definition.
5. The intraband head continues the same way: at w = 0, eta = w' it equals the imaginary-axis head.
"""
import numpy as np

import oracle
import synth


def _case(**kw):
    w = synth.tiny(grid=(10, 10, 10), n_occ=2, n_unocc=5, target_ng=20, **kw)
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(w.paw, w.A, qp.q, gm)
    return w, qp, gm, Q


def test_zero_frequency_continues_to_the_imaginary_axis():
    w, qp, gm, Q = _case()
    s = w.kpoints
    chi_i = oracle.chi0_q(w.A, w.grid, s, s, gm, Q, w.paw.offsets, w.omega)
    for iw, om in enumerate(w.omega):
        chi_r = oracle.chi0_q_real(w.A, w.grid, s, s, gm, Q, w.paw.offsets, np.array([0.0]), om)
        assert np.max(np.abs(chi_r[0] - chi_i[iw])) <= 1e-13 * np.max(np.abs(chi_i[iw]))


def test_negative_frequency_is_the_adjoint_and_absorption_sign():
    w, qp, gm, Q = _case()
    s = w.kpoints
    om = np.array([0.4, 1.1, 2.5])
    cp = oracle.chi0_q_real(w.A, w.grid, s, s, gm, Q, w.paw.offsets, om, 0.05)
    cm = oracle.chi0_q_real(w.A, w.grid, s, s, gm, Q, w.paw.offsets, -om, 0.05)
    assert np.max(np.abs(cm - np.conj(np.transpose(cp, (0, 2, 1))))) <= 1e-14 * np.max(np.abs(cp))
    d = np.imag(np.einsum("wgg->wg", cp))
    assert np.all(d <= 1e-18)
    assert np.min(d) < -1e-6 * np.max(np.abs(cp))
    assert np.all(np.imag(np.einsum("wgg->wg", cm)) >= -1e-18)
    # not Hermitian at real frequencies
    assert np.max(np.abs(cp - np.conj(np.transpose(cp, (0, 2, 1))))) > 1e-3 * np.max(np.abs(cp))


def test_one_transition_written_out():
    w = synth.tiny(grid=(8, 8, 8), n_occ=1, n_unocc=1, target_ng=15)
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(w.paw, w.A, qp.q, gm)
    s = w.kpoints[0]
    om, eta = np.array([-0.7, 0.3, 1.9]), 0.02
    chi = oracle.chi0_q_real(w.A, w.grid, [s], [s], gm, Q, w.paw.offsets, om, eta)
    _, rho = oracle.pair_densities(w.A, w.grid, s, s, gm, Q, w.paw.offsets)
    d = s.eps[0] - s.eps[1]
    vol = abs(np.linalg.det(w.A))
    for iw, x in enumerate(om):
        a = s.weight / vol * (s.f[0] - s.f[1]) * (1 / (x + 1j * eta + d) - 1 / (x + 1j * eta - d))
        ref = a * np.outer(rho[0], np.conj(rho[0]))
        assert np.max(np.abs(chi[iw] - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_intraband_head_continues_to_the_imaginary_axis():
    w = synth.tiny(grid=(10, 10, 10), n_occ=3, n_unocc=5, optical=True, target_ng=12, fermi_T=0.05)
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(w.paw, w.A, qp.q, gm)
    D = synth.paw_d_table(w.paw)
    s = w.kpoints
    chi_i = oracle.chi0_q(w.A, w.grid, s, s, gm, Q, w.paw.offsets, w.omega, optical=True, qhat=qp.qhat, Dtab=D)
    for iw in (0, 3, 7):
        chi_r = oracle.chi0_q_real(w.A, w.grid, s, s, gm, Q, w.paw.offsets, np.array([0.0]), w.omega[iw],
                                   optical=True, qhat=qp.qhat, Dtab=D)
        assert np.max(np.abs(chi_r[0] - chi_i[iw])) <= 1e-13 * np.max(np.abs(chi_i[iw]))
