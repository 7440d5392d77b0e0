"""Pins of the oracle's treatment of spin (Sec. 2.2: the spin index is implicit in Eq. chi0; Table 1 loops
over it): chi0 is the sum of the spin channels' chi0, each a state set with occupations in [0, 1].

1. Spin-unpolarised limit: two identical channels with occupations f/2 give the chi0 of one set with f
   (the reading that f in [0, 2] carries both spins).
2. Two channels with one occupied and one empty state each: chi0 = a_up rho_up rho_up^H +
   a_dn rho_dn rho_dn^H has rank 2, and with x = v^1/2 rho Sylvester's determinant identity gives
       F(w) = ln det(I_2 + diag(|a|) G) - sum_s |a_s| G_ss,   G_st = x_s^H x_t,
   a closed form independent of the oracle's eigenvalue path (and of its Cholesky path); with
   X = diag(|a|) G, det(I_2 + X) = 1 + tr X + det X.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth


def _halved(s):
    return dataclasses.replace(s, f=0.5 * s.f)


def test_spin_unpolarised_limit():
    w = synth.tiny(grid=(10, 10, 10), n_occ=2, n_unocc=6, target_ng=20)
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(w.paw, w.A, qp.q, gm)
    s = w.kpoints[0]
    chi1 = oracle.chi0_q(w.A, w.grid, [s], [s], gm, Q, w.paw.offsets, w.omega)
    h = _halved(s)
    chi2 = oracle.chi0_q(w.A, w.grid, [h, h], [h, h], gm, Q, w.paw.offsets, w.omega)
    assert np.max(np.abs(chi2 - chi1)) <= 1e-14 * np.max(np.abs(chi1))
    # one channel alone is half of it
    chih = oracle.chi0_q(w.A, w.grid, [h], [h], gm, Q, w.paw.offsets, w.omega)
    assert np.max(np.abs(2 * chih - chi1)) <= 1e-14 * np.max(np.abs(chi1))


def _two_channel():
    w = synth.tiny(grid=(12, 12, 12), L=(8.0, 8.5, 9.0), n_occ=1, n_unocc=1, nproj=(2, 2), target_ng=25,
                   q_frac=(0.15, 0.05, 0.0), nw=16, spin_moment=0)
    return w


def test_spin_workload_shape():
    w = synth.tiny(n_occ=3, n_unocc=5, spin_moment=2)
    up, dn = w.kpoints
    assert up.nbands == dn.nbands == 8
    assert np.sum(up.f) == 4.0 and np.sum(dn.f) == 2.0
    assert set(np.unique(up.f)) <= {0.0, 1.0}


def test_two_channel_closed_form():
    w = _two_channel()
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(w.paw, w.A, qp.q, gm)
    chans = w.kpoints
    assert len(chans) == 2 and all(c.nbands == 2 and c.f[0] == 1.0 and c.f[1] == 0.0 for c in chans)
    E, F, chi = oracle.ec_q(w.A, w.grid, chans, chans, gm, Q, w.paw.offsets, qp.q, w.omega, w.omega_weight)
    vs = oracle.coulomb_sqrt(w.A, qp.q, gm)
    # closed form, with rho, a and v^1/2 taken from the definitions written out here
    Bm = 2 * np.pi * np.linalg.inv(w.A).T
    K = qp.q[None, :] + gm @ Bm
    v_half = np.sqrt(4 * np.pi / np.einsum("gc,gc->g", K, K))
    assert np.allclose(v_half, vs, rtol=1e-15)
    xs, D = [], []
    for c in chans:
        pairs, rho = oracle.pair_densities(w.A, w.grid, c, c, gm, Q, w.paw.offsets)
        assert rho.shape[0] == 1
        xs.append(v_half * rho[0])
        D.append(c.eps[0] - c.eps[1])
    G = np.array([[np.vdot(xs[i], xs[j]) for j in range(2)] for i in range(2)])
    Fc = np.empty_like(F)
    for iw, om in enumerate(w.omega):
        a = np.array([c.weight / w.volume * (c.f[0] - c.f[1]) * 2 * d / (om * om + d * d) for c, d in zip(chans, D)])
        X = np.diag(np.abs(a)) @ G
        # det(I_2 + X) = 1 + tr X + det X, so ln det = log1p(tr X + det X), kept apart from the 1
        t = np.real(np.trace(X))
        d = np.real(X[0, 0] * X[1, 1] - X[0, 1] * X[1, 0])
        Fc[iw] = np.log1p(t + d) - t
    assert np.max(np.abs(F - Fc)) <= 1e-12 * np.max(np.abs(Fc))
    Fch = oracle.integrand_cholesky(chi, vs)
    assert np.max(np.abs(Fch - Fc)) <= 1e-12 * np.max(np.abs(Fc))
    assert E == pytest.approx(oracle.ec_from_integrand(Fc, w.omega_weight), rel=1e-12)
    # the channels interact: the energy is not the sum of the one-channel energies
    E1 = sum(oracle.ec_q(w.A, w.grid, [c], [c], gm, Q, w.paw.offsets, qp.q, w.omega, w.omega_weight)[0]
             for c in chans)
    assert abs(E - E1) > 1e-6 * abs(E)
