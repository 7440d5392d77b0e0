"""Pins of the reference gradient (oracle/grad.py): its forward value equals the
numpy oracle, and its gradient matches central finite differences of the numpy
oracle's E_c(q) along random directions (step 1e-5), and the closed-form
derivative of the two-level E_c with respect to the level spacing."""
import numpy as np
import pytest

import oracle
import oracle.grad as G
import synth


def _ec_numpy(wl, s, t, qp, gm, Q, D):
    E, _, _ = oracle.ec_q(wl.A, wl.grid, [s], [t], gm, Q, wl.paw.offsets, qp.q, wl.omega, wl.omega_weight,
                          optical=qp.optical, qhat=qp.qhat, Dtab=D)
    return E


def _replace(s, **kw):
    d = dict(kpt=s.kpt, weight=s.weight, miller=s.miller, C=s.C, eps=s.eps, f=s.f, P=s.P)
    d.update(kw)
    return synth.StateSet(**d)


CASES = {
    "q_finite": lambda: synth.tiny(grid=(8, 8, 8), n_occ=2, n_unocc=4, target_ng=15, nw=8),
    "optical": lambda: synth.tiny(grid=(10, 10, 10), n_occ=2, n_unocc=3, optical=True, target_ng=12, nw=8),
    "distinct_kq": lambda: synth.tiny(grid=(8, 8, 8), n_occ=2, n_unocc=3, target_ng=15, nw=8, extra_kq=True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_gradient_matches_finite_differences(case):
    wl = CASES[case]()
    s, t = wl.kpoints[0], wl.kq_sets()[0]
    qp = wl.qpoints[0]
    gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
    D = synth.paw_d_table(wl.paw)
    E0 = _ec_numpy(wl, s, t, qp, gm, Q, D)
    same = wl.kq is None
    E, g = G.ec_and_grad(wl.A, wl.grid, s, s if same else t, gm, Q, wl.paw.offsets, qp.q, wl.omega,
                         wl.omega_weight, qp.optical, qp.qhat, D)
    assert abs(E - E0) < 1e-12 * max(1.0, abs(E0))
    rng = np.random.default_rng(7)
    h = 1e-5
    for trial in range(6):
        dC = rng.standard_normal(s.C.shape) + 1j * rng.standard_normal(s.C.shape)
        dP = rng.standard_normal(s.P.shape) + 1j * rng.standard_normal(s.P.shape)
        de = rng.standard_normal(s.eps.shape) * 0.1
        which = trial % 3
        kw_p = {}
        kw_m = {}
        if which == 0:
            kw_p["C"], kw_m["C"] = s.C + h * dC, s.C - h * dC
            pred = float(np.real(np.sum(np.conj(g["C_k"]) * dC)))
        elif which == 1:
            kw_p["P"], kw_m["P"] = s.P + h * dP, s.P - h * dP
            pred = float(np.real(np.sum(np.conj(g["P_k"]) * dP)))
        else:
            kw_p["eps"], kw_m["eps"] = s.eps + h * de, s.eps - h * de
            pred = float(np.sum(g["eps_k"] * de))
        sp, sm = _replace(s, **kw_p), _replace(s, **kw_m)
        if same:
            fd = (_ec_numpy(wl, sp, sp, qp, gm, Q, D) - _ec_numpy(wl, sm, sm, qp, gm, Q, D)) / (2 * h)
        else:
            fd = (_ec_numpy(wl, sp, t, qp, gm, Q, D) - _ec_numpy(wl, sm, t, qp, gm, Q, D)) / (2 * h)
        assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred)), (case, which, fd, pred)


def test_two_level_spacing_derivative():
    """dE/d(eps_m) of the two-level closed form: E = (1/2)[sqrt(D^2 + bD) - D - b/2], D = e_m - e_n,
    with b fixed when the pair density does not depend on the energies (finite q)."""
    wl = synth.tiny(grid=(12, 12, 12), L=(8.0, 8.5, 9.0), n_occ=1, n_unocc=1, nproj=(2, 2), target_ng=20,
                    q_frac=(0.15, 0.05, 0.0), nw=64)
    s = wl.kpoints[0]
    qp = wl.qpoints[0]
    gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
    E, g = G.ec_and_grad(wl.A, wl.grid, s, s, gm, Q, wl.paw.offsets, qp.q, wl.omega, wl.omega_weight)
    pairs, rho = oracle.pair_densities(wl.A, wl.grid, s, s, gm, Q, wl.paw.offsets)
    Bm = 2 * np.pi * np.linalg.inv(wl.A).T
    K = qp.q[None, :] + gm @ Bm
    v = 4 * np.pi / np.einsum("gc,gc->g", K, K)
    b = 2.0 * (s.f[0] - s.f[1]) * s.weight * float(np.sum(v * np.abs(rho[0]) ** 2)) / wl.volume
    D = s.eps[1] - s.eps[0]
    dE_dD = 0.5 * ((2 * D + b) / (2 * np.sqrt(D * D + b * D)) - 1.0)
    assert abs(g["eps_k"][1] - dE_dD) < 1e-9 * abs(dE_dD)
    assert abs(g["eps_k"][0] + dE_dD) < 1e-9 * abs(dE_dD)


def test_gradient_over_several_set_pairs():
    """ec_and_grad_sets (Eq. chi0's k sum over two listings: (s, t) and (t', t') with t' a copy of t at
    half weight): its E equals the numpy oracle's over the same pairs, and each listing's gradient
    matches central finite differences that move only that listing's inputs."""
    wl = synth.tiny(grid=(8, 8, 8), n_occ=2, n_unocc=3, target_ng=15, nw=8, extra_kq=True)
    s, t = wl.kpoints[0], wl.kq_sets()[0]
    t2 = _replace(t, weight=0.5)
    qp = wl.qpoints[0]
    gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)

    def ec(ks, kqs):
        return oracle.ec_q(wl.A, wl.grid, ks, kqs, gm, Q, wl.paw.offsets, qp.q, wl.omega, wl.omega_weight)[0]

    E0 = ec([s, t2], [t, t2])
    E, g = G.ec_and_grad_sets(wl.A, wl.grid, [s, t2], [t, t2], gm, Q, wl.paw.offsets, qp.q, wl.omega,
                              wl.omega_weight)
    assert abs(E - E0) < 1e-12 * max(1.0, abs(E0))
    assert set(g[0]) == {"eps_k", "C_k", "P_k", "eps_kq", "C_kq", "P_kq"} and set(g[1]) == {"eps_k", "C_k", "P_k"}
    rng = np.random.default_rng(3)
    h = 1e-5
    dC = rng.standard_normal(t.C.shape) + 1j * rng.standard_normal(t.C.shape)
    dP = rng.standard_normal(t.P.shape) + 1j * rng.standard_normal(t.P.shape)
    # listing 0's k+q set (t) alone
    fd = (ec([s, t2], [_replace(t, C=t.C + h * dC), t2]) - ec([s, t2], [_replace(t, C=t.C - h * dC), t2])) / (2 * h)
    pred = float(np.real(np.sum(np.conj(g[0]["C_kq"]) * dC)))
    assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred)), (fd, pred)
    # listing 1 (t2 in both roles)
    p, m = _replace(t2, P=t2.P + h * dP), _replace(t2, P=t2.P - h * dP)
    fd = (ec([s, p], [t, p]) - ec([s, m], [t, m])) / (2 * h)
    pred = float(np.real(np.sum(np.conj(g[1]["P_k"]) * dP)))
    assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred)), (fd, pred)
