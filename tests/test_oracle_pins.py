"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks one oracle step against something other than the oracle's own
formula: a direct-sum definition evaluated a different way, a closed form, an
invariant, or an independent textbook routine.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = []


def _rand_states(rng, nb, grid):
    """Random complex periodic functions on a grid (no structure), for definition checks."""
    return rng.standard_normal((nb,) + grid) + 1j * rng.standard_normal((nb,) + grid)


# ---------------------------------------------------------------------------
# G-sphere (Sec. 2.1; Table 1 step 6)
# ---------------------------------------------------------------------------
def test_gsphere_matches_python_enumeration():
    A = np.array([[7.0, 0.0, 0.0], [1.0, 6.5, 0.0], [0.5, 0.3, 8.0]])   # non-orthorhombic
    q = np.array([0.05, -0.02, 0.03])
    ecut = 1.7
    B = 2 * np.pi * np.linalg.inv(A).T
    ref = []
    for m in itertools.product(range(-12, 13), repeat=3):
        k = q + m[0] * B[0] + m[1] * B[1] + m[2] * B[2]
        if 0.5 * float(k @ k) <= ecut:
            ref.append(m)
    got = oracle.gsphere(A, q, ecut)
    assert sorted(map(tuple, got.tolist())) == sorted(ref)
    k2 = oracle.sq_norm(oracle.cartesian(got, B, q))
    assert np.all(np.diff(k2) >= -1e-12)


def test_gsphere_sizes_of_the_configurations():
    w = synth.config0()
    assert len(oracle.gsphere(w.A, w.qpoints[0].q, w.qpoints[0].ecut)) == 126
    A = np.diag([12.0, 12.0, 13.0])
    for i, ng in zip((0, 1, 2), (1503, 1500, 1502)):
        q = np.array([0.1 * i * 2 * np.pi / 12.0, 0.0, 0.0])
        assert len(oracle.gsphere(A, q, synth.ecut_for_count(A, q, 1500))) == ng


# ---------------------------------------------------------------------------
# orbitals (Eq. get_wfs)
# ---------------------------------------------------------------------------
def test_orbitals_equal_direct_plane_wave_sum():
    w = synth.tiny(grid=(6, 8, 10), L=(6.0, 7.0, 9.0), target_ng=7)
    s = w.kpoints[0]
    grid = w.grid
    phi = oracle.orbitals(s.C, s.miller, grid)
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)
    # G.r = 2 pi sum_i m_i j_i / N_i for r_j = sum_i (j_i/N_i) a_i
    phase = 2j * np.pi * (np.outer(j[:, 0], s.miller[:, 0]) / grid[0]
                          + np.outer(j[:, 1], s.miller[:, 1]) / grid[1]
                          + np.outer(j[:, 2], s.miller[:, 2]) / grid[2])
    direct = (np.exp(phase) @ s.C.T).T.reshape((-1,) + grid)
    assert np.max(np.abs(phi - direct)) < 1e-12


# ---------------------------------------------------------------------------
# pseudo pair density (Eq. n_G, Eq. fft)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("grid", [(4, 4, 4), (6, 6, 6), (8, 8, 8), (6, 8, 10)])
def test_pair_density_equals_direct_dft(grid):
    rng = np.random.default_rng(5)
    phi = _rand_states(rng, 3, grid)
    gm = np.array([[0, 0, 0], [1, 0, 0], [-1, 2, 0], [0, -1, 1], [1, 1, -1], [-2, 0, 1]], dtype=np.int32)
    gm[:, 0] = np.clip(gm[:, 0], -(grid[0] // 2) + 1, grid[0] // 2)
    pairs = (np.array([0, 0, 1, 2]), np.array([1, 2, 2, 0]))
    got = oracle.pseudo_pair_density(phi, phi, pairs, gm, grid)
    N = grid[0] * grid[1] * grid[2]
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3)
    for p, (n, m) in enumerate(zip(*pairs)):
        prod = (np.conj(phi[n]) * phi[m]).reshape(-1)
        for g, G in enumerate(gm):
            e = np.exp(-2j * np.pi * (j[:, 0] * G[0] / grid[0] + j[:, 1] * G[1] / grid[1] + j[:, 2] * G[2] / grid[2]))
            ref = np.sum(prod * e) / N
            assert abs(got[p, g] - ref) < 1e-13 * max(1.0, abs(ref)) * N


def test_pair_density_equals_plane_wave_convolution():
    w = synth.config0(n_occ=2, n_unocc=5)
    s = w.kpoints[0]
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    phi = oracle.orbitals(s.C, s.miller, w.grid)
    pairs = oracle.pair_list(s.f, s.f)
    fft = oracle.pseudo_pair_density(phi, phi, pairs, gm, w.grid)
    pw = oracle.pseudo_pair_density_pw(s.C, s.miller, s.C, s.miller, pairs, gm)
    assert np.max(np.abs(fft - pw)) < 1e-13


def test_pair_density_distinct_k_and_kq_sets():
    w = synth.tiny(extra_kq=True)
    s, t = w.kpoints[0], w.kq[0]
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    pairs = oracle.pair_list(s.f, t.f)
    phi_s = oracle.orbitals(s.C, s.miller, w.grid)
    phi_t = oracle.orbitals(t.C, t.miller, w.grid)
    fft = oracle.pseudo_pair_density(phi_s, phi_t, pairs, gm, w.grid)
    pw = oracle.pseudo_pair_density_pw(s.C, s.miller, t.C, t.miller, pairs, gm)
    assert np.max(np.abs(fft - pw)) < 1e-13


def test_pair_density_at_g0_is_orthonormality():
    """<psi_n|psi_m> = delta_nm at q = 0, G = 0 for the all-electron pair density (Sec. 2.2): the pseudo
    part plus the PAW term of Eq. n_G_2 with Q^a_ij(0), for states orthonormal under the PAW overlap."""
    w = synth.config0(n_occ=3, n_unocc=6)
    s = w.kpoints[0]
    phi = oracle.orbitals(s.C, s.miller, w.grid)
    nb = s.nbands
    pairs = (np.repeat(np.arange(nb), nb), np.tile(np.arange(nb), nb))
    g0 = np.zeros((1, 3), np.int32)
    Q0 = synth.paw_q_table(w.paw, w.A, np.zeros(3), g0)
    pseudo = oracle.pseudo_pair_density(phi, phi, pairs, g0, w.grid)[:, 0]
    full = pseudo + oracle.paw_correction(s.P, s.P, pairs, Q0, w.paw.offsets)[:, 0]
    assert np.max(np.abs(full - np.eye(nb).reshape(-1))) < 1e-13
    # the PAW term is not negligible here: the pseudo part alone is off by much more than rounding
    assert np.max(np.abs(pseudo - np.eye(nb).reshape(-1))) > 1e-5


def test_pseudo_pair_density_at_g0_independent_model():
    """With plainly orthonormal coefficients (the stress workload) the pseudo part alone is delta_nm."""
    w = synth.config0(n_occ=3, n_unocc=6, paw_model="independent")
    s = w.kpoints[0]
    phi = oracle.orbitals(s.C, s.miller, w.grid)
    nb = s.nbands
    pairs = (np.repeat(np.arange(nb), nb), np.tile(np.arange(nb), nb))
    r0 = oracle.pseudo_pair_density(phi, phi, pairs, np.zeros((1, 3), np.int32), w.grid)[:, 0]
    assert np.max(np.abs(r0 - np.eye(nb).reshape(-1))) < 1e-13


def test_pair_density_parseval():
    grid = (6, 8, 10)
    rng = np.random.default_rng(3)
    phi = _rand_states(rng, 2, grid)
    full = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), -1).reshape(-1, 3).astype(np.int32)
    r = oracle.pseudo_pair_density(phi, phi, (np.array([0]), np.array([1])), full, grid)[0]
    N = np.prod(grid)
    assert abs(np.sum(np.abs(r) ** 2) - np.sum(np.abs(np.conj(phi[0]) * phi[1]) ** 2) / N) < 1e-10


# ---------------------------------------------------------------------------
# PAW correction (Eq. n_G_2)
# ---------------------------------------------------------------------------
def test_paw_correction_matches_separable_closed_form():
    w = synth.config0(n_occ=2, n_unocc=4)
    s = w.kpoints[0]
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(w.paw, w.A, qp.q, gm)
    pairs = oracle.pair_list(s.f, s.f)
    got = oracle.paw_correction(s.P, s.P, pairs, Q, w.paw.offsets)
    B = oracle.reciprocal_rows(w.A)
    K = oracle.cartesian(gm, B, qp.q)
    g = np.exp(-0.5 * oracle.sq_norm(K) * w.paw.sigma ** 2)
    ref = np.zeros_like(got)
    off = w.paw.offsets
    for a in range(len(w.paw.nproj)):
        Pn = s.P[pairs[0]][:, off[a]:off[a + 1]]
        Pm = s.P[pairs[1]][:, off[a]:off[a + 1]]
        bil = np.einsum("pi,ij,pj->p", np.conj(Pn), w.paw.s[a], Pm)
        ref += bil[:, None] * (g * np.exp(-1j * (K @ w.paw.R[a])))[None, :]
    assert np.max(np.abs(got - ref)) < 1e-14


def test_paw_correction_factorises_for_rank_one_table():
    """Q_ij(G) = u_i v_j h(G) gives (sum_i conj(P_ni) u_i)(sum_j P_mj v_j) h(G); catches i<->j swaps."""
    rng = np.random.default_rng(9)
    nproj = [3, 5]
    off = np.array([0, 3, 8])
    P = rng.standard_normal((6, 8)) + 1j * rng.standard_normal((6, 8))
    NG = 7
    rows, us, vs, hs = [], [], [], []
    for a, n in enumerate(nproj):
        u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        h = rng.standard_normal(NG) + 1j * rng.standard_normal(NG)
        rows.append((np.outer(u, v).reshape(-1, 1) * h[None, :]))
        us.append(u), vs.append(v), hs.append(h)
    Q = np.concatenate(rows, 0)
    pairs = (np.array([0, 1, 2, 5]), np.array([3, 4, 5, 0]))
    got = oracle.paw_correction(P, P, pairs, Q, off)
    ref = np.zeros_like(got)
    for a in range(2):
        Pa = P[:, off[a]:off[a + 1]]
        left = np.conj(Pa[pairs[0]]) @ us[a]
        right = Pa[pairs[1]] @ vs[a]
        ref += (left * right)[:, None] * hs[a][None, :]
    assert np.max(np.abs(got - ref)) < 1e-12


# ---------------------------------------------------------------------------
# weights and chi0 (Eq. chi0, Eq. A_iw, Eq. zher, Eq. zher_multi)
# ---------------------------------------------------------------------------
def _cfg0_rho(n_occ=4, n_unocc=12):
    w = synth.config0(n_occ=n_occ, n_unocc=n_unocc)
    s = w.kpoints[0]
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(w.paw, w.A, qp.q, gm)
    pairs, rho = oracle.pair_densities(w.A, w.grid, s, s, gm, Q, w.paw.offsets)
    a = oracle.transition_weights(s.eps, s.eps, s.f, s.f, pairs, s.weight, w.volume, w.omega)
    return w, s, qp, gm, Q, pairs, rho, a


def test_pair_set_and_weight_signs():
    w, s, qp, gm, Q, pairs, rho, a = _cfg0_rho()
    assert pairs[0].size == 4 * 12
    assert np.all(s.f[pairs[0]] == 2.0) and np.all(s.f[pairs[1]] == 0.0)
    assert np.all(a < 0)
    # Fermi-smeared set: every selected pair still gets a <= 0 (f decreases with eps)
    eps, f = synth.fermi_levels(np.random.default_rng(0), 30, 40)
    pr = oracle.pair_list(f, f)
    aa = oracle.transition_weights(eps, eps, f, f, pr, 1.0, 100.0, w.omega)
    assert np.all(aa <= 0) and np.all(pr[0] < pr[1])


def test_weight_large_frequency_asymptote():
    """omega^2 a -> (w/Omega)(f_n - f_m) 2 (e_n - e_m) as omega -> inf."""
    eps = np.array([-0.5, 0.7, 1.9])
    f = np.array([2.0, 0.0, 0.0])
    pr = oracle.pair_list(f, f)
    big = np.array([1e6])
    a = oracle.transition_weights(eps, eps, f, f, pr, 0.5, 20.0, big)[:, 0]
    lim = 0.5 / 20.0 * 2.0 * 2.0 * (eps[0] - eps[pr[1]])
    assert np.allclose(a * big[0] ** 2, lim, rtol=1e-10)


def test_chi0_grouping_is_exact_regrouping():
    """Eq. zher (rank-1) = Eq. zher_multi (rank-Nu) for any Nu and any pair order."""
    w, s, qp, gm, Q, pairs, rho, a = _cfg0_rho(n_occ=2, n_unocc=10)
    ref = oracle.chi0_rank1(rho, a)
    for nu in (1, 3, 7, rho.shape[0]):
        assert np.max(np.abs(oracle.chi0_grouped(rho, a, nu) - ref)) < 1e-15
    perm = np.random.default_rng(1).permutation(rho.shape[0])
    assert np.max(np.abs(oracle.chi0_grouped(rho[perm], a[perm], 4) - ref)) < 1e-15


def test_chi0_hermitian_negative_semidefinite_and_gauge_invariant():
    w, s, qp, gm, Q, pairs, rho, a = _cfg0_rho()
    chi = oracle.chi0_grouped(rho, a)
    assert np.max(np.abs(chi - np.conj(np.transpose(chi, (0, 2, 1))))) < 1e-18
    for c in chi:
        lam = np.linalg.eigvalsh(c)
        assert lam.max() <= 1e-14 * np.abs(lam).max()
        assert lam.min() < 0
    # gauge: C_n -> e^{i theta_n} C_n, P_n -> e^{i theta_n} P_n
    theta = np.random.default_rng(2).uniform(0, 2 * np.pi, s.nbands)
    ph = np.exp(1j * theta)
    s2 = synth.StateSet(kpt=s.kpt, weight=s.weight, miller=s.miller, C=s.C * ph[:, None],
                        eps=s.eps, f=s.f, P=s.P * ph[:, None])
    pairs2, rho2 = oracle.pair_densities(w.A, w.grid, s2, s2, gm, Q, w.paw.offsets)
    chi2 = oracle.chi0_grouped(rho2, a)
    assert np.max(np.abs(chi2 - chi)) < 1e-15


# ---------------------------------------------------------------------------
# integrand and E_c (Eq. rpa, Eq. rpa_c)
# ---------------------------------------------------------------------------
def test_integrand_three_ways_and_sign():
    w, s, qp, gm, Q, pairs, rho, a = _cfg0_rho()
    chi = oracle.chi0_grouped(rho, a)
    vs = oracle.coulomb_sqrt(w.A, qp.q, gm)
    F1 = oracle.integrand_cholesky(chi, vs)
    F2 = oracle.integrand(chi, vs)
    F3 = oracle.integrand_slogdet(chi, vs)
    # ln det(1-K) and Tr K cancel at large w, so the scale of the round-off is |Tr K|
    trk = np.abs([np.real(np.trace(k)) for k in oracle.kernel_matrix(chi, vs)])
    assert np.all(np.abs(F1 - F2) <= 1e-13 * trk)
    # slogdet forms 1 - K, so each of its NG pivots carries a rounding of about eps against 1: an absolute
    # error of order NG eps in ln det that no cancellation against Tr K removes
    ng = chi.shape[1]
    assert np.all(np.abs(F1 - F3) <= 1e-12 * trk + 4.0 * ng * np.finfo(float).eps)
    assert np.all(F1 < 0)
    assert oracle.ec_from_integrand(F1, w.omega_weight) < 0


def test_integrand_weak_coupling():
    """F ~= -Tr K^2/2 as rho -> eps rho (ln(1-x) + x = -x^2/2 + O(x^3))."""
    w, s, qp, gm, Q, pairs, rho, a = _cfg0_rho()
    vs = oracle.coulomb_sqrt(w.A, qp.q, gm)
    e = 1e-3
    chi = oracle.chi0_grouped(e * rho, a)
    K = oracle.kernel_matrix(chi, vs)
    F = oracle.integrand_eigen(chi, vs)
    tr2 = np.array([np.real(np.trace(k @ k)) for k in K])
    assert np.allclose(F, -0.5 * tr2, rtol=1e-5)


def _two_level(optical=False, nw=64):
    L = (8.0, 8.5, 9.0)
    w = synth.tiny(grid=(12, 12, 12), L=L, n_occ=1, n_unocc=1, nproj=(2, 2), target_ng=20,
                   q_frac=(0.15, 0.05, 0.0), nw=nw, optical=optical)
    return w


@pytest.mark.parametrize("optical", [False, True])
@pytest.mark.parametrize("nw", [64, 256])
def test_two_level_closed_form(optical, nw):
    """One occupied + one unoccupied state: chi0 has rank 1 and
    E_c = (1/2)[sqrt(D^2 + b D) - D - b/2], b = 2 (f_n - f_m) w_k s / Omega, s = sum_G v_G |rho_G|^2."""
    w = _two_level(optical, nw=nw)
    s = w.kpoints[0]
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(w.paw, w.A, qp.q, gm)
    Dt = synth.paw_d_table(w.paw)
    E, F, chi = oracle.ec_q(w.A, w.grid, [s], [s], gm, Q, w.paw.offsets, qp.q, w.omega,
                            w.omega_weight, optical=qp.optical, qhat=qp.qhat, Dtab=Dt)
    pairs, rho = oracle.pair_densities(w.A, w.grid, s, s, gm, Q, w.paw.offsets, qp.optical, qp.qhat, Dt)
    assert rho.shape[0] == 1
    vs = oracle.coulomb_sqrt(w.A, qp.q, gm, qp.optical)
    # v_G = 4 pi/|q+G|^2 (4 pi at G = 0 in the optical limit, where |q| cancels)
    Bm = 2 * np.pi * np.linalg.inv(w.A).T
    K = qp.q[None, :] + gm @ Bm
    k2 = np.einsum("gc,gc->g", K, K)
    v = np.where(k2 > 0, 4 * np.pi / np.where(k2 > 0, k2, 1.0), 4 * np.pi)
    sfac = float(np.sum(v * np.abs(rho[0]) ** 2))
    D = s.eps[1] - s.eps[0]
    b = 2.0 * (s.f[0] - s.f[1]) * s.weight * sfac / w.volume
    ref = oracle.two_level_ec(D, b)
    assert ref < 0
    assert abs(E - ref) < 5e-12 * abs(ref)
    Fc = oracle.integrand_cholesky(chi, vs)
    assert abs(oracle.ec_from_integrand(Fc, w.omega_weight) - ref) < 5e-12 * abs(ref)


def test_two_level_closed_form_per_node():
    """At 8 or 16 nodes compare F(w_i) node by node with ln(1+c) - c."""
    w = _two_level(False, nw=8)
    s = w.kpoints[0]
    qp = w.qpoints[0]
    gm = oracle.gsphere(w.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(w.paw, w.A, qp.q, gm)
    E, F, chi = oracle.ec_q(w.A, w.grid, [s], [s], gm, Q, w.paw.offsets, qp.q, w.omega, w.omega_weight)
    pairs, rho = oracle.pair_densities(w.A, w.grid, s, s, gm, Q, w.paw.offsets)
    vs = oracle.coulomb_sqrt(w.A, qp.q, gm)
    sfac = float(np.sum(vs ** 2 * np.abs(rho[0]) ** 2))
    D = s.eps[1] - s.eps[0]
    b = 2.0 * 2.0 * sfac / w.volume
    c = b * D / (w.omega ** 2 + D * D)
    assert np.allclose(F, np.log1p(c) - c, rtol=1e-11)


# ---------------------------------------------------------------------------
# quadrature (Sec. 2.1)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [8, 16, 64])
def test_golub_welsch_matches_library_gauss_legendre(n):
    t, w = oracle.gauss_legendre(n)
    t2, w2 = np.polynomial.legendre.leggauss(n)
    assert np.max(np.abs(t - t2)) < 1e-13 and np.max(np.abs(w - w2)) < 1e-13
    om, ow = oracle.frequency_grid(n)
    om2, ow2 = synth.frequency_grid(n)
    assert np.allclose(om, om2, rtol=1e-12) and np.allclose(ow, ow2, rtol=1e-11)


def test_mapped_rule_integrates_lorentzian():
    """int_0^inf dw/(w^2 + D^2) = pi/(2D)."""
    om, ow = oracle.frequency_grid(16)
    for D in (0.5, 1.0, 2.0):
        val = np.sum(ow / (om ** 2 + D * D))
        assert abs(val - np.pi / (2 * D)) < 2e-6 * np.pi / (2 * D)
    om, ow = oracle.frequency_grid(64)
    assert abs(np.sum(ow / (om ** 2 + 1.0)) - np.pi / 2) < 1e-12


# ---------------------------------------------------------------------------
# optical limit (Eq. n_q0, Eq. nabla; GPU reformulation of the stencil)
# ---------------------------------------------------------------------------
def _stencil_coefficients(p=6):
    # central first-derivative weights of order 2p: c_k = 2 (-1)^{k+1} (p!)^2 / (k (p-k)! (p+k)!)
    return np.array([2.0 * (-1) ** (k + 1) * math.factorial(p) ** 2
                     / (k * math.factorial(p - k) * math.factorial(p + k)) for k in range(1, p + 1)])


def test_momentum_plane_wave_equals_fft_derivative_and_stencil():
    rng = np.random.default_rng(4)
    L = np.array([6.0, 6.5, 7.0])
    A = np.diag(L)
    grid = (24, 24, 24)
    kpt = np.zeros(3)
    miller = synth.wavefunction_sphere(A, kpt, 0.9)
    C = synth.orthonormal_coefficients(rng, A, kpt, miller, 4)
    pairs = (np.array([0, 0, 1]), np.array([1, 2, 3]))
    qhat = np.array([1.0, 0.0, 0.0])
    pw = oracle.momentum_pw(C, miller, kpt, A, pairs, qhat)
    phi = oracle.orbitals(C, miller, grid)
    N = np.prod(grid)
    # FFT derivative along x: multiply by i G_x in reciprocal space
    spec = np.fft.fftn(phi, axes=(1, 2, 3))
    gx = 2 * np.pi * np.fft.fftfreq(grid[0], d=L[0] / grid[0])
    dphi = np.fft.ifftn(spec * (1j * gx)[None, :, None, None], axes=(1, 2, 3))
    fftd = np.array([-1j * np.sum(np.conj(phi[n]) * dphi[m]) / N for n, m in zip(*pairs)])
    assert np.max(np.abs(fftd - pw)) < 1e-12
    # 13-point stencil (6 neighbours per side)
    c = _stencil_coefficients(6)
    h = L[0] / grid[0]
    dst = np.zeros_like(phi)
    for k, ck in enumerate(c, start=1):
        dst += ck * (np.roll(phi, -k, axis=1) - np.roll(phi, k, axis=1)) / (2 * h)
    sten = np.array([-1j * np.sum(np.conj(phi[n]) * dst[m]) / N for n, m in zip(*pairs)])
    assert np.max(np.abs(sten - pw)) < 1e-6


def test_optical_head_is_hermitian_pairing_consistent():
    """n(G=0) of (m, n) is minus the conjugate of that of (n, m): the momentum matrix is
    Hermitian and the energy denominator flips sign."""
    w = synth.tiny(grid=(10, 10, 10), n_occ=2, n_unocc=3, optical=True, target_ng=9)
    s = w.kpoints[0]
    Dt = synth.paw_d_table(w.paw)
    fwd = (np.array([0, 1, 0]), np.array([2, 3, 4]))
    bwd = (fwd[1], fwd[0])
    h1 = oracle.optical_head(s.C, s.miller, s.kpt, w.A, s.P, Dt, w.paw.offsets, s.eps, fwd, np.array([1.0, 0, 0]))
    h2 = oracle.optical_head(s.C, s.miller, s.kpt, w.A, s.P, Dt, w.paw.offsets, s.eps, bwd, np.array([1.0, 0, 0]))
    assert np.max(np.abs(h1 + np.conj(h2))) < 1e-14
