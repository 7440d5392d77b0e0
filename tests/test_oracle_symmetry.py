"""Pins of the oracle's symmetry unfolding (Eq. kmap, Eq. trans_wfs; Table 1 steps 4 and 7).

Model: a simple-cubic cell with seven atoms (one at the origin, six at +-a/4 along the axes: an orbit
of the full cubic group, so every operation maps atoms onto atoms, some across a lattice vector), a
local potential V(G) = sum_a v(|G|) e^{-i G.R_a} (real and invariant under the 48 operations) and
plane-wave Hamiltonians H(k)_GG' = |k+G|^2/2 delta + V(G - G'). Projector functions of every atom are
real s and p functions (a Gaussian and x_c times it), so their Fourier transforms are known in closed
form and the projections at any k can be formed directly, P_k = sum_Q C_k(Q) <p~|e^{i(k+G_Q).r}>.

1. Eigenvectors at k1 unfolded by an operation are eigenvectors of H(k) at the transformed k with the
   same eigenvalues (pins the grid remap, U against U^-1 for a three-fold axis, the conjugation of time
   reversal and the sign of G0).
2. The rotated projections equal the projections formed directly at k from the unfolded coefficients
   (pins D against its transpose, the atom map and the Bloch phase of atoms mapped across a lattice
   vector).
3. chi0 built from unfolded k and k+q sets equals chi0 from states diagonalised directly at k and k+q
   (gauge invariance; pins the whole unfolding inside the chi0 path, the PAW term included).
"""
import dataclasses

import numpy as np
import pytest

import oracle
import oracle.symmetry as osym
import synth

L = 7.0
A = L * np.eye(3)
GRID = (12, 12, 12)
ATOMS = np.array([[0, 0, 0], [0.25, 0, 0], [0.75, 0, 0], [0, 0.25, 0], [0, 0.75, 0], [0, 0, 0.25],
                  [0, 0, 0.75]])
SIGMA = 0.6
NB = 8

C3 = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]])     # three-fold axis along (1, 1, 1)
C4 = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]])    # four-fold axis along z
MX = np.diag([-1, 1, 1])                              # mirror x -> -x
OPS = [(C3, 0, (0, 0, 0)), (C3, 1, (0, 0, 0)), (C4, 0, (1, 0, 0)), (C4.T, 1, (0, -1, 1)), (MX, 1, (0, 0, 0)),
       (C3 @ C4, 0, (0, 1, 0))]


@dataclasses.dataclass
class _Set:
    kpt: np.ndarray
    weight: float
    miller: np.ndarray
    C: np.ndarray
    eps: np.ndarray
    f: np.ndarray
    P: np.ndarray
    dfde: object = None


def _vg(gcart):
    g2 = oracle.sq_norm(gcart)
    out = np.zeros(gcart.shape[:-1], dtype=np.complex128)
    for x in ATOMS:
        R = x @ A
        out += -0.8 * np.exp(-0.3 * g2) * np.exp(-1j * (gcart @ R))
    return out


def _states(k, ecut=2.0):
    B = oracle.reciprocal_rows(A)
    miller = synth.wavefunction_sphere(A, k, ecut)
    kg = oracle.cartesian(miller, B, k)
    d = miller[:, None, :] - miller[None, :, :]
    V = _vg(oracle.cartesian(d.reshape(-1, 3), B).reshape(d.shape[0], d.shape[1], 3))
    V[np.arange(len(miller)), np.arange(len(miller))] = 0.0
    H = np.diag(0.5 * oracle.sq_norm(kg)).astype(np.complex128) + V
    e, U = np.linalg.eigh(H)
    return miller, e, U.T.copy(), H


def _proj_table(k, miller):
    """<p~^a_i | e^{i(k+G_Q).r}> for s and p projectors: e^{i K.R_a} (1, i K_x, i K_y, i K_z) e^{-K^2 s^2/2}."""
    B = oracle.reciprocal_rows(A)
    K = oracle.cartesian(miller, B, k)
    g = np.exp(-0.5 * SIGMA ** 2 * oracle.sq_norm(K))
    cols = []
    for x in ATOMS:
        ph = np.exp(1j * (K @ (x @ A))) * g
        cols += [ph, 1j * K[:, 0] * ph, 1j * K[:, 1] * ph, 1j * K[:, 2] * ph]
    return np.stack(cols, axis=1)


OFFSETS = np.arange(0, 4 * len(ATOMS) + 1, 4)


def _atom_map(U):
    Ui = np.rint(np.linalg.inv(U)).astype(int)
    amap, shift = [], []
    for x in ATOMS:
        y = Ui @ x
        for b, xb in enumerate(ATOMS):
            d = y - xb
            if np.allclose(d, np.rint(d), atol=1e-12):
                amap.append(b)
                shift.append(np.rint(d).astype(int))
                break
        else:
            raise AssertionError("atoms not closed under the operation")
    return np.array(amap), np.array(shift)


def _dblocks(U):
    T = osym.cartesian_rotation(U, A)
    blk = np.zeros((4, 4))
    blk[0, 0] = 1.0
    blk[1:, 1:] = T
    return np.tile(blk.reshape(-1), len(ATOMS))


def _ibz_set(k1, nb=NB, occ=3):
    miller, e, C, _ = _states(k1)
    assert e[nb] - e[nb - 1] > 1e-4
    f = np.zeros(nb)
    f[:occ] = 2.0
    P = C[:nb] @ _proj_table(k1, miller)
    return _Set(kpt=np.asarray(k1, dtype=float), weight=0.25, miller=miller, C=C[:nb], eps=e[:nb], f=f, P=P)


K1 = np.array([0.11, 0.047, 0.023]) * 2 * np.pi / L


def test_symmetric_model_is_symmetric():
    # every operation used is a symmetry of the lattice and of the atoms
    moved = 0
    for U, _, _ in OPS:
        T = osym.cartesian_rotation(U, A)
        assert np.allclose(T @ T.T, np.eye(3), atol=1e-14)
        amap, shift = _atom_map(U)
        moved += int(np.any(shift != 0))
    # some operations map atoms across a lattice vector (the Bloch phase of the rotated projections)
    assert moved >= 2


@pytest.mark.parametrize("iop", range(len(OPS)))
def test_unfolded_states_are_eigenstates(iop):
    U, tr, g0 = OPS[iop]
    s1 = _ibz_set(K1)
    u = osym.unfold_set(s1, U, tr, g0, A, GRID, *_atom_map(U), _dblocks(U), OFFSETS)
    k = u.kpt
    # not the same k (the operation moves the point)
    assert np.linalg.norm(k - K1) > 0.05
    miller, e, _, H = _states(k)
    # the unfolded coefficients live on the plane-wave sphere at k
    idx = {tuple(m): i for i, m in enumerate(u.miller)}
    sel = np.array([idx[tuple(m)] for m in miller])
    rest = np.setdiff1d(np.arange(u.miller.shape[0]), sel)
    assert np.max(np.abs(u.C[:, rest])) < 1e-12
    c = u.C[:, sel]
    assert np.allclose(np.sum(np.abs(c) ** 2, axis=1), 1.0, atol=1e-12)
    resid = H @ c.T - c.T * s1.eps[None, :]
    assert np.max(np.abs(resid)) < 1e-10
    assert np.allclose(e[:NB], s1.eps, atol=1e-10)


@pytest.mark.parametrize("iop", range(len(OPS)))
def test_rotated_projections_equal_direct(iop):
    U, tr, g0 = OPS[iop]
    s1 = _ibz_set(K1)
    amap, shift = _atom_map(U)
    u = osym.unfold_set(s1, U, tr, g0, A, GRID, amap, shift, _dblocks(U), OFFSETS)
    direct = u.C @ _proj_table(u.kpt, u.miller)
    assert np.max(np.abs(u.P - direct)) < 1e-11 * np.max(np.abs(direct))


def _qtable(q, gm):
    """Q^a_ij(q+G) = s_ij e^{-|K|^2 s^2/2} e^{-i K.R_a}, s = diag(s0, s1, s1, s1): invariant under every
    operation (the p block is a multiple of the identity)."""
    B = oracle.reciprocal_rows(A)
    K = oracle.cartesian(gm, B, q)
    g = np.exp(-0.5 * SIGMA ** 2 * oracle.sq_norm(K))
    s = np.diag([0.3, -0.1, -0.1, -0.1])
    rows = []
    for x in ATOMS:
        ph = g * np.exp(-1j * (K @ (x @ A)))
        for i in range(4):
            for j in range(4):
                rows.append(s[i, j] * ph)
    return np.array(rows)


@pytest.mark.parametrize("iop", [0, 1, 3, 5])
def test_chi0_from_unfolded_sets(iop):
    U, tr, g0 = OPS[iop]
    q = np.array([0.09, -0.05, 0.07]) * 2 * np.pi / L
    T = osym.cartesian_rotation(U, A)
    sgn = -1.0 if tr else 1.0
    k = sgn * T @ K1 + np.asarray(g0, dtype=float) @ oracle.reciprocal_rows(A)
    # k + q = sgn T k2 + G0
    k2 = sgn * (T.T @ (k + q - np.asarray(g0, dtype=float) @ oracle.reciprocal_rows(A)))
    s1, s2 = _ibz_set(K1), _ibz_set(k2)
    amap, shift = _atom_map(U)
    D = _dblocks(U)
    uk = osym.unfold_set(s1, U, tr, g0, A, GRID, amap, shift, D, OFFSETS)
    ukq = osym.unfold_set(s2, U, tr, g0, A, GRID, amap, shift, D, OFFSETS)
    assert np.allclose(uk.kpt, k, atol=1e-13) and np.allclose(ukq.kpt, k + q, atol=1e-13)
    dk, dkq = _ibz_set(k), _ibz_set(k + q)
    gm = oracle.gsphere(A, q, 1.2)
    assert 10 < len(gm) < 60
    Q = _qtable(q, gm)
    omega = np.array([0.3, 1.1])
    chi_u = oracle.chi0_q(A, GRID, [uk], [ukq], gm, Q, OFFSETS, omega)
    chi_d = oracle.chi0_q(A, GRID, [dk], [dkq], gm, Q, OFFSETS, omega)
    assert np.max(np.abs(chi_u - chi_d)) < 1e-11 * np.max(np.abs(chi_d))
    # the PAW term matters here (it is not a small correction that a wrong phase could hide under)
    chi_0 = oracle.chi0_q(A, GRID, [uk], [ukq], gm, 0 * Q, OFFSETS, omega)
    assert np.max(np.abs(chi_0 - chi_d)) > 1e-3 * np.max(np.abs(chi_d))


def _all_pins():
    test_symmetric_model_is_symmetric()
    for i in range(len(OPS)):
        test_unfolded_states_are_eigenstates(i)
        test_rotated_projections_equal_direct(i)
    for i in (0, 1, 3, 5):
        test_chi0_from_unfolded_sets(i)


_orig_orb = osym.unfold_orbitals
_orig_rot = osym.rotate_projections


def _inv(U):
    return np.rint(np.linalg.inv(U)).astype(int)


def _dT(D, offsets):
    out = np.array(D, dtype=float)
    o = 0
    for a in range(len(offsets) - 1):
        n = offsets[a + 1] - offsets[a]
        out[o:o + n * n] = out[o:o + n * n].reshape(n, n).T.reshape(-1)
        o += n * n
    return out


MUTANTS = {
    "remap by U instead of U^-1": ("unfold_orbitals", lambda phi, U, tr, g0, grid: _orig_orb(phi, _inv(U), tr, g0, grid)),
    "time reversal without conjugation": ("unfold_orbitals", lambda phi, U, tr, g0, grid: _orig_orb(phi, U, 0, g0, grid)),
    "G0 phase of the wrong sign": ("unfold_orbitals",
                                  lambda phi, U, tr, g0, grid: _orig_orb(phi, U, tr, -np.asarray(g0), grid)),
    "D transposed": ("rotate_projections", lambda P, off, am, sh, D, k1, A_, tr: _orig_rot(P, off, am, sh, _dT(D, off), k1,
                                                                                          A_, tr)),
    "Bloch phase dropped": ("rotate_projections",
                            lambda P, off, am, sh, D, k1, A_, tr: _orig_rot(P, off, am, 0 * np.asarray(sh), D, k1, A_, tr)),
    "projections not conjugated under time reversal": ("rotate_projections",
                                                        lambda P, off, am, sh, D, k1, A_, tr: _orig_rot(P, off, am, sh, D,
                                                                                                       k1, A_, 0)),
    "atom map inverted": ("rotate_projections",
                          lambda P, off, am, sh, D, k1, A_, tr: _orig_rot(P, off, np.argsort(am), sh, D, k1, A_, tr)),
}


def test_unmutated_pins_pass():
    _all_pins()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_unfolding_mistake_is_caught(monkeypatch, name):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(osym, attr, fn)
    with pytest.raises(AssertionError):
        _all_pins()
