"""Planted mistakes in the oracle (on the CPU) must make at least one pin fail.

Each case replaces one oracle function with a plausible wrong variant (a dropped
factor, a flipped sign, a conjugate on the wrong operand, a transposed index)
and checks that the pin written for that step catches it.
"""
import numpy as np
import pytest
import scipy.fft as sfft

import oracle
import oracle.rpa as R
import test_oracle_optical as optical_pins
import test_oracle_pins as pins


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(R, name, fn)
    monkeypatch.setattr(oracle, name, fn)


def _weights_no_factor_two(eps_k, eps_kq, f_k, f_kq, pairs, w_k, volume, omega):
    n, m = pairs
    d = np.asarray(eps_k)[n] - np.asarray(eps_kq)[m]
    df = np.asarray(f_k)[n] - np.asarray(f_kq)[m]
    w = np.asarray(omega)[None, :]
    return (w_k / volume) * df[:, None] * d[:, None] / (w * w + d[:, None] ** 2)


def _pair_density_wrong_sign(phi_k, phi_kq, pairs, gmiller, grid, batch=64):
    n_idx, m_idx = pairs
    ntot = grid[0] * grid[1] * grid[2]
    i1, i2, i3 = R.grid_index(gmiller, grid)
    prod = np.conj(phi_k[n_idx]) * phi_kq[m_idx]
    spec = sfft.ifftn(prod, axes=(1, 2, 3)) * ntot
    return spec[:, i1, i2, i3] / ntot


def _paw_conj_on_wrong_side(P_k, P_kq, pairs, Qtab, offsets):
    n_idx, m_idx = pairs
    out = np.zeros((n_idx.size, Qtab.shape[1]), dtype=np.complex128)
    qoff = 0
    for a in range(len(offsets) - 1):
        lo, hi = offsets[a], offsets[a + 1]
        npj = hi - lo
        Qa = Qtab[qoff:qoff + npj * npj].reshape(npj, npj, -1)
        qoff += npj * npj
        out += np.einsum("pi,pj,ijg->pg", P_k[n_idx][:, lo:hi], np.conj(P_kq[m_idx][:, lo:hi]), Qa)
    return out


def _paw_transposed(P_k, P_kq, pairs, Qtab, offsets):
    n_idx, m_idx = pairs
    out = np.zeros((n_idx.size, Qtab.shape[1]), dtype=np.complex128)
    qoff = 0
    for a in range(len(offsets) - 1):
        lo, hi = offsets[a], offsets[a + 1]
        npj = hi - lo
        Qa = Qtab[qoff:qoff + npj * npj].reshape(npj, npj, -1)
        qoff += npj * npj
        out += np.einsum("pi,pj,jig->pg", np.conj(P_k[n_idx][:, lo:hi]), P_kq[m_idx][:, lo:hi], Qa)
    return out


def _coulomb_no_sqrt(A, q, gmiller, optical=False):
    B = R.reciprocal_rows(A)
    k = np.sqrt(R.sq_norm(R.cartesian(gmiller, B, q)))
    k[k == 0] = 1.0
    return R.FOUR_PI / k ** 2


def _integrand_dropped_trace(chi, vsqrt):
    K = R.kernel_matrix(chi, vsqrt)
    return np.array([np.sum(np.log1p(-np.linalg.eigvalsh(k))) for k in K])


def _grid_no_jacobian(n, w0=1.0):
    t, w = R.gauss_legendre(n)
    x = 0.5 * (t + 1.0)
    return w0 * x / (1.0 - x), 0.5 * w * w0


def _orbitals_conjugated(C, miller, grid):
    return np.conj(sfft.fftn(_place(C, miller, grid), axes=(1, 2, 3)))


def _place(C, miller, grid):
    box = np.zeros((C.shape[0],) + tuple(grid), dtype=np.complex128)
    i1, i2, i3 = R.grid_index(miller, grid)
    box[:, i1, i2, i3] = C
    return box


def _chi0_missing_conj(rho, a, group=None):
    nw = a.shape[1]
    return np.stack([(rho.T * a[:, w][None, :]) @ rho for w in range(nw)])


def _head_variant(paw_sign=-1.0, conj=False, flip_denominator=False, transpose_d=False):
    def head(C_k, miller_k, kpt, A, P_k, Dtab, offsets, eps, pairs, qhat):
        n_idx, m_idx = pairs
        pseudo = R.momentum_pw(C_k, miller_k, kpt, A, pairs, qhat)
        Dq = np.tensordot(np.asarray(qhat, dtype=np.float64), Dtab, axes=(0, 0))
        paw = np.zeros(n_idx.size, dtype=np.complex128)
        qoff = 0
        for a in range(len(offsets) - 1):
            lo, hi = offsets[a], offsets[a + 1]
            npj = hi - lo
            Da = Dq[qoff:qoff + npj * npj].reshape(npj, npj)
            qoff += npj * npj
            if transpose_d:
                Da = Da.T
            paw += np.einsum("pi,ij,pj->p", np.conj(P_k[n_idx][:, lo:hi]), Da, P_k[m_idx][:, lo:hi])
        de = np.asarray(eps)[m_idx] - np.asarray(eps)[n_idx]
        if flip_denominator:
            de = -de
        out = (pseudo + paw_sign * 1j * paw) / de
        return np.conj(out) if conj else out
    return head


def _gsphere_strict(A, q, ecut):
    return ORIG_GSPHERE(A, q, ecut * 0.97)


ORIG_GSPHERE = R.gsphere

CASES = [
    ("transition_weights", _weights_no_factor_two, lambda: pins.test_two_level_closed_form(False, 64)),
    ("pseudo_pair_density", _pair_density_wrong_sign, lambda: pins.test_pair_density_equals_direct_dft((6, 8, 10))),
    ("paw_correction", _paw_conj_on_wrong_side, pins.test_paw_correction_matches_separable_closed_form),
    ("paw_correction", _paw_transposed, pins.test_paw_correction_factorises_for_rank_one_table),
    ("coulomb_sqrt", _coulomb_no_sqrt, lambda: pins.test_two_level_closed_form(False, 64)),
    ("integrand", _integrand_dropped_trace, pins.test_integrand_three_ways_and_sign),
    ("frequency_grid", _grid_no_jacobian, pins.test_mapped_rule_integrates_lorentzian),
    ("orbitals", _orbitals_conjugated, pins.test_orbitals_equal_direct_plane_wave_sum),
    ("chi0_grouped", _chi0_missing_conj, pins.test_chi0_hermitian_negative_semidefinite_and_gauge_invariant),
    ("gsphere", _gsphere_strict, pins.test_gsphere_matches_python_enumeration),
    ("optical_head", _head_variant(conj=True), optical_pins.test_pseudo_head_is_the_kp_limit_of_the_pair_density),
    ("optical_head", _head_variant(flip_denominator=True),
     optical_pins.test_pseudo_head_is_the_kp_limit_of_the_pair_density),
    ("optical_head", _head_variant(paw_sign=+1.0), optical_pins.test_paw_head_equals_the_all_electron_head),
    ("optical_head", _head_variant(transpose_d=True), optical_pins.test_paw_head_equals_the_all_electron_head),
]


def test_unmutated_head_variant_passes_both_head_pins(monkeypatch):
    """The reference form of the mutated head (every switch off) passes, so the cases above fail only
    through their planted mistake."""
    _patch(monkeypatch, "optical_head", _head_variant())
    optical_pins.test_pseudo_head_is_the_kp_limit_of_the_pair_density()
    optical_pins.test_paw_head_equals_the_all_electron_head()


@pytest.mark.parametrize("name,bad,pin", CASES, ids=[f"{c[0]}:{i}" for i, c in enumerate(CASES)])
def test_planted_mistake_is_caught(monkeypatch, name, bad, pin):
    _patch(monkeypatch, name, bad)
    with pytest.raises(AssertionError):
        pin()
