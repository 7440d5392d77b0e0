"""Planted mistakes in the oracle's spin, intraband-head and real-frequency parts (readings R12-R14), on the
CPU: each case replaces one oracle function with a plausible wrong variant and checks that the pin written
for that part fails. The unmutated pins pass in their own modules.
"""
import numpy as np
import pytest

import oracle
import oracle.rpa as R
import test_oracle_intraband as intraband_pins
import test_oracle_realfreq as realfreq_pins
import test_oracle_spin as spin_pins

_weights = R.transition_weights
_weights_real = R.transition_weights_real
_head = R.intraband_head
_velocity = R.band_velocity
_chi0_q = R.chi0_q


def _patch(monkeypatch, name, fn):
    monkeypatch.setattr(R, name, fn)
    monkeypatch.setattr(oracle, name, fn)


# --- spin (R12): channels of f in [0, 1]
def _weights_spin_doubled(eps_k, eps_kq, f_k, f_kq, pairs, w_k, volume, omega):
    """A spin factor of 2 applied to channels that already carry one spin each."""
    a = _weights(eps_k, eps_kq, f_k, f_kq, pairs, w_k, volume, omega)
    return 2.0 * a if max(np.max(f_k), np.max(f_kq)) <= 1.0 else a


def _chi0_first_channel(A, grid, ksets, kqsets, *args, **kw):
    """Only the first state set (spin channel) summed."""
    return _chi0_q(A, grid, ksets[:1], kqsets[:1], *args, **kw)


# --- intraband head (R13)
def _head_over_w(sets, A, Dtab, offsets, qhat, omega):
    return _head(sets, A, Dtab, offsets, qhat, omega) * np.asarray(omega)


def _head_doubled(sets, A, Dtab, offsets, qhat, omega):
    return 2.0 * _head(sets, A, Dtab, offsets, qhat, omega)


def _head_sign(sets, A, Dtab, offsets, qhat, omega):
    return -_head(sets, A, Dtab, offsets, qhat, omega)


def _velocity_without_k(C_k, miller_k, kpt, A, P_k, Dtab, offsets, qhat):
    """The band velocity from G_Q alone (k dropped from the momentum)."""
    return _velocity(C_k, miller_k, np.zeros(3), A, P_k, Dtab, offsets, qhat)


# --- real frequencies (R14)
def _weights_real_resonant_only(eps_k, eps_kq, f_k, f_kq, pairs, w_k, volume, omega, eta):
    n, m = pairs
    d = (np.asarray(eps_k)[n] - np.asarray(eps_kq)[m])[:, None]
    df = (np.asarray(f_k)[n] - np.asarray(f_kq)[m])[:, None]
    z = np.asarray(omega, dtype=np.float64)[None, :] + 1j * eta
    return (w_k / volume) * df * (1.0 / (z + d))


def _weights_real_eta_sign(eps_k, eps_kq, f_k, f_kq, pairs, w_k, volume, omega, eta):
    return _weights_real(eps_k, eps_kq, f_k, f_kq, pairs, w_k, volume, omega, -eta)


def _weights_real_conjugated(eps_k, eps_kq, f_k, f_kq, pairs, w_k, volume, omega, eta):
    return np.conj(_weights_real(eps_k, eps_kq, f_k, f_kq, pairs, w_k, volume, omega, eta))


CASES = [
    ("transition_weights", _weights_spin_doubled, spin_pins.test_two_channel_closed_form),
    ("chi0_q", _chi0_first_channel, spin_pins.test_spin_unpolarised_limit),
    ("intraband_head", _head_over_w, intraband_pins.test_intraband_head_is_the_small_q_limit),
    ("intraband_head", _head_doubled, intraband_pins.test_intraband_head_is_the_small_q_limit),
    ("intraband_head", _head_sign, intraband_pins.test_intraband_head_is_the_small_q_limit),
    ("band_velocity", _velocity_without_k, intraband_pins.test_intraband_head_is_the_small_q_limit),
    ("transition_weights_real", _weights_real_resonant_only,
     realfreq_pins.test_zero_frequency_continues_to_the_imaginary_axis),
    ("transition_weights_real", _weights_real_eta_sign,
     realfreq_pins.test_negative_frequency_is_the_adjoint_and_absorption_sign),
    ("transition_weights_real", _weights_real_conjugated, realfreq_pins.test_one_transition_written_out),
]


@pytest.mark.parametrize("name,bad,pin", CASES, ids=[f"{c[0]}:{i}" for i, c in enumerate(CASES)])
def test_planted_mistake_is_caught(monkeypatch, name, bad, pin):
    _patch(monkeypatch, name, bad)
    with pytest.raises(AssertionError):
        pin()
