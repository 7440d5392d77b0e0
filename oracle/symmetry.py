"""FP64 reference of the symmetry unfolding IBZ -> BZ (Eq. kmap, Eq. trans_wfs; Table 1 steps 4 and 7).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading R15 (conventions the paper leaves to the crystal-symmetry code)
-----------------------------------------------------------------------
* A point operation T acts on fractional real-space coordinates as x -> U x with U an integer 3x3
  matrix (r = sum_i x_i a_i, so T = A^T U A^-T as a Cartesian matrix, which must be orthogonal).
* Eq. kmap: the Brillouin-zone point is k = (-1)^s T k1 + G0, k1 in the irreducible zone, s = 1 when
  time reversal is used, G0 = sum_i g0_i b_i a reciprocal lattice vector chosen by the caller.
* Eq. trans_wfs: psi_nk(r) = psi_nk1(T^-1 r), complex conjugated when s = 1. In terms of the periodic
  parts that the path works with, u_nk(r) = e^{-i G0.r} [conj] u_nk1(T^-1 r).
* Table 1 step 7 (projections at k outside the irreducible zone, from rotated projector functions):
  with T^-1 R_a = R_b + L_a (atom b, lattice vector L_a) and real projector functions that transform as
  p^a_i(T y) = sum_j D^a_ij p^a_j(y) (D^a: the rotation of the atom's angular channels, supplied with
  the operation),
      P^a_nk,i = e^{i k1.L_a} sum_j D^a_ij P^b_nk1,j        (s = 0)
  and its complex conjugate for s = 1 (the projector functions are real). Atoms a and b are of one
  species, so they carry the same number of projectors.

The orbital transform is taken on the real-space grid, as the paper does it (the grid point
T^-1 r_j is another grid point when U maps the grid onto itself); the unfolded set is returned with
coefficients on every grid frequency (the DFT of the transformed orbitals), so no rotated plane-wave
sphere is formed here.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.fft as sfft

from .rpa import orbitals, reciprocal_rows


def cartesian_rotation(U, A):
    """Cartesian matrix of the operation x -> U x on fractional coordinates: r = A^T x -> A^T U x."""
    A = np.asarray(A, dtype=np.float64)
    return A.T @ np.asarray(U, dtype=np.float64) @ np.linalg.inv(A.T)


def transformed_k(k1, U, A, time_reversal, g0):
    """Eq. kmap: k = (-1)^s T k1 + G0 (Cartesian)."""
    T = cartesian_rotation(U, A)
    s = -1.0 if time_reversal else 1.0
    return s * (T @ np.asarray(k1, dtype=np.float64)) + np.asarray(g0, dtype=np.float64) @ reciprocal_rows(A)


def unfold_orbitals(phi, U, time_reversal, g0, grid):
    """Eq. trans_wfs on the grid: u_k(r_j) = e^{-i G0.r_j} [conj] u_k1(T^-1 r_j).

    phi: complex [nb, N1, N2, N3], point j at fractional x_j = j / N. T^-1 r_j has fractional
    coordinates U^-1 x_j; its grid index is N * U^-1 (j / N) mod N, which must be integral.
    """
    N = np.asarray(grid, dtype=np.int64)
    Ui = np.rint(np.linalg.inv(np.asarray(U, dtype=np.float64))).astype(np.int64)
    assert np.array_equal(Ui @ np.asarray(U, dtype=np.int64), np.eye(3, dtype=np.int64)), "U not unimodular"
    j = np.stack(np.meshgrid(*[np.arange(n) for n in grid], indexing="ij"), axis=-1).reshape(-1, 3)
    # source index of each point: N_c * sum_d Ui[c, d] j_d / N_d, exactly integral for a grid-preserving U
    num = np.zeros_like(j)
    src = np.zeros_like(j)
    for c in range(3):
        acc = np.zeros(j.shape[0], dtype=np.int64)
        den = 1
        for d in range(3):
            den = np.lcm(den, int(N[d]))
        for d in range(3):
            acc += Ui[c, d] * j[:, d] * (den // N[d])
        num[:, c] = acc * N[c]
        assert np.all(num[:, c] % den == 0), "U does not map the grid onto itself"
        src[:, c] = np.mod(num[:, c] // den, N[c])
    out = phi[:, src[:, 0], src[:, 1], src[:, 2]]
    if time_reversal:
        out = np.conj(out)
    x = j / N
    out = out * np.exp(-2j * np.pi * (x @ np.asarray(g0, dtype=np.float64)))[None, :]
    return out.reshape(phi.shape)


def grid_coefficients(phi, grid):
    """C(m) = (1/N) sum_j u(r_j) e^{-2 pi i m.j/N} for every grid frequency m in [-N/2, N/2) per axis:
    the inverse of `orbitals` on the whole grid. Returns (C [nb, N], miller [N, 3])."""
    nb = phi.shape[0]
    ntot = int(np.prod(grid))
    F = sfft.fftn(phi, axes=(1, 2, 3), workers=-1) / ntot
    axes = [np.fft.fftfreq(n, 1.0 / n).astype(np.int64) for n in grid]
    m = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    return F.reshape(nb, -1), m.astype(np.int32)


def rotate_projections(P, offsets, atom_map, atom_shift, D, k1, A, time_reversal):
    """Table 1 step 7: P^a_nk,i = e^{i k1.L_a} sum_j D^a_ij P^b_nk1,j (conjugated for time reversal).

    P: [nb, sum Np] at k1; offsets: [natoms+1]; atom_map[a] = b, atom_shift[a] = L_a (lattice units,
    T^-1 R_a = R_b + L_a); D: flat [sum_a Np_a^2], block of atom a row-major (i, j); k1 Cartesian.
    """
    P = np.asarray(P)
    out = np.empty_like(P)
    A = np.asarray(A, dtype=np.float64)
    doff = 0
    for a in range(len(offsets) - 1):
        lo, hi = offsets[a], offsets[a + 1]
        npa = hi - lo
        b = int(atom_map[a])
        blo, bhi = offsets[b], offsets[b + 1]
        assert bhi - blo == npa, "atoms of one orbit carry the same projectors"
        Da = np.asarray(D[doff:doff + npa * npa], dtype=np.float64).reshape(npa, npa)
        doff += npa * npa
        L = np.asarray(atom_shift[a], dtype=np.float64) @ A
        phase = np.exp(1j * float(np.dot(k1, L)))
        blk = phase * (P[:, blo:bhi] @ Da.T)
        out[:, lo:hi] = np.conj(blk) if time_reversal else blk
    return out


def unfold_set(s, U, time_reversal, g0, A, grid, atom_map, atom_shift, D, offsets):
    """The state set at k = (-1)^s T k1 + G0 from the set `s` at k1 (Eq. kmap, Eq. trans_wfs, Table 1
    steps 4 and 7). The returned set carries the same eigenvalues, occupations and weight, the
    coefficients of the transformed orbitals on every grid frequency, and the rotated projections."""
    phi = orbitals(s.C, s.miller, grid)
    phi_k = unfold_orbitals(phi, U, time_reversal, g0, grid)
    C, miller = grid_coefficients(phi_k, grid)
    P = rotate_projections(s.P, offsets, atom_map, atom_shift, D, s.kpt, A, time_reversal) \
        if s.P.shape[1] else s.P.copy()
    return dataclasses.replace(s, C=C, miller=miller, P=P, kpt=transformed_k(s.kpt, U, A, time_reversal, g0))
