"""Seeded synthetic workloads shaped after the paper's five systems (Table 5) and
its timing workload (Table 2): cells, grids, plane-wave states, eigenvalues,
occupations, PAW projections, synthetic PAW tables, q-points and the imaginary
frequency grid.

This module holds inputs only. It draws random numbers and lays out the
problem; it evaluates none of the response-function arithmetic (no pair
densities, no chi0, no weights, no log-determinants). Both the CPU oracle and
the GPU library receive exactly the arrays produced here.

Conventions
-----------
* Hartree atomic units (bohr, Ha).
* Lattice rows ``A[i]`` are the cell vectors a_i; reciprocal rows satisfy
  a_i . b_j = 2 pi delta_ij.
* Miller triples m give G = m1 b1 + m2 b2 + m3 b3; on an N-point axis an index
  m maps to grid position m mod N.
* Plane-wave coefficients C_n(Q) multiply e^{i (k+G_Q).r} with no 1/sqrt(Omega);
  the states are orthonormal (under the PAW overlap in the default model,
  plainly in the "independent" model; see below).
* PAW projections are stored per band as one row over all atoms,
  ``P[n, off[a] + i]`` = <p~_i^a | psi~_n>.
* Two projection models:
  - "overlap" (default): the projections are a linear map of the
    coefficients, P = C Pi, with Pi[Q, off_a + i] an atom-centred projector in
    plane-wave space (smooth envelope times e^{i (k+Q).R_a}), and the states
    are orthonormal under the PAW overlap
    1 + sum_a Pi_a s^a Pi_a^H, i.e.
    sum_Q C_n^* C_m + sum_a sum_ij conj(P_ni) s^a_ij P_mj = delta_nm.
    This is what the all-electron normalisation of Sec. 2.2 asks of the pair
    density at q = 0, G = 0, given Q^a_ij(0) = s^a_ij.
  - "independent" (stress workload): C orthonormal on its own and P drawn
    independently, Re and Im ~ N(0, 0.1). The full pair density at G -> 0 then
    carries sum_a P^* s P for n != m, which the Coulomb head amplifies.
* Q^a_ij(K) (the augmentation form factor of the PAW pair density) needs
  partial waves that are not available, so a separable Gaussian model stands
  in: Q^a_ij(K) = s^a_ij exp(-|K|^2 sigma^2 / 2) e^{-i K.R_a}, s^a real
  symmetric. The nabla analogue D^a (used only in the q -> 0 limit) is real
  antisymmetric per Cartesian direction.
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import List, Optional, Sequence

import numpy as np
import scipy.linalg as scipy_linalg

TWO_PI = 2.0 * np.pi


# ----------------------------------------------------------------------------
# geometry helpers (input layout only)
# ----------------------------------------------------------------------------
def reciprocal_rows(A: np.ndarray) -> np.ndarray:
    """Rows b_i with a_i . b_j = 2 pi delta_ij."""
    return TWO_PI * np.linalg.inv(np.asarray(A, dtype=np.float64)).T


def cart(miller: np.ndarray, B: np.ndarray, shift=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Cartesian shift + m1 b1 + m2 b2 + m3 b3, summed in a fixed order."""
    m = np.asarray(miller, dtype=np.float64)
    out = np.empty(m.shape[:-1] + (3,))
    for c in range(3):
        out[..., c] = shift[c] + m[..., 0] * B[0, c] + m[..., 1] * B[1, c] + m[..., 2] * B[2, c]
    return out


def _box(mmax: Sequence[int]) -> np.ndarray:
    r = [np.arange(-int(M), int(M) + 1) for M in mmax]
    g = np.stack(np.meshgrid(*r, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.int32)


def _sphere_box(A, radius: float, shift) -> np.ndarray:
    """Every Miller triple whose |shift + G| could be <= radius."""
    # |m_i| <= (radius + |shift|) * |a_i| / (2 pi)
    a_len = np.linalg.norm(np.asarray(A, dtype=np.float64), axis=1)
    s = float(np.linalg.norm(shift))
    mmax = np.floor((radius + s) * a_len / TWO_PI).astype(int) + 1
    return _box(mmax)


def sphere_sq_lengths(A, shift, radius):
    B = reciprocal_rows(A)
    m = _sphere_box(A, radius, shift)
    k = cart(m, B, shift)
    k2 = k[:, 0] * k[:, 0] + k[:, 1] * k[:, 1] + k[:, 2] * k[:, 2]
    return m, k2


def ecut_for_count(A, q, target: int) -> float:
    """Smallest chi cutoff whose sphere |q+G|^2/2 <= Ecut holds >= target vectors.

    The value returned is the midpoint between that shell and the next one, so
    the sphere it selects does not depend on rounding at the boundary.
    """
    radius = 1.0
    while True:
        m, k2 = sphere_sq_lengths(A, q, radius)
        inside = np.sort(k2[k2 <= radius * radius])
        if inside.size > target + 64:
            break
        radius *= 1.3
    st = inside[target - 1]
    above = inside[inside > st * (1 + 1e-12) + 1e-14]
    snext = above[0]
    return 0.25 * (st + snext)


def wavefunction_sphere(A, kpt, ecut_wf: float) -> np.ndarray:
    """Miller list of the plane-wave basis |k+Q|^2/2 <= ecut_wf, ordered by |k+Q| then lexicographically."""
    radius = np.sqrt(2.0 * ecut_wf)
    m, k2 = sphere_sq_lengths(A, kpt, radius)
    sel = k2 <= 2.0 * ecut_wf
    m, k2 = m[sel], k2[sel]
    order = np.lexsort((m[:, 2], m[:, 1], m[:, 0], k2))
    return np.ascontiguousarray(m[order], dtype=np.int32)


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class StateSet:
    """One k (or k+q) state set."""
    kpt: np.ndarray          # (3,) Cartesian, bohr^-1
    weight: float            # w_k (1/N_k)
    miller: np.ndarray       # int32 [NQ, 3]
    C: np.ndarray            # complex128 [nb, NQ]; states orthonormal (see the module docstring)
    eps: np.ndarray          # float64 [nb], ascending
    f: np.ndarray            # float64 [nb], in [0, 2], non-increasing
    P: np.ndarray            # complex128 [nb, sum Np]
    dfde: Optional[np.ndarray] = None   # float64 [nb], -df/d eps (Fermi-smeared sets), else None

    @property
    def nbands(self):
        return self.C.shape[0]


@dataclasses.dataclass
class Paw:
    nproj: List[int]         # Np per atom
    s: List[np.ndarray]      # real symmetric (Np, Np) per atom
    R: np.ndarray            # (Na, 3) Cartesian positions
    D: List[np.ndarray]      # real (3, Np, Np), antisymmetric per direction
    sigma: float = 0.5

    @property
    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.nproj)]).astype(np.int32)

    @property
    def qoffsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum([n * n for n in self.nproj])]).astype(np.int32)


@dataclasses.dataclass
class QPoint:
    q: np.ndarray            # (3,) Cartesian
    ecut: float              # chi cutoff (Ha); sphere |q+G|^2/2 <= ecut
    weight: float = 1.0      # w_q
    optical: bool = False    # q -> 0 limit along qhat
    qhat: np.ndarray = dataclasses.field(default_factory=lambda: np.array([1.0, 0.0, 0.0]))


@dataclasses.dataclass
class Workload:
    name: str
    A: np.ndarray            # (3, 3) lattice rows (bohr)
    grid: tuple              # (N1, N2, N3)
    kpoints: List[StateSet]  # state sets at k; k+q uses the same set (see below)
    paw: Paw
    qpoints: List[QPoint]
    omega: np.ndarray        # [nw] imaginary frequencies (Ha)
    omega_weight: np.ndarray # [nw] quadrature weights for d omega
    seed: int
    kq: Optional[List[StateSet]] = None   # distinct k+q sets; None -> same as kpoints

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.A)))

    def kq_sets(self) -> List[StateSet]:
        return self.kq if self.kq is not None else self.kpoints

    def digest(self) -> str:
        h = hashlib.sha256()
        for s in self.kpoints + (self.kq or []):
            for arr in (s.miller, s.C, s.eps, s.f, s.P):
                h.update(np.ascontiguousarray(arr).tobytes())
        h.update(np.ascontiguousarray(self.omega).tobytes())
        return h.hexdigest()[:16]


# ----------------------------------------------------------------------------
# draws
# ----------------------------------------------------------------------------
def orthonormal_coefficients(rng, A, kpt, miller, nb):
    """Re, Im ~ N(0,1) x exp(-|k+Q|^2/8), then orthonormal rows by QR with diag(R) > 0."""
    B = reciprocal_rows(A)
    kq = cart(miller, B, kpt)
    env = np.exp(-(kq[:, 0] ** 2 + kq[:, 1] ** 2 + kq[:, 2] ** 2) / 8.0)
    NQ = miller.shape[0]
    if nb > NQ:
        raise ValueError(f"{nb} bands need at least as many plane waves (have {NQ})")
    X = (rng.standard_normal((nb, NQ)) + 1j * rng.standard_normal((nb, NQ))) * env[None, :]
    Qm, R = np.linalg.qr(X.T)            # X^T = Qm R, Qm: NQ x nb
    d = np.diag(R)
    ph = d / np.abs(d)
    Qm = Qm * ph[None, :]
    return np.ascontiguousarray(Qm.T)


def gapped_levels(rng, n_occ, n_unocc, occ_range=(-0.8, -0.3), unocc_range=(0.0, 3.0), fmax=2.0):
    """Sorted levels, f = fmax below the gap (2: both spins in one set; 1: one spin channel)."""
    eo = np.sort(rng.uniform(occ_range[0], occ_range[1], n_occ))
    eu = np.sort(rng.uniform(unocc_range[0], unocc_range[1], n_unocc))
    eps = np.concatenate([eo, eu])
    f = np.concatenate([np.full(n_occ, float(fmax)), np.zeros(n_unocc)])
    return eps, f


def fermi_levels(rng, n_below, n_above, T=0.01, mu=0.0, fmax=2.0):
    """Sorted levels around mu with Fermi-Dirac occupations f = fmax/(1 + e^{(eps - mu)/T})."""
    eb = np.sort(rng.uniform(-0.8, 0.0, n_below))
    ea = np.sort(rng.uniform(0.0, 3.0, n_above))
    eps = np.concatenate([eb, ea])
    x = np.clip((eps - mu) / T, -700.0, 700.0)
    f = float(fmax) / (1.0 + np.exp(x))
    return eps, f


def raw_coefficients(rng, A, kpt, miller, nb):
    """Re, Im ~ N(0,1) x exp(-|k+Q|^2/8), not yet orthonormal; [nb, NQ]."""
    B = reciprocal_rows(A)
    kq = cart(miller, B, kpt)
    env = np.exp(-(kq[:, 0] ** 2 + kq[:, 1] ** 2 + kq[:, 2] ** 2) / 8.0)
    NQ = miller.shape[0]
    if nb > NQ:
        raise ValueError(f"{nb} bands need at least as many plane waves (have {NQ})")
    # same draws as (N + 1j N) * env, built in place (no large temporaries)
    X = np.empty((nb, NQ), dtype=np.complex128)
    X.real = rng.standard_normal((nb, NQ))
    X.imag = rng.standard_normal((nb, NQ))
    X *= env[None, :]
    return X


def projector_map(rng, A, kpt, miller, paw, overlap_spread=0.5):
    """Pi[Q, off_a + i] = beta z_Qi exp(-|k+Q|^2/8) e^{i (k+Q).R_a}, z_Qi complex N(0,1), each column
    scaled to unit norm, then all columns by one beta chosen so that the eigenvalues of the overlap
    1 + sum_a Pi_a s^a Pi_a^H lie in [1 - overlap_spread, 1 + overlap_spread]; [NQ, sum Np]."""
    B = reciprocal_rows(A)
    kq = cart(miller, B, kpt)
    env = np.exp(-(kq[:, 0] ** 2 + kq[:, 1] ** 2 + kq[:, 2] ** 2) / 8.0)
    NQ = miller.shape[0]
    off = paw.offsets
    tot = int(off[-1])
    Z = rng.standard_normal((NQ, tot)) + 1j * rng.standard_normal((NQ, tot))
    Pi = Z * env[:, None]
    for a in range(len(paw.nproj)):
        Pi[:, off[a]:off[a + 1]] *= np.exp(1j * (kq @ paw.R[a]))[:, None]
    Pi /= np.linalg.norm(Pi, axis=0)[None, :]
    # the nonzero eigenvalues of Pi S Pi^H (S = blockdiag s^a) are those of G^1/2 S G^1/2, G = Pi^H Pi
    S = np.zeros((tot, tot))
    for a, n in enumerate(paw.nproj):
        S[off[a]:off[a + 1], off[a]:off[a + 1]] = paw.s[a]
    G = Pi.conj().T @ Pi
    w, V = np.linalg.eigh(G)
    Gh = (V * np.sqrt(np.maximum(w, 0.0))[None, :]) @ V.conj().T
    lam = np.linalg.eigvalsh(Gh @ S @ Gh)
    beta = np.sqrt(overlap_spread / max(np.max(np.abs(lam)), 1e-300))
    return np.ascontiguousarray(beta * Pi)


def paw_orthonormal_states(C0, Pi, paw, device=None):
    """Gram-Schmidt of the rows of C0 under the PAW overlap: returns (C, P) with P = C Pi and
    sum_Q C_n^* C_m + sum_a sum_ij conj(P_ni) s^a_ij P_mj = delta_nm (positive diagonal of the
    triangular factor, the generalised form of QR with diag(R) > 0).

    device: None for numpy on the host; a torch device string (e.g. "cuda:0") to run the Gram matrix,
    its Cholesky factor and the triangular solves there in complex128 (same result up to rounding; for
    the large workloads, whose host generation takes minutes)."""
    if device is not None:
        return _paw_orthonormal_states_torch(C0, Pi, paw, device)
    P0 = C0 @ Pi
    off = paw.offsets
    G = C0.conj() @ C0.T
    for a in range(len(paw.nproj)):
        Pa = P0[:, off[a]:off[a + 1]]
        G += Pa.conj() @ paw.s[a] @ Pa.T
    G = 0.5 * (G + G.conj().T)
    M = np.linalg.cholesky(G)                       # G = M M^H
    Mc = np.conj(M)
    C = scipy_linalg.solve_triangular(Mc, C0, lower=True)
    P = scipy_linalg.solve_triangular(Mc, P0, lower=True)
    return np.ascontiguousarray(C), np.ascontiguousarray(P)


def _paw_orthonormal_states_torch(C0, Pi, paw, device):
    import torch
    c0 = torch.from_numpy(C0).to(device)
    pi = torch.from_numpy(np.ascontiguousarray(Pi)).to(device)
    p0 = c0 @ pi
    off = paw.offsets
    G = c0.conj() @ c0.T
    for a in range(len(paw.nproj)):
        pa = p0[:, off[a]:off[a + 1]]
        sa = torch.from_numpy(np.asarray(paw.s[a], dtype=np.complex128)).to(device)
        G += pa.conj() @ sa @ pa.T
    G = 0.5 * (G + G.conj().T)
    M = torch.linalg.cholesky(G)
    Mc = M.conj()

    def lower_solve(L, R):
        # forward substitution by row blocks: X_i = L_ii^-1 (R_i - L_i,<i X_<i), all matrix products
        X = torch.empty_like(R)
        bs = 256
        for i0 in range(0, L.shape[0], bs):
            i1 = min(L.shape[0], i0 + bs)
            rhs = R[i0:i1] - L[i0:i1, :i0] @ X[:i0] if i0 else R[i0:i1]
            X[i0:i1] = torch.linalg.inv(L[i0:i1, i0:i1]) @ rhs
        return X

    C = lower_solve(Mc, c0)
    P = lower_solve(Mc, p0)
    out = np.ascontiguousarray(C.cpu().numpy()), np.ascontiguousarray(P.cpu().numpy())
    del c0, pi, p0, G, M, Mc, C, P
    return out


def draw_projections(rng, nb, nproj_total):
    """P with Re, Im ~ N(0, 0.1) each."""
    return 0.1 * rng.standard_normal((nb, nproj_total)) + 0.1j * rng.standard_normal((nb, nproj_total))


def draw_paw(rng, A, nproj: Sequence[int]) -> Paw:
    s, D = [], []
    for n in nproj:
        Bm = rng.standard_normal((n, n))
        s.append(0.5 * (Bm + Bm.T))
    R = rng.uniform(0.0, 1.0, (len(nproj), 3)) @ np.asarray(A, dtype=np.float64)
    for n in nproj:
        Cm = rng.standard_normal((3, n, n))
        D.append(0.1 * 0.5 * (Cm - np.transpose(Cm, (0, 2, 1))))
    return Paw(nproj=list(nproj), s=s, R=R, D=D)


def frequency_grid(nw: int, w0: float = 1.0):
    """Gauss-Legendre nodes on [-1, 1] mapped to [0, inf) by omega = w0 x/(1-x), x = (t+1)/2.

    Returns (omega, weight) with weight = d omega per node, so that
    int_0^inf g(omega) d omega ~= sum_i weight_i g(omega_i).
    """
    t, w = np.polynomial.legendre.leggauss(nw)
    x = 0.5 * (t + 1.0)
    omega = w0 * x / (1.0 - x)
    weight = 0.5 * w * w0 / (1.0 - x) ** 2
    return omega, weight


# ----------------------------------------------------------------------------
# synthetic PAW tables evaluated on a caller-supplied G list
# ----------------------------------------------------------------------------
def paw_q_table(paw: Paw, A, q, gmiller) -> np.ndarray:
    """Q[qoff[a] + i*Np + j, G] = s^a_ij exp(-|q+G|^2 sigma^2/2) exp(-i (q+G).R_a), complex128."""
    B = reciprocal_rows(A)
    K = cart(gmiller, B, q)
    K2 = K[:, 0] ** 2 + K[:, 1] ** 2 + K[:, 2] ** 2
    g = np.exp(-0.5 * K2 * paw.sigma ** 2)
    rows = []
    for a, n in enumerate(paw.nproj):
        phase = np.exp(-1j * (K @ paw.R[a]))
        rows.append((paw.s[a].reshape(n * n, 1) * (g * phase)[None, :]))
    return np.ascontiguousarray(np.concatenate(rows, axis=0).astype(np.complex128))


def paw_d_table(paw: Paw) -> np.ndarray:
    """D[c, qoff[a] + i*Np + j] = D^a_c,ij (real), the PAW nabla correction."""
    cols = [paw.D[a].reshape(3, n * n) for a, n in enumerate(paw.nproj)]
    return np.ascontiguousarray(np.concatenate(cols, axis=1).astype(np.float64))


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------
def _assemble(name, A, grid, seed, kpts, kweights, levels, nproj, qpoints, nw,
              extra_kq=False, w0=1.0, paw_model="overlap", device=None):
    """Draw a workload from one seeded generator.

    paw_model "overlap" draws, in this order: per k the raw coefficients and the levels; s^a, R_a,
    D^a; per k the projector map Pi, then orthonormalises (C, P = C Pi) under the PAW overlap; then,
    with extra_kq, per set the raw coefficients and levels of a distinct k+q set (same Pi).
    paw_model "independent" draws C (orthonormal on its own), eps_occ, eps_unocc per k; then P per k;
    then s^a, R_a, D^a; then the distinct k+q sets (C, levels, P).
    """
    rng = np.random.default_rng(seed)
    A = np.asarray(A, dtype=np.float64)
    ecut_max = max(qp.ecut for qp in qpoints)
    ecut_wf = 4.0 * ecut_max
    nproj_total = int(sum(nproj))
    sets = []
    kq = None
    channels = levels if isinstance(levels, (list, tuple)) else [levels]
    if paw_model == "overlap":
        raw = []
        for ik, k in enumerate(kpts):
            miller = wavefunction_sphere(A, k, ecut_wf)
            for lev in channels:
                C0 = raw_coefficients(rng, A, k, miller, lev(None, dry=True))
                eps, f = lev(rng)
                raw.append((ik, k, kweights[ik], miller, C0, eps, f))
        paw = draw_paw(rng, A, nproj)
        pis = []
        pi_k = {}
        for i in range(len(raw)):
            ik, k, w, miller, C0, eps, f = raw[i]
            raw[i] = None                  # the raw draw is released once orthonormalised
            if ik not in pi_k:             # one projector map per k, shared by its spin channels
                pi_k[ik] = projector_map(rng, A, k, miller, paw)
            Pi = pi_k[ik]
            pis.append(Pi)
            C, P = paw_orthonormal_states(C0, Pi, paw, device)
            del C0
            lev = channels[i % len(channels)]
            dfde = lev.dfde(f) if hasattr(lev, "dfde") else None
            sets.append(StateSet(kpt=np.asarray(k, dtype=np.float64), weight=float(w), miller=miller,
                                 C=C, eps=eps, f=f, P=P, dfde=dfde))
        if extra_kq:
            kq = []
            for i, (s, Pi) in enumerate(zip(sets, pis)):
                C0 = raw_coefficients(rng, A, s.kpt, s.miller, s.nbands)
                eps2, f2 = channels[i % len(channels)](rng)
                C2, P2 = paw_orthonormal_states(C0, Pi, paw, device)
                kq.append(StateSet(kpt=s.kpt.copy(), weight=s.weight, miller=s.miller, C=C2,
                                   eps=eps2, f=f2, P=P2))
    elif paw_model == "independent":
        if len(channels) != 1:
            raise ValueError("spin channels need the overlap projection model")
        pend = []
        for ik, k in enumerate(kpts):
            miller = wavefunction_sphere(A, k, ecut_wf)
            nb = levels(None, dry=True)
            C = orthonormal_coefficients(rng, A, k, miller, nb)
            eps, f = levels(rng)
            pend.append((k, kweights[ik], miller, C, eps, f))
        for (k, w, miller, C, eps, f) in pend:
            P = draw_projections(rng, C.shape[0], nproj_total)
            sets.append(StateSet(kpt=np.asarray(k, dtype=np.float64), weight=float(w), miller=miller,
                                 C=C, eps=eps, f=f, P=P))
        paw = draw_paw(rng, A, nproj)
        if extra_kq:
            kq = []
            for s in sets:
                C2 = orthonormal_coefficients(rng, A, s.kpt, s.miller, s.nbands)
                eps2, f2 = levels(rng)
                P2 = draw_projections(rng, s.nbands, nproj_total)
                kq.append(StateSet(kpt=s.kpt.copy(), weight=s.weight, miller=s.miller, C=C2,
                                   eps=eps2, f=f2, P=P2))
    else:
        raise ValueError(f"unknown paw_model {paw_model!r}")
    omega, ow = frequency_grid(nw, w0)
    wl = Workload(name=name, A=A, grid=tuple(int(x) for x in grid), kpoints=sets, paw=paw,
                  qpoints=qpoints, omega=omega, omega_weight=ow, seed=seed, kq=kq)
    check_alias_free(wl)
    return wl


def _spin_gapped(n_occ, n_unocc, moment):
    """Two spin channels (f in [0, 1]) with n_occ + moment/2 and n_occ - moment/2 occupied states and the
    same number of bands in each."""
    up, dn = n_occ + moment // 2, n_occ - moment // 2
    nb = n_occ + n_unocc

    def channel(n_o):
        def levels(rng, dry=False):
            if dry:
                return nb
            return gapped_levels(rng, n_o, nb - n_o, fmax=1.0)
        return levels
    return [channel(up), channel(dn)]


def _gapped(n_occ, n_unocc):
    def levels(rng, dry=False):
        if dry:
            return n_occ + n_unocc
        return gapped_levels(rng, n_occ, n_unocc)
    return levels


def _fermi(n_below, n_above, T, fmax=2.0):
    def levels(rng, dry=False):
        if dry:
            return n_below + n_above
        return fermi_levels(rng, n_below, n_above, T, fmax=fmax)
    # -df/d eps of f = fmax/(1 + e^{(eps - mu)/T}) from f itself
    levels.dfde = lambda f: f * (fmax - f) / (fmax * T)
    return levels


def max_abs_miller(m: np.ndarray) -> np.ndarray:
    return np.abs(np.asarray(m)).max(axis=0)


def check_alias_free(wl: Workload):
    """Pair products of two plane-wave sets are exact on the grid for every chi G-vector."""
    N = np.asarray(wl.grid)
    for qp in wl.qpoints:
        gm, _ = sphere_sq_lengths(wl.A, qp.q, np.sqrt(2.0 * qp.ecut))
        _, k2 = sphere_sq_lengths(wl.A, qp.q, np.sqrt(2.0 * qp.ecut))
        gm = gm[k2 <= 2.0 * qp.ecut]
        mc = max_abs_miller(gm)
        for s, t in zip(wl.kpoints, wl.kq_sets()):
            tot = max_abs_miller(s.miller) + max_abs_miller(t.miller) + mc
            if np.any(tot > N - 1):
                raise ValueError(f"grid {tuple(N)} aliases: |m_k|+|m_kq|+|m_chi| = {tuple(tot)}")
            if np.any(2 * max_abs_miller(s.miller) >= N):
                raise ValueError("wavefunction sphere does not fit the grid")


def config0(seed: int = 0, n_occ: int = 4, n_unocc: int = 60, nw: int = 8, extra_kq=False,
            paw_model: str = "overlap") -> Workload:
    """Tiny plain FP64 case: cubic L=10 bohr, 16^3 grid, Gamma, q=(0.1,0,0) 2pi/L,
    4 occupied + 60 unoccupied states, 2 atoms x 4 projectors, ~120 G, 8 frequencies."""
    L = 10.0
    A = np.eye(3) * L
    q = np.array([0.1 * TWO_PI / L, 0.0, 0.0])
    ecut = ecut_for_count(A, q, 120)
    qps = [QPoint(q=q, ecut=ecut)]
    return _assemble("cfg0-tiny", A, (16, 16, 16), seed, [np.zeros(3)], [1.0],
                     _gapped(n_occ, n_unocc), [4, 4], qps, nw, extra_kq=extra_kq, paw_model=paw_model)


def config1(seed: int = 1, n_occ: int = 16, n_unocc: int = 800, nw: int = 16,
            target_ng: int = 1500, grid=(48, 48, 48), which_q=(0, 1, 2),
            paw_model: str = "overlap", spin_moment: int = 0) -> Workload:
    """O2-in-box scale: 12x12x13 bohr, 48^3 grid, Gamma, 16 occupied + 800 unoccupied,
    2 atoms x 13 projectors, ~1500 G, 16 frequencies, q = 0 (optical), 0.1, 0.2 x 2pi/12 along x."""
    A = np.diag([12.0, 12.0, 13.0])
    qs = []
    for i in which_q:
        if i == 0:
            q = np.zeros(3)
            qs.append(QPoint(q=q, ecut=ecut_for_count(A, q, target_ng), optical=True,
                             qhat=np.array([1.0, 0.0, 0.0]), weight=1.0 / 3))
        else:
            q = np.array([0.1 * i * TWO_PI / 12.0, 0.0, 0.0])
            qs.append(QPoint(q=q, ecut=ecut_for_count(A, q, target_ng), weight=1.0 / 3))
    levels = _spin_gapped(n_occ, n_unocc, spin_moment) if spin_moment else _gapped(n_occ, n_unocc)
    return _assemble("cfg1-o2box", A, grid, seed, [np.zeros(3)], [1.0],
                     levels, [13, 13], qs, nw, paw_model=paw_model)


def config2(seed: int = 2, n_below: int = 120, n_above: int = 3000, nk: int = 8, nw: int = 16,
            target_ng: int = 4000, T: float = 0.01, paw_model: str = "overlap", device=None) -> Workload:
    """Metal-slab scale: 9x9x36 bohr, 40x40x160 grid, 2x2x2 Gamma-centred k (independent sets,
    w_k = 1/8), 120 + 3000 Fermi-smeared states (T = 0.01 Ha), 20 atoms x 18 projectors,
    ~4000 G, 16 frequencies, q = (0.1 2pi/9, 0, 0)."""
    A = np.diag([9.0, 9.0, 36.0])
    B = reciprocal_rows(A)
    frac = [(i, j, k) for i in (0, 1) for j in (0, 1) for k in (0, 1)][:nk]
    kpts = [0.5 * (i * B[0] + j * B[1] + k * B[2]) for (i, j, k) in frac]
    q = np.array([0.1 * TWO_PI / 9.0, 0.0, 0.0])
    qps = [QPoint(q=q, ecut=ecut_for_count(A, q, target_ng))]
    return _assemble("cfg2-slab", A, (40, 40, 160), seed, kpts, [1.0 / len(kpts)] * len(kpts),
                     _fermi(n_below, n_above, T), [18] * 20, qps, nw, paw_model=paw_model, device=device)


def config3_qpoints(seed: int = 3, nq: int = 64):
    A = np.diag([9.0, 9.0, 36.0])
    B = reciprocal_rows(A)
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, nq)
    targets = np.rint(200.0 * 15.0 ** u).astype(int)
    mp = [(2 * i - 5) / 8.0 for i in range(1, 5)]
    fr = [(a, b, c) for a in mp for b in mp for c in mp][:nq]
    qps = []
    for t, (a, b, c) in zip(targets, fr):
        q = a * B[0] + b * B[1] + c * B[2]
        qps.append(QPoint(q=q, ecut=ecut_for_count(A, q, int(t)), weight=1.0 / nq))
    return A, qps


def config3(seed: int = 3, n_occ: int = 60, n_unocc: int = 1500, nq: int = 64, nw: int = 16,
            paw_model: str = "overlap", device=None) -> Workload:
    """Batching form: 9x9x36 bohr, 40x40x160 grid, Gamma, 60 + 1500 states, 64 q-points of a
    4x4x4 Monkhorst-Pack mesh without Gamma, G-sphere sizes log-uneven in [200, 3000]."""
    A, qps = config3_qpoints(seed, nq)
    return _assemble("cfg3-batched", A, (40, 40, 160), seed, [np.zeros(3)], [1.0],
                     _gapped(n_occ, n_unocc), [18] * 20, qps, nw, paw_model=paw_model, device=device)


def tiny(grid=(8, 8, 8), L=(7.0, 7.5, 8.0), n_occ=2, n_unocc=5, nproj=(2, 3), target_ng=15,
         q_frac=(0.1, 0.0, 0.0), nw=8, seed=11, optical=False, extra_kq=False, ecut_wf_scale=None,
         paw_model="overlap", spin_moment=None, fermi_T=None):
    """Small cases on tiny grids for direct-sum checks and ragged shapes."""
    A = np.diag(np.asarray(L, dtype=np.float64))
    B = reciprocal_rows(A)
    q = q_frac[0] * B[0] + q_frac[1] * B[1] + q_frac[2] * B[2]
    if optical:
        q = np.zeros(3)
    qp = QPoint(q=q, ecut=ecut_for_count(A, q, target_ng), optical=optical)
    if fermi_T is not None:
        levels = _fermi(n_occ, n_unocc, fermi_T)
    elif spin_moment is None:
        levels = _gapped(n_occ, n_unocc)
    else:
        levels = _spin_gapped(n_occ, n_unocc, spin_moment)
    return _assemble("tiny", A, grid, seed, [np.zeros(3)], [1.0], levels,
                     list(nproj), [qp], nw, extra_kq=extra_kq, paw_model=paw_model)


# ----------------------------------------------------------------------------
# a cubic crystal with point symmetry: state sets of irreducible-zone k-points for the unfolding
# (Eq. kmap, Eq. trans_wfs; Table 1 steps 4 and 7)
# ----------------------------------------------------------------------------
# one atom at the origin and six at +-a/4 along the axes (stored in [0, 1)): an orbit of the full cubic
# group, so every cubic operation maps atoms onto atoms, some of them across a lattice vector
CUBIC_ATOMS = np.array([[0.0, 0.0, 0.0], [0.25, 0.0, 0.0], [0.75, 0.0, 0.0], [0.0, 0.25, 0.0],
                        [0.0, 0.75, 0.0], [0.0, 0.0, 0.25], [0.0, 0.0, 0.75]])


@dataclasses.dataclass
class SymWorkload:
    A: np.ndarray
    grid: tuple
    atoms: np.ndarray        # (Na, 3) fractional positions
    paw: Paw                 # s and p projectors per atom (Np = 4: s, p_x, p_y, p_z)
    sets: List[StateSet]     # state sets at the requested k-points
    qpoint: QPoint
    omega: np.ndarray
    omega_weight: np.ndarray


def atom_images(U, atoms):
    """(atom_map, atom_shift) of the fractional operation x -> U x: T^-1 R_a = R_b + L_a."""
    Ui = np.rint(np.linalg.inv(np.asarray(U, dtype=np.float64))).astype(np.int64)
    amap, shift = [], []
    for x in atoms:
        y = Ui @ x
        for b, xb in enumerate(atoms):
            d = y - xb
            if np.allclose(d, np.rint(d), atol=1e-12):
                amap.append(b)
                shift.append(np.rint(d).astype(np.int32))
                break
        else:
            raise ValueError("the atoms are not closed under the operation")
    return np.asarray(amap, dtype=np.int32), np.asarray(shift, dtype=np.int32).reshape(-1, 3)


def cartesian_op(U, A):
    A = np.asarray(A, dtype=np.float64)
    return A.T @ np.asarray(U, dtype=np.float64) @ np.linalg.inv(A.T)


def sp_rotation_blocks(U, A, natoms):
    """Flat D blocks [natoms * 16] for s + p projector functions: p_i(T y) = sum_j D_ij p_j(y) gives
    D = 1 for s and the Cartesian matrix of the operation for (p_x, p_y, p_z)."""
    blk = np.zeros((4, 4))
    blk[0, 0] = 1.0
    blk[1:, 1:] = cartesian_op(U, A)
    return np.tile(blk.reshape(-1), natoms)


def sp_projector_map(A, kpt, miller, paw, beta=1.0):
    """Pi[Q, 4a + i] = beta <p~^a_i|e^{i(k+G_Q).r}> for real s and p Gaussian projector functions:
    e^{i K.R_a} (1, i K_x, i K_y, i K_z) e^{-|K|^2 sigma^2/2}, K = k + G_Q; [NQ, 4 Na]."""
    B = reciprocal_rows(A)
    K = cart(miller, B, kpt)
    g = np.exp(-0.5 * paw.sigma ** 2 * (K[:, 0] ** 2 + K[:, 1] ** 2 + K[:, 2] ** 2))
    cols = []
    for a in range(len(paw.nproj)):
        ph = np.exp(1j * (K @ paw.R[a])) * g
        cols += [ph, 1j * K[:, 0] * ph, 1j * K[:, 1] * ph, 1j * K[:, 2] * ph]
    return beta * np.stack(cols, axis=1)


def symmetric_cubic(kpoints, seed=21, L=7.0, grid=(12, 12, 12), n_occ=3, n_unocc=9, target_ng=19,
                    q=(0.09, -0.05, 0.07), nw=8, beta=0.35):
    """State sets at the given Cartesian k-points of a simple-cubic crystal (CUBIC_ATOMS, s + p
    projectors with s^a = diag(0.3, -0.1, -0.1, -0.1), the same for every atom, so that the PAW overlap
    and the Q table are invariant under every cubic operation). Per k-point, in order: raw coefficients
    and gapped levels, then the PAW orthonormalisation with the s + p projector map. q in units of
    2 pi / L."""
    rng = np.random.default_rng(seed)
    A = L * np.eye(3)
    atoms = CUBIC_ATOMS.copy()
    na = atoms.shape[0]
    paw = Paw(nproj=[4] * na, s=[np.diag([0.3, -0.1, -0.1, -0.1]) for _ in range(na)], R=atoms @ A,
              D=[np.zeros((3, 4, 4)) for _ in range(na)], sigma=0.6)
    qv = np.asarray(q, dtype=np.float64) * 2 * np.pi / L
    qp = QPoint(q=qv, ecut=ecut_for_count(A, qv, target_ng))
    levels = _gapped(n_occ, n_unocc)
    sets = []
    for k in kpoints:
        k = np.asarray(k, dtype=np.float64)
        miller = wavefunction_sphere(A, k, 4.0 * qp.ecut)
        C0 = raw_coefficients(rng, A, k, miller, n_occ + n_unocc)
        eps, f = levels(rng)
        C, P = paw_orthonormal_states(C0, sp_projector_map(A, k, miller, paw, beta), paw)
        sets.append(StateSet(kpt=k, weight=1.0 / len(kpoints), miller=miller, C=C, eps=eps, f=f, P=P))
    omega, ow = frequency_grid(nw)
    return SymWorkload(A=A, grid=tuple(grid), atoms=atoms, paw=paw, sets=sets, qpoint=qp, omega=omega,
                       omega_weight=ow)
