"""Reference gradient of E_c(q) with respect to eigenvalues, plane-wave
coefficients and PAW projections.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no adjoint; this module differentiates the definition of
Eq. rpa with Eq. chi0, Eq. n_G_2, Eq. fft and Eq. n_q0 (readings R1-R11 of
:mod:`oracle.rpa`) with CPU float64 torch autograd, on a second, independent
formulation of the same forward pass: pair densities by FFT of the real-space
product, the PAW term by einsum, chi0 as a weighted Gram matrix, and
F(w) = sum_l [ln(1 - lambda_l) + lambda_l] from a Hermitian eigendecomposition
(ln det through log1p).

Conventions: complex gradients follow torch, grad = dE/dRe + i dE/dIm, so
the change of E along a complex direction d is Re sum conj(grad) d. The
coefficients C and projections P are free variables (no re-orthonormalisation);
occupations are held fixed.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rpa as R


def _t(x, dtype=torch.float64):
    return torch.as_tensor(np.asarray(x)).to(dtype)


def ec_torch(A, grid, C_k, C_kq, miller_k, miller_kq, eps_k, eps_kq, f_k, f_kq, P_k, P_kq, w_k,
             gmiller, Qtab, offsets, q, omega, omega_weight, optical=False, qhat=(1.0, 0.0, 0.0), Dtab=None,
             kpt=(0.0, 0.0, 0.0), same_set=False):
    """E_c(q) as a differentiable function of (C_k, C_kq, eps_k, eps_kq, P_k, P_kq).

    With same_set=True the k+q arguments are ignored and the k tensors are used
    for both sides, so that their gradient carries both contributions.
    """
    X, a = _pair_terms(A, grid, C_k, C_kq, miller_k, miller_kq, eps_k, eps_kq, f_k, f_kq, P_k, P_kq, w_k,
                       gmiller, Qtab, offsets, q, omega, optical, qhat, Dtab, kpt, same_set)
    return _ec_from_terms([(X, a)], omega, omega_weight)


def _pair_terms(A, grid, C_k, C_kq, miller_k, miller_kq, eps_k, eps_kq, f_k, f_kq, P_k, P_kq, w_k,
                gmiller, Qtab, offsets, q, omega, optical, qhat, Dtab, kpt, same_set):
    """One (k, k+q) pair's share of Eq. chi0: X = v^1/2 rho [pairs, NG] and the weights a [pairs, nw]."""
    if same_set:
        C_kq, eps_kq, P_kq, miller_kq, f_kq = C_k, eps_k, P_k, miller_k, f_k
    grid = tuple(int(g) for g in grid)
    N = grid[0] * grid[1] * grid[2]
    volume = abs(np.linalg.det(A))
    n_idx, m_idx = R.pair_list(np.asarray(f_k), np.asarray(f_kq))
    n_t = torch.as_tensor(n_idx)
    m_t = torch.as_tensor(m_idx)

    def to_grid(C, miller):
        box = torch.zeros((C.shape[0],) + grid, dtype=torch.complex128)
        i1, i2, i3 = R.grid_index(miller, grid)
        box[:, i1, i2, i3] = C
        return torch.fft.ifftn(box, dim=(1, 2, 3)) * N

    phi_k = to_grid(C_k, miller_k)
    phi_kq = phi_k if same_set else to_grid(C_kq, miller_kq)
    g1, g2, g3 = R.grid_index(gmiller, grid)
    prod = torch.conj(phi_k[n_t]) * phi_kq[m_t]
    spec = torch.fft.fftn(prod, dim=(1, 2, 3)) / N
    rho = spec[:, g1, g2, g3]

    Qt = torch.as_tensor(Qtab)
    qoff = 0
    for a in range(len(offsets) - 1):
        lo, hi = int(offsets[a]), int(offsets[a + 1])
        npj = hi - lo
        Qa = Qt[qoff:qoff + npj * npj].reshape(npj, npj, -1)
        qoff += npj * npj
        rho = rho + torch.einsum("pi,pj,ijg->pg", torch.conj(P_k[n_t][:, lo:hi]), P_kq[m_t][:, lo:hi], Qa)

    if optical:
        zero = np.nonzero(np.all(np.asarray(gmiller) == 0, axis=1))[0]
        if zero.size:
            g0 = int(zero[0])
            B = R.reciprocal_rows(A)
            kG = R.cartesian(miller_k, B, kpt)
            qh = np.asarray(qhat, dtype=np.float64)
            qh = qh / np.linalg.norm(qh)
            proj = torch.as_tensor(kG @ qh).to(torch.complex128)
            mom = torch.einsum("pq,pq->p", torch.conj(C_k[n_t]) * proj[None, :], C_kq[m_t])
            Dq = torch.as_tensor(np.tensordot(qh, Dtab, axes=(0, 0))).to(torch.complex128)
            paw = torch.zeros(n_idx.size, dtype=torch.complex128)
            qo = 0
            for a in range(len(offsets) - 1):
                lo, hi = int(offsets[a]), int(offsets[a + 1])
                npj = hi - lo
                Da = Dq[qo:qo + npj * npj].reshape(npj, npj)
                qo += npj * npj
                paw = paw + torch.einsum("pi,ij,pj->p", torch.conj(P_k[n_t][:, lo:hi]), Da, P_kq[m_t][:, lo:hi])
            head = (mom - 1j * paw) / (eps_kq[m_t] - eps_k[n_t]).to(torch.complex128)
            rho = torch.cat([rho[:, :g0], head[:, None], rho[:, g0 + 1:]], dim=1)

    d = eps_k[n_t] - eps_kq[m_t]
    df = _t(np.asarray(f_k)[n_idx] - np.asarray(f_kq)[m_idx])
    om = _t(omega)[None, :]
    a = (w_k / volume) * df[:, None] * 2.0 * d[:, None] / (om * om + d[:, None] ** 2)   # [P, nw]

    vs = _t(R.coulomb_sqrt(A, q, gmiller, optical)).to(torch.complex128)
    X = rho * vs[None, :]                                                                  # [P, NG]
    return X, a


def _ec_from_terms(terms, omega, omega_weight):
    """Eq. rpa from K(w) = sum over the pairs' terms of X^T diag(a(w)) conj(X) (Eq. chi0's k sum)."""
    E = torch.zeros((), dtype=torch.float64)
    wq = _t(omega_weight)
    for w in range(len(omega)):
        K = None
        for X, a in terms:
            Kt = (X.T * a[:, w].to(torch.complex128)[None, :]) @ torch.conj(X)
            K = Kt if K is None else K + Kt
        K = 0.5 * (K + torch.conj(K.T))
        lam = torch.linalg.eigvalsh(K)
        F = torch.sum(torch.log1p(-lam) + lam)
        E = E + wq[w] * F
    return E / (2.0 * np.pi)


def ec_and_grad(A, grid, sk, skq, gmiller, Qtab, offsets, q, omega, omega_weight, optical=False,
                qhat=(1.0, 0.0, 0.0), Dtab=None):
    """E_c(q) and its gradient for one (k, k+q) set pair (attributes C, miller, eps, f, P, kpt, weight).

    Returns (E, grads) with grads = dict(eps_k, C_k, P_k[, eps_kq, C_kq, P_kq]) as numpy arrays.
    """
    same = skq is sk
    Ck = torch.tensor(np.asarray(sk.C), dtype=torch.complex128, requires_grad=True)
    ek = torch.tensor(np.asarray(sk.eps), dtype=torch.float64, requires_grad=True)
    Pk = torch.tensor(np.asarray(sk.P), dtype=torch.complex128, requires_grad=True)
    if same:
        Ckq, ekq, Pkq = Ck, ek, Pk
    else:
        Ckq = torch.tensor(np.asarray(skq.C), dtype=torch.complex128, requires_grad=True)
        ekq = torch.tensor(np.asarray(skq.eps), dtype=torch.float64, requires_grad=True)
        Pkq = torch.tensor(np.asarray(skq.P), dtype=torch.complex128, requires_grad=True)
    E = ec_torch(A, grid, Ck, Ckq, sk.miller, skq.miller, ek, ekq, sk.f, skq.f, Pk, Pkq, sk.weight, gmiller,
                 Qtab, offsets, q, omega, omega_weight, optical, qhat, Dtab, sk.kpt, same_set=same)
    E.backward()
    grads = {"eps_k": ek.grad.numpy().copy(), "C_k": Ck.grad.numpy().copy(), "P_k": Pk.grad.numpy().copy()}
    if not same:
        grads.update(eps_kq=ekq.grad.numpy().copy(), C_kq=Ckq.grad.numpy().copy(), P_kq=Pkq.grad.numpy().copy())
    return float(E.detach()), grads


def ec_and_grad_sets(A, grid, ksets, kqsets, gmiller, Qtab, offsets, q, omega, omega_weight, optical=False,
                     qhat=(1.0, 0.0, 0.0), Dtab=None):
    """E_c(q) of several (k, k+q) set pairs (Eq. chi0's k sum) and its gradient per listing: pair i gets
    leaves of its own (its k+q set shares its k set's leaves when it is the same object), so grads[i] is
    the derivative with respect to the inputs of that listing. Returns (E, [grads dict per pair])."""
    leaves, terms = [], []
    for sk, skq in zip(ksets, kqsets):
        same = skq is sk
        Ck = torch.tensor(np.asarray(sk.C), dtype=torch.complex128, requires_grad=True)
        ek = torch.tensor(np.asarray(sk.eps), dtype=torch.float64, requires_grad=True)
        Pk = torch.tensor(np.asarray(sk.P), dtype=torch.complex128, requires_grad=True)
        if same:
            Ckq, ekq, Pkq = Ck, ek, Pk
        else:
            Ckq = torch.tensor(np.asarray(skq.C), dtype=torch.complex128, requires_grad=True)
            ekq = torch.tensor(np.asarray(skq.eps), dtype=torch.float64, requires_grad=True)
            Pkq = torch.tensor(np.asarray(skq.P), dtype=torch.complex128, requires_grad=True)
        leaves.append((same, Ck, ek, Pk, Ckq, ekq, Pkq))
        terms.append(_pair_terms(A, grid, Ck, Ckq, sk.miller, skq.miller, ek, ekq, sk.f, skq.f, Pk, Pkq, sk.weight,
                                 gmiller, Qtab, offsets, q, omega, optical, qhat, Dtab, sk.kpt, same))
    E = _ec_from_terms(terms, omega, omega_weight)
    E.backward()
    out = []
    for same, Ck, ek, Pk, Ckq, ekq, Pkq in leaves:
        g = {"eps_k": ek.grad.numpy().copy(), "C_k": Ck.grad.numpy().copy(), "P_k": Pk.grad.numpy().copy()}
        if not same:
            g.update(eps_kq=ekq.grad.numpy().copy(), C_kq=Ckq.grad.numpy().copy(), P_kq=Pkq.grad.numpy().copy())
        out.append(g)
    return float(E.detach()), out
