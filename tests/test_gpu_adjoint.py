"""The hand-written adjoint (rpa_ec_backward) against the oracle's reference
gradient (torch float64 autograd on the CPU, itself pinned by finite
differences) and against central finite differences of the library's own
FP64 E_c on the 48^3 grid."""
import numpy as np
import pytest

import oracle
import oracle.grad as G
import synth
from helpers import gpu_inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rpa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1307_8052_amd as m
    return m


CASES = {
    "q_finite": lambda: synth.tiny(grid=(8, 8, 8), n_occ=2, n_unocc=4, target_ng=15, nw=8),
    "optical": lambda: synth.tiny(grid=(10, 10, 10), n_occ=2, n_unocc=3, optical=True, target_ng=12, nw=8),
    "distinct_kq": lambda: synth.tiny(grid=(8, 8, 8), n_occ=2, n_unocc=3, target_ng=15, nw=8, extra_kq=True),
    "cfg0_small": lambda: synth.config0(n_occ=2, n_unocc=10),
    # NG = 300: five 64-wide block columns, so the factorisation ends on an unpaired panel step
    "five_blocks": lambda: synth.tiny(grid=(24, 24, 24), L=(8.0, 8.5, 9.0), n_occ=2, n_unocc=6, target_ng=300,
                                      nw=8),
}


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("optical", [False, True])
def test_adjoint_over_several_set_pairs(rpa, optical):
    """Eq. chi0's k sum in the adjoint: listings (s, t) and (t', t') with t' a copy of t at half weight
    (k-point weights 1 and 1/2) in one call; each listing's gradient against the oracle's reference.
    At the optical q-point both listings use their k set as k+q: (s, s) and (t', t')."""
    wl = synth.tiny(grid=(10, 10, 10), n_occ=2, n_unocc=3, target_ng=12 if optical else 15, nw=8, extra_kq=True,
                    optical=optical)
    s, t = wl.kpoints[0], wl.kq_sets()[0]
    t2 = synth.StateSet(kpt=t.kpt, weight=0.5, miller=t.miller, C=t.C, eps=t.eps, f=t.f, P=t.P)
    qp = wl.qpoints[0]
    gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
    D = synth.paw_d_table(wl.paw)
    okq = [s, t2] if optical else [t, t2]
    E_ref, g_ref = G.ec_and_grad_sets(wl.A, wl.grid, [s, t2], okq, gm, Q, wl.paw.offsets, qp.q, wl.omega,
                                      wl.omega_weight, qp.optical, qp.qhat, D)
    dev = "cuda:0"
    S = rpa.States.from_synth(s, wl.paw, dev)
    T = rpa.States.from_synth(t, wl.paw, dev)
    T2 = rpa.States.from_synth(t2, wl.paw, dev)
    qs = rpa.QSpec(qp.q, gm, Q, optical=qp.optical, qhat=qp.qhat, Dpaw=D, device=dev)
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ec, g = ctx.ec_backward([S, T2], [S, T2] if optical else [T, T2], qs, fr)
        ctx.check()
    assert abs(float(ec.cpu()[0]) - E_ref) < 1e-10
    for i, (gg, gr) in enumerate(zip(g, g_ref)):
        assert set(gg) == set(gr)
        for key in gr:
            r = _rel(gg[key].cpu().numpy(), gr[key])
            print(f"optical={optical} pair {i} {key}: rel={r:.3e}", flush=True)
            assert r < 1e-9, (i, key)


@pytest.mark.parametrize("path,chunk", [(0, 0), (0, 24), (1, 24)])
def test_adjoint_owner_segments(rpa, path, chunk):
    """Occupied bands with 40 transitions each (16^3 grid, 3 + 40 states, distinct k+q states): the register
    x-y adjoint (path 0) cuts each band's pairs into segments whose partial sums are added afterwards, also
    with the pairs spread over chunks of 24; path 1 runs the LDS form on the same inputs. Both against the
    oracle's reference gradient."""
    wl = synth.config0(n_occ=3, n_unocc=40, extra_kq=True)
    s, t = wl.kpoints[0], wl.kq_sets()[0]
    qp = wl.qpoints[0]
    gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
    D = synth.paw_d_table(wl.paw)
    E_ref, g_ref = G.ec_and_grad(wl.A, wl.grid, s, t, gm, Q, wl.paw.offsets, qp.q, wl.omega, wl.omega_weight,
                                 qp.optical, qp.qhat, D)
    ks, kqs, qs, fr, _ = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.set_pair_path(path)
        ctx.set_chunk_pairs(chunk)
        ec, g = ctx.ec_backward(ks[0], kqs[0], qs, fr)
        ctx.check()
    assert abs(float(ec.cpu()[0]) - E_ref) < 1e-10
    for key in ["eps_k", "C_k", "P_k", "eps_kq", "C_kq", "P_kq"]:
        r = _rel(g[key].cpu().numpy(), g_ref[key])
        print(f"path {path} chunk {chunk} {key}: rel={r:.3e}", flush=True)
        assert r < 1e-9, key


def test_adjoint_stage_profiler(rpa):
    """The adjoint's stages in the stage profiler: a backward call over 3 + 40 states (120 transitions) in
    chunks of at most 50 pairs times one inverse, one batched W(omega) rho product per chunk (all
    frequencies), one group of adjoint pair transforms per chunk, and the forward pass's own Cholesky
    stage."""
    wl = synth.config0(n_occ=3, n_unocc=40)
    ks, _, qs, fr, _ = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.set_chunk_pairs(50)
        ctx.ec_backward(ks[0], ks[0], qs, fr)
        ctx.profile(True)
        ctx.ec_backward(ks[0], ks[0], qs, fr)
        prof = ctx.profile_get()
        ctx.profile(False)
    print({k: (round(v[0], 3), v[1]) for k, v in prof.items()}, flush=True)
    assert prof["adjoint_inverse"][1] == 1
    assert prof["adjoint_gemm"][1] == 3
    assert prof["adjoint_pairs"][1] == 3
    assert prof["adjoint_rest"][1] > 0 and prof["cholesky"][1] == 1 and prof["herk"][1] >= 1
    assert all(v[0] > 0 for v in prof.values() if v[1])


def test_adjoint_rejects_more_than_64_frequencies(rpa):
    """The adjoint takes at most 64 frequencies: 65 is RPA_ERR_UNSUPPORTED before any launch."""
    wl = synth.tiny(grid=(8, 8, 8), n_occ=2, n_unocc=4, target_ng=15, nw=8)
    ks, _, qs, _, _ = gpu_inputs(rpa, wl)
    x = np.linspace(0.01, 0.99, 65)
    fr = rpa.Freq(x / (1 - x), np.full(65, 0.01))
    with rpa.Context(wl.A, wl.grid) as ctx:
        with pytest.raises(rpa.RpaError) as ei:
            ctx.ec_backward(ks[0], ks[0], qs, fr)
        assert ei.value.status == -7


@pytest.mark.parametrize("case", list(CASES))
def test_adjoint_matches_reference_gradient(rpa, case):
    wl = CASES[case]()
    s, t = wl.kpoints[0], wl.kq_sets()[0]
    qp = wl.qpoints[0]
    gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
    D = synth.paw_d_table(wl.paw)
    same = wl.kq is None
    E_ref, g_ref = G.ec_and_grad(wl.A, wl.grid, s, s if same else t, gm, Q, wl.paw.offsets, qp.q, wl.omega,
                                 wl.omega_weight, qp.optical, qp.qhat, D)
    ks, kqs, qs, fr, gm2 = gpu_inputs(rpa, wl)
    assert np.array_equal(gm, gm2)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ec, g = ctx.ec_backward(ks[0], ks[0] if same else kqs[0], qs, fr)
        ctx.check()
    assert abs(float(ec.cpu()[0]) - E_ref) < 1e-10
    keys = ["eps_k", "C_k", "P_k"] + ([] if same else ["eps_kq", "C_kq", "P_kq"])
    for key in keys:
        got = g[key].cpu().numpy()
        r = _rel(got, g_ref[key])
        print(f"{case} {key}: rel={r:.3e}", flush=True)
        assert r < 1e-9, key


def test_adjoint_directional_derivatives_48cubed(rpa):
    """48^3 grid, NG = 1500, 4 + 40 states, q = 0.1 x 2pi/12: the gradient's directional derivative along
    20 random unit directions equals the central difference (step 1e-5) of the library's E_c."""
    wl = synth.config1(n_occ=4, n_unocc=40, which_q=(1,))
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    s = wl.kpoints[0]
    rng = np.random.default_rng(20)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ec, g = ctx.ec_backward(ks[0], ks[0], qs, fr)
        gC, gP, ge = g["C_k"].cpu().numpy(), g["P_k"].cpu().numpy(), g["eps_k"].cpu().numpy()

        def energy(C, P, eps):
            st = rpa.States(C, s.miller, eps, s.f, P, wl.paw.offsets, s.kpt, s.weight)
            e, _ = ctx.ec([st], [st], qs, fr, "fp64")
            return float(e.cpu()[0])

        h = 1e-5
        for trial in range(20):
            dC = rng.standard_normal(s.C.shape) + 1j * rng.standard_normal(s.C.shape)
            dP = rng.standard_normal(s.P.shape) + 1j * rng.standard_normal(s.P.shape)
            de = rng.standard_normal(s.eps.shape)
            nrm = np.sqrt(np.sum(np.abs(dC) ** 2) + np.sum(np.abs(dP) ** 2) + np.sum(de ** 2))
            dC, dP, de = dC / nrm, dP / nrm, de / nrm
            fd = (energy(s.C + h * dC, s.P + h * dP, s.eps + h * de)
                  - energy(s.C - h * dC, s.P - h * dP, s.eps - h * de)) / (2 * h)
            pred = float(np.real(np.sum(np.conj(gC) * dC)) + np.real(np.sum(np.conj(gP) * dP)) + np.sum(ge * de))
            print(f"direction {trial}: fd={fd:.10e} adjoint={pred:.10e}", flush=True)
            assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred))


def test_autograd_function(rpa):
    wl = CASES["q_finite"]()
    s = wl.kpoints[0]
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        C = torch.tensor(s.C, dtype=torch.complex128, device="cuda:0", requires_grad=True)
        P = torch.tensor(s.P, dtype=torch.complex128, device="cuda:0", requires_grad=True)
        eps = torch.tensor(s.eps, dtype=torch.float64, requires_grad=True)
        E = rpa.ec_autograd(ctx, C, eps, P, ks[0], qs, fr)
        (2.5 * E).backward()
        _, g = ctx.ec_backward(ks[0], ks[0], qs, fr, dEc=2.5)
        assert torch.allclose(C.grad, g["C_k"], rtol=1e-12, atol=1e-18)
        assert torch.allclose(P.grad, g["P_k"], rtol=1e-12, atol=1e-18)
        assert torch.allclose(eps.grad, g["eps_k"].cpu(), rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("iq", [0, 1])
def test_adjoint_full_o2box_directional_derivatives(rpa, iq):
    """The differentiation form at O2-in-box size: all 16 + 800 states (12,800 pairs, NG ~ 1500), the optical
    q-point and q = 0.1 x 2 pi/12. The gradient's directional derivative along 10 random unit directions of
    (C, P, eps) equals the central difference (step 1e-5) of the library's FP64 E_c."""
    wl = synth.config1(which_q=(iq,))
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    s = wl.kpoints[0]
    rng = np.random.default_rng(40 + iq)
    D = synth.paw_d_table(wl.paw)
    qp = wl.qpoints[0]
    with rpa.Context(wl.A, wl.grid) as ctx:
        ec, g = ctx.ec_backward(ks[0], ks[0], qs, fr)
        gC, gP, ge = g["C_k"].cpu().numpy(), g["P_k"].cpu().numpy(), g["eps_k"].cpu().numpy()

        def energy(C, P, eps):
            st = rpa.States(C, s.miller, eps, s.f, P, wl.paw.offsets, s.kpt, s.weight)
            e, _ = ctx.ec([st], [st], qs, fr, "fp64")
            return float(e.cpu()[0])

        e0 = energy(s.C, s.P, s.eps)
        assert abs(e0 - float(ec.cpu()[0])) < 1e-12
        h = 1e-5
        for trial in range(10):
            dC = rng.standard_normal(s.C.shape) + 1j * rng.standard_normal(s.C.shape)
            dP = rng.standard_normal(s.P.shape) + 1j * rng.standard_normal(s.P.shape)
            de = rng.standard_normal(s.eps.shape)
            nrm = np.sqrt(np.sum(np.abs(dC) ** 2) + np.sum(np.abs(dP) ** 2) + np.sum(de ** 2))
            dC, dP, de = dC / nrm, dP / nrm, de / nrm
            fd = (energy(s.C + h * dC, s.P + h * dP, s.eps + h * de)
                  - energy(s.C - h * dC, s.P - h * dP, s.eps - h * de)) / (2 * h)
            pred = float(np.real(np.sum(np.conj(gC) * dC)) + np.real(np.sum(np.conj(gP) * dP)) + np.sum(ge * de))
            print(f"q{iq} direction {trial}: fd={fd:.10e} adjoint={pred:.10e} diff={fd - pred:.2e}", flush=True)
            assert abs(fd - pred) < 1e-6 * max(1.0, abs(pred))
