"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Sizes: tiny grids (direct checks, ragged sphere boxes, distinct k and k+q
sets), the 16^3 configuration with 4 + 60 states, and reduced-band variants
of the 48^3 configuration. Tolerances:
  FP64 path   - pair densities and chi0 within 1e-12 of the largest element,
                E_c within 1e-10 Ha;
  split path  - pair densities (FP32 FFT) within 2e-6 relative, chi0 within
                2e-4 of the largest element, E_c within 1e-6 Ha.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from helpers import gpu_inputs, oracle_q

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rpa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1307_8052_amd as m
    return m


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


WORKLOADS = {
    "tiny8": lambda: synth.tiny(grid=(8, 8, 8)),
    "tiny6x8x10": lambda: synth.tiny(grid=(6, 8, 10), L=(6.0, 7.0, 9.0), target_ng=9),
    "tiny12_distinct_kq": lambda: synth.tiny(grid=(12, 12, 12), L=(8.0, 8.5, 9.0), n_occ=3, n_unocc=7,
                                             target_ng=40, extra_kq=True),
    "tiny10_optical": lambda: synth.tiny(grid=(10, 10, 10), n_occ=2, n_unocc=4, optical=True, target_ng=12),
    "cfg0": lambda: synth.config0(),
    # the stress workload: projections drawn apart from the coefficients, a large PAW term
    "cfg0_independent": lambda: synth.config0(paw_model="independent"),
    # Fermi-smeared partly filled bands at q -> 0: the intraband head (sets carry -df/de)
    "tiny10_metal_optical": lambda: synth.tiny(grid=(10, 10, 10), n_occ=3, n_unocc=5, optical=True, target_ng=12,
                                               fermi_T=0.05),
    # two spin channels (occupations in [0, 1]) with a moment of 2
    "tiny12_spin": lambda: synth.tiny(grid=(12, 12, 12), L=(8.0, 8.5, 9.0), n_occ=3, n_unocc=7, target_ng=40,
                                      spin_moment=2),
}


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("name", list(WORKLOADS))
@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_pair_density(rpa, name, prec, path):
    """Path 0 runs the register-resident transforms where the grid has them (8^3, 10^3, 12^3, 16^3; the
    6x8x10 grid falls back to the LDS passes), path 1 always the LDS passes."""
    wl = WORKLOADS[name]()
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    s, t = wl.kpoints[0], wl.kq_sets()[0]
    ref_g = oracle.gsphere(wl.A, wl.qpoints[0].q, wl.qpoints[0].ecut)
    assert np.array_equal(gm, ref_g)
    pairs = oracle.pair_list(s.f, t.f)
    Q = synth.paw_q_table(wl.paw, wl.A, wl.qpoints[0].q, ref_g)
    _, rho_ref = oracle.pair_densities(wl.A, wl.grid, s, t, ref_g, Q, wl.paw.offsets, wl.qpoints[0].optical,
                                       wl.qpoints[0].qhat, synth.paw_d_table(wl.paw))
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.set_pair_path(path)
        rho = ctx.pair_density(ks[0], kqs[0], qs, pairs[0], pairs[1], prec).cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 2e-6
    print(f"{name} {prec} path {path}: pairs={pairs[0].size} NG={len(gm)} rel={_rel(rho, rho_ref):.3e}",
          flush=True)
    assert _rel(rho, rho_ref) < tol


def test_pair_density_unsorted_pairs_and_diagonal(rpa):
    """Arbitrary pair order (including n = m) and the G = 0 normalisation of the pseudo part (the stress
    workload, whose coefficients are orthonormal on their own)."""
    wl = synth.tiny(grid=(8, 8, 8), n_occ=2, n_unocc=5, q_frac=(0.0, 0.0, 0.0), nproj=(1,), target_ng=7,
                    paw_model="independent")
    wl.qpoints[0].q = np.zeros(3)
    s = wl.kpoints[0]
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    qs.Qpaw = qs.Qpaw * 0
    pn = np.array([3, 0, 6, 2, 2, 5], dtype=np.int32)
    pm = np.array([1, 0, 6, 4, 2, 1], dtype=np.int32)
    with rpa.Context(wl.A, wl.grid) as ctx:
        rho = ctx.pair_density(ks[0], ks[0], qs, pn, pm).cpu().numpy()
    phi = oracle.orbitals(s.C, s.miller, wl.grid)
    ref = oracle.pseudo_pair_density(phi, phi, (pn.astype(np.int64), pm.astype(np.int64)), gm, wl.grid)
    assert _rel(rho, ref) < 1e-12
    g0 = int(np.nonzero(np.all(gm == 0, axis=1))[0][0])
    assert np.allclose(rho[:, g0], (pn == pm).astype(float), atol=1e-13)


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("name", ["tiny8", "tiny12_distinct_kq", "tiny10_optical", "cfg0", "cfg0_independent",
                                  "tiny10_metal_optical", "tiny12_spin"])
def test_chi0_and_ec_fp64(rpa, name, path):
    wl = WORKLOADS[name]()
    ref = oracle_q(wl)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.set_pair_path(path)
        chi = ctx.chi0(ks, kqs, qs, fr, "fp64").cpu().numpy()
        ec, F = ctx.ec(ks, kqs, qs, fr, "fp64")
        ctx.check()
        ec = float(ec.cpu()[0])
        F = F.cpu().numpy()
    r = _rel(chi, ref["chi"])
    print(f"{name}: NG={len(gm)} chi rel={r:.3e} E={ec:.12f} ref={ref['E']:.12f} dE={ec - ref['E']:.3e}", flush=True)
    assert r < 1e-12
    assert np.max(np.abs(F - ref["F"])) < 1e-10
    assert abs(ec - ref["E"]) < 1e-10


@pytest.mark.parametrize("target_ng,grid", [(150, (16, 16, 16)), (250, (24, 24, 24)), (300, (24, 24, 24)),
                                             (421, (24, 24, 24))])
def test_ec_block_column_counts(rpa, target_ng, grid):
    """The blocked factorisation pairs its 64-wide panel steps and looks two block columns ahead: NG padded
    to 192, 256, 320 and 448 gives 3, 4, 5 and 7 block columns (an unpaired last step, a look-ahead clipped
    at the last block column). FP64 E_c and F(w) against the oracle, and the split path's E_c."""
    wl = synth.tiny(grid=grid, L=(8.0, 8.5, 9.0), n_occ=2, n_unocc=10, target_ng=target_ng)
    ref = oracle_q(wl)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    assert np.array_equal(gm, ref["gm"])
    with rpa.Context(wl.A, wl.grid) as ctx:
        ec, F = ctx.ec(ks, kqs, qs, fr, "fp64")
        ecb, _ = ctx.ec(ks, kqs, qs, fr, "split_bf16")
        ecf, Ff = ctx.ec_from_chi0(qs, fr, torch.from_numpy(ref["chi"]))
        ctx.check()
        ec, ecb, ecf = float(ec.cpu()[0]), float(ecb.cpu()[0]), float(ecf.cpu()[0])
        F, Ff = F.cpu().numpy(), Ff.cpu().numpy()
    print(f"NG={len(gm)} blocks={(len(gm) + 63) // 64}: E={ec:.14f} from oracle chi0 {ecf:.14f} "
          f"split {ecb:.12f} ref={ref['E']:.14f}", flush=True)
    assert abs(ec - ref["E"]) < 1e-10
    assert np.max(np.abs(F - ref["F"])) < 1e-10
    assert abs(ecf - ref["E"]) < 1e-12
    assert np.max(np.abs(Ff - ref["F"])) < 1e-12
    assert abs(ecb - ref["E"]) < 1e-6


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_chi0_and_ec_split(rpa, prec):
    wl = synth.config0()
    ref = oracle_q(wl)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        chi = ctx.chi0(ks, kqs, qs, fr, prec).cpu().numpy()
        ec, F = ctx.ec(ks, kqs, qs, fr, prec)
        ctx.check()
        ec = float(ec.cpu()[0])
    r = _rel(chi, ref["chi"])
    print(f"cfg0 {prec}: chi rel={r:.3e} E={ec:.10f} ref={ref['E']:.10f} dE={ec - ref['E']:.3e}", flush=True)
    assert r < 2e-4
    assert abs(ec - ref["E"]) < 1e-6


def test_ec_from_oracle_chi0(rpa):
    wl = synth.config0(n_occ=2, n_unocc=20)
    ref = oracle_q(wl)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ec, F = ctx.ec_from_chi0(qs, fr, torch.from_numpy(ref["chi"]))
        ctx.check()
    assert abs(float(ec.cpu()[0]) - ref["E"]) < 1e-12
    assert np.max(np.abs(F.cpu().numpy() - ref["F"])) < 1e-12


def test_not_positive_definite_is_reported(rpa):
    """A chi0 with one positive weight large enough to make 1 - K indefinite."""
    wl = synth.config0(n_occ=1, n_unocc=3)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    NG = len(gm)
    chi = np.zeros((wl.omega.size, NG, NG), dtype=np.complex128)
    v = np.zeros(NG, dtype=np.complex128)
    v[3] = 1.0
    chi[2] = 50.0 * np.outer(v, v)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.ec_from_chi0(qs, fr, torch.from_numpy(chi))
        with pytest.raises(rpa.RpaError) as ei:
            ctx.check()
    assert ei.value.status == -5 and "frequency index 2" in str(ei.value)


def test_stage_profiler(rpa):
    """The stage profiler the benchmark reads: every stage name is accepted, an unknown one is an input error;
    one batched split-precision call over two q-points times two packing groups and two rank-k launches (one
    chunk per q), each with positive elapsed time, one x-y pair transform (shared by the two q-points, whose
    state sets are the same) and two z passes, and one Cholesky stage; nothing is recorded after profiling
    stops."""
    wl = synth.config1(n_occ=2, n_unocc=20, which_q=(0, 1))
    qspecs = []
    for iq in range(2):
        ks, _, qs, fr, _ = gpu_inputs(rpa, wl, iq)
        qspecs.append(qs)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.ec_batched(ks, ks, qspecs, fr, "split_bf16")   # plans and workspaces outside the timed call
        ctx.profile(True)
        ctx.ec_batched(ks, ks, qspecs, fr, "split_bf16")
        prof = ctx.profile_get()
        ctx.profile(False)
        ctx.ec_batched(ks, ks, qspecs, fr, "split_bf16")
        after = ctx.profile_get()
        with pytest.raises(rpa.RpaError):
            ms = ctypes.c_double(0)
            n = ctypes.c_longlong(0)
            rpa._check(ctx._L.rpa_profile_get(ctx._h, b"no_such_stage", ctypes.byref(ms), ctypes.byref(n)), ctx._h)
    print({k: (round(v[0], 3), v[1]) for k, v in prof.items()}, flush=True)
    assert set(prof) == set(rpa.Context.STAGES)
    assert prof["herk"][1] == 2 and prof["herk"][0] > 0
    assert prof["split_pack"][1] == 2 and prof["split_pack"][0] > 0
    assert prof["cholesky"][1] == 1 and prof["cholesky"][0] > 0
    assert prof["pair_xy"][1] == 1 and prof["pair_z_gather"][1] == 2
    assert all(v[0] >= 0 for v in prof.values())
    assert all(v[1] == 0 for v in after.values())


def test_no_transitions_give_zero(rpa):
    """All states fully occupied: no pair has f_n - f_m > 0, chi0 vanishes and E_c is exactly 0."""
    wl = synth.tiny(grid=(8, 8, 8), n_occ=4, n_unocc=3)
    s = wl.kpoints[0]
    s.f = np.full_like(s.f, 2.0)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        for prec in ("fp64", "split_bf16"):
            chi = ctx.chi0(ks, kqs, qs, fr, prec).cpu().numpy()
            ec, F = ctx.ec(ks, kqs, qs, fr, prec)
            ctx.check()
            assert not np.any(chi)
            assert float(ec.cpu()[0]) == 0.0 and not np.any(F.cpu().numpy())


def test_degenerate_optical_transition_is_rejected(rpa):
    wl = synth.tiny(grid=(10, 10, 10), n_occ=2, n_unocc=4, optical=True, target_ng=12)
    s = wl.kpoints[0]
    s.eps = s.eps.copy()
    s.eps[2] = s.eps[1]    # an occupied and an empty state at the same energy
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        with pytest.raises(rpa.RpaError) as ei:
            ctx.ec(ks, kqs, qs, fr)
    assert ei.value.status == -1 and "degenerate" in str(ei.value)


def test_alias_and_shape_errors_before_launch(rpa):
    wl = synth.config0(n_occ=1, n_unocc=3)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, (12, 12, 12)) as ctx:
        with pytest.raises(rpa.RpaError) as ei:
            ctx.ec(ks, kqs, qs, fr)
        assert ei.value.status in (-3,)
    bad = rpa.States(wl.kpoints[0].C, wl.kpoints[0].miller, wl.kpoints[0].eps[::-1].copy(), wl.kpoints[0].f,
                     wl.kpoints[0].P, wl.paw.offsets)
    with rpa.Context(wl.A, wl.grid) as ctx:
        with pytest.raises(rpa.RpaError) as ei:
            ctx.ec([bad], [bad], qs, fr)
        assert ei.value.status == -1


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_o2box_pair_density_register_path(rpa, prec):
    """48^3 grid, NG = 1503 (optical q): 2 occupied x 12 unoccupied pairs through the register-resident
    transforms, element by element against the oracle, and equal (to rounding) to the LDS passes."""
    wl = synth.config1(n_occ=2, n_unocc=12, which_q=(0,))
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    s = wl.kpoints[0]
    pairs = oracle.pair_list(s.f, s.f)
    Q = synth.paw_q_table(wl.paw, wl.A, wl.qpoints[0].q, gm)
    _, ref = oracle.pair_densities(wl.A, wl.grid, s, s, gm, Q, wl.paw.offsets, wl.qpoints[0].optical,
                                   wl.qpoints[0].qhat, synth.paw_d_table(wl.paw))
    with rpa.Context(wl.A, wl.grid) as ctx:
        reg = ctx.pair_density(ks[0], ks[0], qs, pairs[0], pairs[1], prec).cpu().numpy()
        ctx.set_pair_path(1)
        lds = ctx.pair_density(ks[0], ks[0], qs, pairs[0], pairs[1], prec).cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 2e-6
    print(f"o2box pairs {prec}: reg rel={_rel(reg, ref):.3e} lds rel={_rel(lds, ref):.3e} "
          f"reg-lds={_rel(reg, lds):.3e}", flush=True)
    assert _rel(reg, ref) < tol
    assert _rel(lds, ref) < tol
    assert _rel(reg, lds) < tol


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_paw_term_forms_and_band_windows(rpa, prec):
    """The PAW term's two MFMA forms (48^3 grid, NG = 1500, 4 + 40 states): factorised per band n (the
    default here: chunks span 4 bands n and 40 bands m) and per band m, in one pass per chunk (window bound
    1000) or in passes of at most 7 bands m. Pair densities in the oracle's order (n-major: every pass a
    run of consecutive pairs) against the oracle for every form; pair densities and chi0 of the m form
    equal bit for bit whatever the window."""
    wl = synth.config1(n_occ=4, n_unocc=40, which_q=(1,))
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    s = wl.kpoints[0]
    pairs = oracle.pair_list(s.f, s.f)
    Q = synth.paw_q_table(wl.paw, wl.A, wl.qpoints[0].q, gm)
    _, ref = oracle.pair_densities(wl.A, wl.grid, s, s, gm, Q, wl.paw.offsets, wl.qpoints[0].optical,
                                   wl.qpoints[0].qhat, synth.paw_d_table(wl.paw))
    out = {}
    with rpa.Context(wl.A, wl.grid) as ctx:
        for win in (0, 1000, 7):
            ctx.set_paw_window(win)
            out[win] = (ctx.pair_density(ks[0], ks[0], qs, pairs[0], pairs[1], prec).cpu().numpy(),
                        ctx.chi0(ks, ks, qs, fr, prec).cpu().numpy())
        with pytest.raises(rpa.RpaError):
            ctx.set_paw_window(-1)
    tol = 1e-12 if prec == "fp64" else 2e-6
    for win, (rho, chi) in out.items():
        print(f"paw window {win} {prec}: rho rel={_rel(rho, ref):.3e} chi vs n form "
              f"{_rel(chi, out[0][1]):.3e}", flush=True)
        assert _rel(rho, ref) < tol
        assert _rel(chi, out[0][1]) < (1e-12 if prec == "fp64" else 1e-5)
    assert np.array_equal(out[1000][0], out[7][0])
    assert np.array_equal(out[1000][1], out[7][1])


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_slab_pair_density_z_quads(rpa, prec):
    """The metal-slab grid (40 x 40 x 160, NG = 303): the z pass of 160 points runs by quads of lanes (a
    whole line does not fit one lane), keeping the sphere's z window; element by element against the
    oracle, and equal (to rounding) to the LDS passes."""
    wl = synth.config2(n_below=2, n_above=6, nk=1, target_ng=300)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    s = wl.kpoints[0]
    pairs = oracle.pair_list(s.f, s.f)
    Q = synth.paw_q_table(wl.paw, wl.A, wl.qpoints[0].q, gm)
    _, ref = oracle.pair_densities(wl.A, wl.grid, s, s, gm, Q, wl.paw.offsets, wl.qpoints[0].optical,
                                   wl.qpoints[0].qhat, synth.paw_d_table(wl.paw))
    with rpa.Context(wl.A, wl.grid) as ctx:
        quad = ctx.pair_density(ks[0], ks[0], qs, pairs[0], pairs[1], prec).cpu().numpy()
        ctx.set_pair_path(1)
        lds = ctx.pair_density(ks[0], ks[0], qs, pairs[0], pairs[1], prec).cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 2e-6
    print(f"slab pairs {prec}: {pairs[0].size} pairs, quad rel={_rel(quad, ref):.3e} lds rel={_rel(lds, ref):.3e} "
          f"quad-lds={_rel(quad, lds):.3e}", flush=True)
    assert _rel(quad, ref) < tol
    assert _rel(lds, ref) < tol
    assert _rel(quad, lds) < tol


@pytest.mark.parametrize("iq", [0, 1])
def test_o2box_reduced_bands(rpa, iq):
    """48^3 grid, ~1500 G-vectors, optical and finite q, with 4 occupied + 40 unoccupied states."""
    wl = synth.config1(n_occ=4, n_unocc=40, which_q=(0, 1))
    ref = oracle_q(wl, iq)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl, iq)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ec, F = ctx.ec(ks, kqs, qs, fr, "fp64")
        ec16, _ = ctx.ec(ks, kqs, qs, fr, "split_fp16")
        ecb, _ = ctx.ec(ks, kqs, qs, fr, "split_bf16")
        ctx.check()
        ec, ec16, ecb = float(ec.cpu()[0]), float(ec16.cpu()[0]), float(ecb.cpu()[0])
    print(f"o2box q{iq}: NG={len(gm)} E64={ec:.12f} Efp16={ec16:.12f} Ebf16={ecb:.12f} ref={ref['E']:.12f}",
          flush=True)
    assert abs(ec - ref["E"]) < 1e-10
    assert abs(ec16 - ref["E"]) < 1e-6
    assert abs(ecb - ref["E"]) < 1e-6


@pytest.mark.parametrize("variant", [1, 4, 5])
@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_split_kernel_variants(rpa, variant, prec):
    """The split rank-k kernels (64x64 tiles; 64x128 pipelined with FP64 accumulation, four or eight waves)
    against the oracle on the 16^3 workload (NG = 126) and a tiny grid (NG = 15: one tile, mostly
    padding)."""
    for wl in (synth.config0(), synth.tiny(grid=(8, 8, 8))):
        ref = oracle_q(wl)
        ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
        with rpa.Context(wl.A, wl.grid) as ctx:
            ctx.tune_set(len(gm), variant, prec)
            assert ctx.tune_get(len(gm), prec) == variant
            chi = ctx.chi0(ks, kqs, qs, fr, prec).cpu().numpy()
            ec, F = ctx.ec(ks, kqs, qs, fr, prec)
            ctx.check()
        r = _rel(chi, ref["chi"])
        dE = float(ec.cpu()[0]) - ref["E"]
        print(f"variant {variant} {prec} NG={len(gm)}: chi rel={r:.3e} dE={dE:.3e}", flush=True)
        assert r < 2e-4
        assert abs(dE) < 1e-6


@pytest.mark.parametrize("prec", ["fp64", "split_fp16"])
def test_batched_graph_replays_match_per_q_calls(rpa, prec):
    """Several q-points in one call, captured into a graph and replayed three times with eager work and
    synchronisations in between; every replay is bit-identical to the eager batched call, which agrees with
    the per-q calls and the oracle, and the weighted sum is formed."""
    wl = synth.tiny(grid=(12, 12, 12), L=(8.0, 8.5, 9.0), n_occ=3, n_unocc=9, target_ng=40)
    Bm = 2 * np.pi * np.linalg.inv(wl.A).T
    qpts = [synth.QPoint(q=f * Bm[0] + g * Bm[1], ecut=synth.ecut_for_count(wl.A, f * Bm[0] + g * Bm[1], t),
                         weight=w)
            for f, g, t, w in ((0.1, 0.0, 40, 0.5), (0.25, 0.1, 25, 0.3), (0.0, 0.3, 60, 0.2))]
    wl.qpoints = qpts
    ks = [rpa.States.from_synth(wl.kpoints[0], wl.paw, "cuda:0")]
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    qspecs = []
    for qp in qpts:
        gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
        qspecs.append(rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight))
    with rpa.Context(wl.A, wl.grid) as ctx:
        per_q = []
        for qs in qspecs:
            e, _ = ctx.ec(ks, ks, qs, fr, prec)
            per_q.append(float(e.cpu()[0]))
        ec0, F0 = ctx.ec_batched(ks, ks, qspecs, fr, prec, use_graph=False)
        ctx.check()
        eager = ec0.cpu().numpy().copy()
        # the batch shares one x-y pair transform over the three spheres' box (a wider box can move the y
        # pass from quads of lanes to whole lines: FP32 rounding, not bits, may differ from a single-q call)
        rtol = 1e-12 if prec == "fp64" else 1e-6
        assert np.allclose(eager[:3], per_q, rtol=rtol, atol=0)
        assert abs(eager[3] - sum(q.weight * e for q, e in zip(qspecs, eager[:3]))) < 1e-13
        out = None
        for rep in range(3):
            out = ctx.ec_batched(ks, ks, qspecs, fr, prec, use_graph=True, out=out)
            ctx.check()
            got = out[0].cpu().numpy().copy()
            print(f"{prec} replay {rep}: {got}", flush=True)
            assert np.array_equal(got, eager), (rep, got, eager)
            # eager work between replays reuses the same context
            e, _ = ctx.ec(ks, ks, qspecs[1], fr, prec)
            torch.cuda.synchronize()
            assert float(e.cpu()[0]) == per_q[1]
        # the oracle for each q
        for qs, qp, e in zip(qspecs, qpts, per_q):
            wl1 = synth.Workload(name="t", A=wl.A, grid=wl.grid, kpoints=wl.kpoints, paw=wl.paw, qpoints=[qp],
                                 omega=wl.omega, omega_weight=wl.omega_weight, seed=0)
            ref = oracle_q(wl1)
            assert abs(e - ref["E"]) < (1e-10 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("pair", [(4, 5)])
@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_split_kernel_twins_are_bit_identical(rpa, prec, pair):
    """Variant 5 issues the same products in the same order as variant 4 (the same tiles split over eight
    waves instead of four): chi0 is bit-identical, here on the 48^3 grid (NG = 1500) with 2 x 300 pairs
    (19 K-steps: two FP64 flushes and a ragged last step)."""
    wl = synth.config1(n_occ=2, n_unocc=300, which_q=(1,))
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    out = {}
    with rpa.Context(wl.A, wl.grid) as ctx:
        for v in pair:
            ctx.tune_set(len(gm), v, prec)
            out[v] = ctx.chi0(ks, kqs, qs, fr, prec).cpu().numpy()
        ctx.check()
    a, b = pair
    print(f"{prec} {pair}: max|chi| = {np.abs(out[a]).max():.3e}", flush=True)
    assert np.abs(out[a]).max() > 0
    assert np.array_equal(out[a], out[b])


def _golden_o2box():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "o2box_ec.json")
    with open(path) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def o2box_full():
    return synth.config1()


@pytest.mark.parametrize("iq", [0, 1])
def test_o2box_full_size_against_oracle(rpa, o2box_full, iq):
    """All 16 x 800 pairs of the O2-in-box workload (NG ~ 1500, 16 frequencies) at the optical q-point and
    at q = 0.1 x 2 pi/12: E_c(q) and F(w) of the FP64 path within 1e-10 Ha of the oracle, and of both split
    precisions within 1e-6 Ha. The oracle's values were written by tests/golden/make_o2box_ec.py, which
    calls the FP64 CPU oracle alone on the same seeded inputs."""
    wl = o2box_full
    gold = _golden_o2box()["qpoints"][iq]
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl, iq)
    assert len(gm) == gold["NG"]
    with rpa.Context(wl.A, wl.grid) as ctx:
        e64, F64 = ctx.ec(ks, kqs, qs, fr, "fp64")
        eb, Fb = ctx.ec(ks, kqs, qs, fr, "split_bf16")
        eh, Fh = ctx.ec(ks, kqs, qs, fr, "split_fp16")
        ctx.check()
    e64, eb, eh = (float(x.cpu()[0]) for x in (e64, eb, eh))
    Fref = np.asarray(gold["F"])
    print(f"o2box q{iq}: NG={len(gm)} ref={gold['E_c']:.12f} fp64 dE={e64 - gold['E_c']:.3e} "
          f"bf16 dE={eb - gold['E_c']:.3e} fp16 dE={eh - gold['E_c']:.3e}", flush=True)
    assert abs(e64 - gold["E_c"]) < 1e-10
    assert np.max(np.abs(F64.cpu().numpy() - Fref)) < 1e-9
    assert abs(eb - gold["E_c"]) < 1e-6
    assert abs(eh - gold["E_c"]) < 1e-6


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_o2box_full_size_chi0_band_subset(rpa, o2box_full, prec):
    """chi0 of the O2-in-box q-point 1 (NG = 1500) element by element against the oracle on a band subset:
    all 16 occupied states and every 37th unoccupied one (352 pairs)."""
    wl = o2box_full
    s = wl.kpoints[0]
    keep = np.concatenate([np.arange(16), 16 + np.arange(0, 800, 37)])
    sub = synth.StateSet(kpt=s.kpt, weight=s.weight, miller=s.miller, C=np.ascontiguousarray(s.C[keep]),
                         eps=s.eps[keep].copy(), f=s.f[keep].copy(), P=np.ascontiguousarray(s.P[keep]))
    wl1 = synth.Workload(name="sub", A=wl.A, grid=wl.grid, kpoints=[sub], paw=wl.paw, qpoints=[wl.qpoints[1]],
                         omega=wl.omega, omega_weight=wl.omega_weight, seed=0)
    ref = oracle_q(wl1)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl1)
    with rpa.Context(wl.A, wl.grid) as ctx:
        chi = ctx.chi0(ks, kqs, qs, fr, prec).cpu().numpy()
        ec, _ = ctx.ec(ks, kqs, qs, fr, prec)
        ctx.check()
    r = _rel(chi, ref["chi"])
    dE = float(ec.cpu()[0]) - ref["E"]
    print(f"o2box subset {prec}: pairs={16 * len(keep[16:])} chi rel={r:.3e} dE={dE:.3e}", flush=True)
    assert r < (1e-12 if prec == "fp64" else 2e-4)
    assert abs(dE) < (1e-10 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("variant", [4, 5])
@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("case", ["o2box_chunks", "slab_two_k"])
def test_split_accumulate_branch(rpa, prec, case, variant):
    """Updates after the first one into a q-point's accumulator (the branch that reads C and adds): the pair
    sum split into chunks by a bound on the chunk size, over one k set at NG = 1500 (4 x 40 pairs in chunks
    of 64) and over two k sets of the metal slab at NG ~ 500 (chunks of 48). chi0 element by element and
    E_c against the oracle."""
    if case == "o2box_chunks":
        wl = synth.config1(n_occ=4, n_unocc=40, which_q=(1,))
        chunk = 64
    else:
        wl = synth.config2(n_below=6, n_above=24, nk=2, target_ng=500)
        chunk = 48
    ref = oracle_q(wl)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    npairs = [int(np.sum(s.f[:, None] - t.f[None, :] > 1e-8)) for s, t in zip(wl.kpoints, wl.kq_sets())]
    nchunks = sum((p + chunk - 1) // chunk for p in npairs)
    assert nchunks >= 3
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.tune_set(len(gm), variant, prec)
        ctx.set_chunk_pairs(chunk)
        chi = ctx.chi0(ks, kqs, qs, fr, prec).cpu().numpy()
        ec, _ = ctx.ec(ks, kqs, qs, fr, prec)
        ctx.set_chunk_pairs(0)
        chi1 = ctx.chi0(ks, kqs, qs, fr, prec).cpu().numpy()
        ctx.check()
    r = _rel(chi, ref["chi"])
    dE = float(ec.cpu()[0]) - ref["E"]
    print(f"{case} {prec}: NG={len(gm)} pairs={npairs} chunks={nchunks} chi rel={r:.3e} dE={dE:.3e} "
          f"vs one chunk {_rel(chi, chi1):.3e}", flush=True)
    assert r < 2e-4
    assert abs(dE) < 1e-6
    assert _rel(chi, chi1) < 1e-6


def test_nan_workspace_does_not_reach_an_uneven_batch(rpa):
    """A failed factorisation (a chi0 with 1 - K not positive definite) leaves NaN in the context's chi0
    workspace; an uneven split batch on the same context afterwards must not see it: its E_c values are
    finite and bit-identical to the same batch on a fresh context."""
    wl = synth.config3(n_occ=2, n_unocc=10, nq=4)
    ks = [rpa.States.from_synth(wl.kpoints[0], wl.paw, "cuda:0")]
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    qspecs, ngs = [], []
    for qp in wl.qpoints:
        gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
        ngs.append(len(gm))
        qspecs.append(rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight))
    # smallest sphere first: its accumulator (padded to the largest sphere) is where the NaN lands
    order = np.argsort(ngs)
    qspecs = [qspecs[i] for i in order]
    ngs = [ngs[i] for i in order]
    assert (ngs[0] + 63) // 64 < (ngs[-1] + 63) // 64
    nbig = ngs[-1]
    # +1e3 on the diagonal of chi0: 1 - K has large negative eigenvalues at every frequency
    bad = torch.zeros((len(wl.omega), nbig, nbig), dtype=torch.complex128, device="cuda:0")
    bad.diagonal(dim1=1, dim2=2).fill_(1e3)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.set_autotune(False)
        # the batch first, so that its workspace is allocated and the failed call below writes into it
        e0, _ = ctx.ec_batched(ks, ks, qspecs, fr, "split_bf16")
        ctx.check()
        first = e0.cpu().numpy().copy()
        ctx.ec_from_chi0(qspecs[-1], fr, bad)
        with pytest.raises(rpa.RpaError) as ei:
            ctx.check()
        assert ei.value.status == -5
        e1, _ = ctx.ec_batched(ks, ks, qspecs, fr, "split_bf16")
        ctx.check()
        got = e1.cpu().numpy().copy()
    assert np.array_equal(first, got)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.set_autotune(False)
        e2, _ = ctx.ec_batched(ks, ks, qspecs, fr, "split_bf16")
        ctx.check()
        fresh = e2.cpu().numpy().copy()
    print(f"NG={ngs} after NOT_PD: {got} fresh: {fresh}", flush=True)
    assert np.all(np.isfinite(got))
    assert np.array_equal(got, fresh)


def test_autotune_records_a_variant(rpa):
    with rpa.Context(np.eye(3) * 10.0, (16, 16, 16)) as ctx:
        v = ctx.autotune(NG=700, npairs=512, nw=4, precision="split_bf16")
        assert v in (1, 4, 5)
        assert ctx.tune_get(700, "split_bf16") == v


def test_calls_autotune_per_size_bucket(rpa):
    """A split call with a sphere in a new size bucket records a variant for it (and the call's result stays
    within the split bound of the FP64 path)."""
    wl = synth.config1(n_occ=2, n_unocc=20, which_q=(1,))
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ng = len(gm)
        before = ctx.tune_get(ng, "split_bf16")
        e, _ = ctx.ec(ks, kqs, qs, fr, "split_bf16")
        e64, _ = ctx.ec(ks, kqs, qs, fr, "fp64")
        ctx.check()
        after = ctx.tune_get(ng, "split_bf16")
        print(f"NG={ng}: default variant {before}, tuned {after}", flush=True)
        assert after in (1, 4, 5)
        assert abs(float(e.cpu()[0]) - float(e64.cpu()[0])) < 1e-6


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
@pytest.mark.parametrize("name", ["tiny10_metal_optical", "tiny12_spin"])
def test_chi0_and_ec_split_metal_and_spin(rpa, name, prec):
    """The intraband head and the spin sum through the split precisions."""
    wl = WORKLOADS[name]()
    ref = oracle_q(wl)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        chi = ctx.chi0(ks, kqs, qs, fr, prec).cpu().numpy()
        ec, _ = ctx.ec(ks, kqs, qs, fr, prec)
        ctx.check()
    r = _rel(chi, ref["chi"])
    dE = float(ec.cpu()[0]) - ref["E"]
    print(f"{name} {prec}: chi rel={r:.3e} dE={dE:.3e}", flush=True)
    assert r < 2e-4
    assert abs(dE) < 1e-6


def test_intraband_head_needs_no_adjoint(rpa):
    """The adjoint has no intraband term: a set with -df/de at an optical q-point is refused before any
    launch."""
    wl = WORKLOADS["tiny10_metal_optical"]()
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        with pytest.raises(rpa.RpaError) as ei:
            ctx.ec_backward(ks[0], kqs[0], qs, fr)
        assert ei.value.status == -7


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
@pytest.mark.parametrize("name", ["tiny8", "tiny10_optical", "tiny10_metal_optical", "cfg0"])
def test_chi0_real_frequencies(rpa, name, prec):
    """chi0(q, w + i eta) at real frequencies of both signs against the oracle (reading: Eq. chi0 with
    i w -> w + i eta, orderings paired), element by element; at w = 0, eta = w' it equals the imaginary-axis
    chi0 at i w'."""
    wl = WORKLOADS[name]()
    qp = wl.qpoints[0]
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    s = wl.kpoints
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
    D = synth.paw_d_table(wl.paw)
    om, eta = np.array([-1.3, -0.2, 0.0, 0.15, 0.6, 2.4]), 0.04
    ref = oracle.chi0_q_real(wl.A, wl.grid, s, wl.kq_sets(), gm, Q, wl.paw.offsets, om, eta, optical=qp.optical,
                             qhat=qp.qhat, Dtab=D)
    with rpa.Context(wl.A, wl.grid) as ctx:
        chi = ctx.chi0_real(ks, kqs, qs, om, eta, prec).cpu().numpy()
        z = ctx.chi0_real(ks, kqs, qs, [0.0], float(wl.omega[2]), prec).cpu().numpy()
        ci = ctx.chi0(ks, kqs, qs, fr, prec).cpu().numpy()
        ctx.check()
    r = _rel(chi, ref)
    print(f"{name} {prec}: real-frequency chi0 rel={r:.3e}, continuation {_rel(z[0], ci[2]):.3e}", flush=True)
    tol = 1e-12 if prec == "fp64" else 2e-4
    assert r < tol
    assert _rel(z[0], ci[2]) < tol
