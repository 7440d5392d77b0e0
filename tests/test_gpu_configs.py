"""The metal-slab and uneven-batch workload shapes, through the C ABI: at reduced band counts against the
oracle, and the metal slab at full size (split against FP64 over one k-point, sampled pair densities
against the oracle).

Same cells, grids, occupations and PAW sizes as the full workloads (9 x 9 x 36 bohr, 40 x 40 x 160 grid,
20 atoms x 18 projectors), with fewer states so that the FP64 oracle finishes in seconds:
  metal slab  - two k-points off Gamma, Fermi-smeared occupations (T = 0.01 Ha), 6 + 24 states,
                NG = 303;
  uneven batch - eight q-points of the 4 x 4 x 4 mesh with spheres of 252 to 1752 vectors, 4 + 24 states.
The 40 x 40 x 160 grid runs x and y through the register kernels and z by quads of lanes (path 0), or all
three axes through the LDS passes (path 1).
"""
import dataclasses

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


def _split_tol(E):
    return 1e-6


@pytest.fixture(scope="module")
def slab():
    wl = synth.config2(n_below=6, n_above=24, nk=2, target_ng=300)
    return wl, oracle_q(wl)


@pytest.mark.parametrize("path", [0, 1])
def test_metal_slab_reduced(rpa, slab, path):
    wl, ref = slab
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    assert np.array_equal(gm, ref["gm"])
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.set_pair_path(path)
        chi = ctx.chi0(ks, kqs, qs, fr, "fp64").cpu().numpy()
        ec, F = ctx.ec(ks, kqs, qs, fr, "fp64")
        ecs, _ = ctx.ec(ks, kqs, qs, fr, "split_bf16")
        ctx.check()
    ec, ecs, F = float(ec.cpu()[0]), float(ecs.cpu()[0]), F.cpu().numpy()
    r = _rel(chi, ref["chi"])
    print(f"slab path {path}: NG={len(gm)} chi rel={r:.3e} E={ec:.12f} ref={ref['E']:.12f} "
          f"dE={ec - ref['E']:.3e} split dE={ecs - ref['E']:.3e}", flush=True)
    assert r < 1e-12
    assert np.max(np.abs(F - ref["F"])) < 1e-10
    assert abs(ec - ref["E"]) < 1e-10
    assert abs(ecs - ref["E"]) < _split_tol(ref["E"])


def test_uneven_batch_reduced(rpa):
    """Eight q-points in one call (one leading dimension, padded to the largest sphere): equal to the per-q
    calls, a captured graph replay bit-identical to the eager call, the small spheres against the oracle,
    and the split precision within its bound of the FP64 batch."""
    wl = synth.config3(n_occ=4, n_unocc=24, nq=8)
    ks = [rpa.States.from_synth(wl.kpoints[0], wl.paw, "cuda:0")]
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    qspecs, ngs = [], []
    for qp in wl.qpoints:
        gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
        ngs.append(len(gm))
        qspecs.append(rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight))
    assert min(ngs) < 300 and max(ngs) > 1700
    with rpa.Context(wl.A, wl.grid) as ctx:
        per_q = []
        for qs in qspecs:
            e, _ = ctx.ec(ks, ks, qs, fr, "fp64")
            per_q.append(float(e.cpu()[0]))
        ec0, _ = ctx.ec_batched(ks, ks, qspecs, fr, "fp64")
        eager = ec0.cpu().numpy().copy()
        out = ctx.ec_batched(ks, ks, qspecs, fr, "fp64", use_graph=True)
        out = ctx.ec_batched(ks, ks, qspecs, fr, "fp64", use_graph=True, out=out)
        graph = out[0].cpu().numpy().copy()
        ecs, _ = ctx.ec_batched(ks, ks, qspecs, fr, "split_bf16")
        ctx.check()
        split = ecs.cpu().numpy()
    print(f"NG={ngs} E={eager[:len(ngs)]}", flush=True)
    assert np.allclose(eager[:len(ngs)], per_q, rtol=1e-12, atol=0)
    assert np.array_equal(graph, eager)
    assert abs(eager[len(ngs)] - sum(q.weight * e for q, e in zip(qspecs, per_q))) < 1e-12 * max(1.0, abs(eager[len(ngs)]))
    for i, e in enumerate(eager[:len(ngs)]):
        assert abs(split[i] - e) < _split_tol(e), (i, split[i], e)
    small = [i for i, n in enumerate(ngs) if n < 400]
    assert len(small) >= 3
    for i in small:
        wl1 = synth.Workload(name="t", A=wl.A, grid=wl.grid, kpoints=wl.kpoints, paw=wl.paw,
                             qpoints=[wl.qpoints[i]], omega=wl.omega, omega_weight=wl.omega_weight, seed=0)
        ref = oracle_q(wl1)
        print(f"q{i} NG={ngs[i]}: E={eager[i]:.12f} ref={ref['E']:.12f}", flush=True)
        assert abs(eager[i] - ref["E"]) < 1e-10


def test_uneven_batch_split_graph_replays(rpa):
    """Split precision on the slab grid in a captured graph (z passes by quads of lanes, the per-n PAW form,
    per-class chi0 storage): three replays, each after an eager call of another shape on the same context,
    every replay bit-identical to the eager batch."""
    wl = synth.config3(n_occ=4, n_unocc=24, nq=4)
    ks = [rpa.States.from_synth(wl.kpoints[0], wl.paw, "cuda:0")]
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    qspecs = []
    for qp in wl.qpoints:
        gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
        qspecs.append(rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight))
    with rpa.Context(wl.A, wl.grid) as ctx:
        eager = ctx.ec_batched(ks, ks, qspecs, fr, "split_bf16")[0].cpu().numpy().copy()
        out = None
        for rep in range(3):
            ctx.ec(ks, ks, qspecs[rep % len(qspecs)], fr, "split_bf16")
            out = ctx.ec_batched(ks, ks, qspecs, fr, "split_bf16", use_graph=True, out=out)
            got = out[0].cpu().numpy().copy()
            ctx.check()
            print(f"replay {rep}: {got[:len(qspecs)]}", flush=True)
            assert np.array_equal(got, eager), rep


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_chi0_add_sums_over_k(rpa, slab, prec):
    """rpa_chi0_add one k-point at a time gives the chi0 of rpa_chi0 over both k-points (Eq. chi0's k sum),
    and the oracle's."""
    wl, ref = slab
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl)
    with rpa.Context(wl.A, wl.grid) as ctx:
        both = ctx.chi0(ks, kqs, qs, fr, prec)
        acc = torch.zeros_like(both)
        for i in range(len(ks)):
            ctx.chi0_add([ks[i]], [kqs[i]], qs, fr, acc, prec)
        ctx.check()
    both, acc = both.cpu().numpy(), acc.cpu().numpy()
    print(f"{prec}: chi0_add vs chi0 {_rel(acc, both):.3e}, vs oracle {_rel(acc, ref['chi']):.3e}", flush=True)
    assert _rel(acc, both) < 1e-13
    assert _rel(acc, ref["chi"]) < (1e-12 if prec == "fp64" else 2e-4)


@pytest.mark.parametrize("iq", [0, 1])
def test_spin_polarised_o2box_reduced(rpa, iq):
    """Spin-polarised O2-in-box shape (two channels with f in [0, 1], 5 + 39 and 3 + 41 states: a moment
    of 2, as in the O2 triplet), optical and finite q: chi0 and E_c of the two channels together against
    the oracle (Eq. chi0 with the spin sum written out as two state sets)."""
    wl = synth.config1(n_occ=4, n_unocc=40, which_q=(0, 1), spin_moment=2)
    assert len(wl.kpoints) == 2 and wl.kpoints[0].f.max() == 1.0
    ref = oracle_q(wl, iq)
    ks, kqs, qs, fr, gm = gpu_inputs(rpa, wl, iq)
    with rpa.Context(wl.A, wl.grid) as ctx:
        chi = ctx.chi0(ks, kqs, qs, fr, "fp64").cpu().numpy()
        ec, F = ctx.ec(ks, kqs, qs, fr, "fp64")
        ecs, _ = ctx.ec(ks, kqs, qs, fr, "split_bf16")
        ctx.check()
    ec, ecs = float(ec.cpu()[0]), float(ecs.cpu()[0])
    r = _rel(chi, ref["chi"])
    print(f"spin q{iq}: NG={len(gm)} chi rel={r:.3e} E={ec:.12f} ref={ref['E']:.12f} split dE={ecs - ref['E']:.3e}",
          flush=True)
    assert r < 1e-12
    assert abs(ec - ref["E"]) < 1e-10
    assert abs(ecs - ref["E"]) < 1e-6


def test_metal_slab_full_size_one_kpoint(rpa):
    """The metal slab at full size (120 + 3000 Fermi-smeared states, NG = 4011, 20 x 18 projectors, 16
    frequencies), k-point 0 alone: split-precision E_c of that k-point's chi0 within 1e-6 Ha of the FP64
    path (the FP64 path itself is pinned to the oracle at full O2-box size, at every reduced size and, on
    sampled pairs and G-vectors, at this size: the tests below), chi0
    of the two paths within the split tolerance, about 20 chunks of the split kernel's accumulate branch."""
    dev = "cuda:0"
    wl = synth.config2(device=dev)
    s = wl.kpoints[0]
    qp = wl.qpoints[0]
    gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
    assert len(gm) == 4011
    qs = rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight, device=dev)
    st = rpa.States.from_synth(s, wl.paw, dev)
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.set_chunk_pairs(50000)
        chi64 = ctx.chi0([st], [st], qs, fr, "fp64")
        e64 = float(ctx.ec_from_chi0(qs, fr, chi64)[0].cpu()[0])
        chis = ctx.chi0([st], [st], qs, fr, "split_bf16")
        es = float(ctx.ec_from_chi0(qs, fr, chis)[0].cpu()[0])
        ctx.check()
        diff = float(torch.max(torch.abs(chis - chi64)).cpu()) / float(torch.max(torch.abs(chi64)).cpu())
    print(f"slab k0: E_fp64={e64:.12f} E_split={es:.12f} diff={es - e64:.3e} chi rel={diff:.3e}", flush=True)
    assert abs(es - e64) < 1e-6
    assert diff < 2e-4


# bands of the full metal-slab set (120 + 3000 states) sampled for the pair densities: deep, mid and top
# occupied states, the partly occupied ones at the Fermi level (f from 1.98 to 0.1) and far empty ones
SLAB_BANDS = [0, 60, 117, 119, 120, 121, 125, 140, 600, 3119]


@pytest.fixture(scope="module")
def slab_full_k0(rpa):
    """One k-point of the metal slab at full size: 120 + 3000 Fermi-smeared states on the 40 x 40 x 160
    grid, NG = 4011, 20 x 18 projectors; the library's state set and sphere, and the oracle's pair
    densities for every pair of SLAB_BANDS with f_n - f_m above the pair threshold (Eq. n_G_2, Sec. 2.2),
    computed from those bands alone."""
    dev = "cuda:0"
    wl = synth.config2(nk=1, device=dev)
    s, qp = wl.kpoints[0], wl.qpoints[0]
    gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
    ref_g = oracle.gsphere(wl.A, qp.q, qp.ecut)
    assert np.array_equal(gm, ref_g) and len(gm) == 4011
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, ref_g)
    keep = np.asarray(SLAB_BANDS)
    sub = dataclasses.replace(s, C=np.ascontiguousarray(s.C[keep]), eps=s.eps[keep].copy(), f=s.f[keep].copy(),
                              P=np.ascontiguousarray(s.P[keep]), dfde=None)
    pairs, rho = oracle.pair_densities(wl.A, wl.grid, sub, sub, ref_g, Q, wl.paw.offsets)
    qs = rpa.QSpec(qp.q, gm, Q, weight=qp.weight, device=dev)
    st = rpa.States.from_synth(s, wl.paw, dev)
    return dict(wl=wl, A=wl.A, grid=wl.grid, gm=ref_g, Q=Q, qs=qs, st=st, sub=sub, pn=keep[pairs[0]],
                pm=keep[pairs[1]], rho=rho, f=s.f)


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_metal_slab_full_size_pair_density_sample(rpa, slab_full_k0, prec, path):
    """Pair densities of the full-size metal slab (all 3120 states resident, NG = 4011, 20 x 18 projectors)
    for sampled pairs, element by element against the oracle: z by quads of lanes (path 0) and the LDS
    passes (path 1); FP64 transforms to 1e-12 and the FP32 transforms of the split path to 2e-6 of
    max |rho|, the bounds of every other grid."""
    d = slab_full_k0
    pn, pm = d["pn"], d["pm"]
    assert len(pn) >= 30 and np.any((d["f"][pn] < 2.0 - 1e-3) & (d["f"][pm] > 1e-3))
    with rpa.Context(d["A"], d["grid"]) as ctx:
        ctx.set_pair_path(path)
        rho = ctx.pair_density(d["st"], d["st"], d["qs"], pn, pm, prec).cpu().numpy()
        ctx.check()
    r = _rel(rho, d["rho"])
    print(f"slab full {prec} path {path}: pairs={len(pn)} NG={rho.shape[1]} rel={r:.3e}", flush=True)
    assert r < (1e-12 if prec == "fp64" else 2e-6)


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_metal_slab_full_size_chi0_sampled_block(rpa, slab_full_k0, prec):
    """chi0 at the slab's full sphere (NG = 4011: 63 tiles of 64 with a ragged last one, 16 frequencies)
    from the pairs of SLAB_BANDS, on a block of sampled G-vectors (the first and last 64 and 200 spread
    between): the oracle computes chi0 on that G list alone (chi0(G, G') needs only rho(G) and rho(G')),
    the library the whole matrix; FP64 to 1e-12, split to 2e-4 of the block's largest element."""
    d = slab_full_k0
    wl, gm, NG = d["wl"], d["gm"], len(d["gm"])
    sel = np.unique(np.concatenate([np.arange(64), np.linspace(0, NG - 1, 200).astype(np.int64),
                                    np.arange(NG - 64, NG)]))
    ref = oracle.chi0_q(wl.A, wl.grid, [d["sub"]], [d["sub"]], gm[sel], d["Q"][:, sel], wl.paw.offsets,
                        wl.omega)
    st = rpa.States.from_synth(d["sub"], wl.paw, "cuda:0")
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    idx = torch.as_tensor(sel, device="cuda:0")
    with rpa.Context(wl.A, wl.grid) as ctx:
        chi = ctx.chi0([st], [st], d["qs"], fr, prec)
        ctx.check()
        blk = chi.index_select(1, idx).index_select(2, idx).cpu().numpy()
        del chi
    r = _rel(blk, ref)
    print(f"slab full chi0 {prec}: pairs={len(d['pn'])} NG={NG} block={len(sel)} rel={r:.3e}", flush=True)
    assert np.max(np.abs(ref)) > 0
    assert r < (1e-12 if prec == "fp64" else 2e-4)


def test_metal_slab_full_size_optical_head_sampled_block(rpa, slab_full_k0):
    """The metallic q -> 0 head at full slab size (Sec. 2.2 with Fermi-smeared bands): the bands of
    SLAB_BANDS with their -df/de, at the optical q-point along x (the q = 0 sphere, the nabla tables of the
    20 x 18 projectors): chi0 on a block of sampled G-vectors that holds G = 0 against the oracle's chi0 on
    that G list; the head (with the intraband term), the wings and the body each to 1e-12 (FP64) and 2e-4
    (split) of their own largest element."""
    d = slab_full_k0
    wl = d["wl"]
    s = wl.kpoints[0]
    keep = np.asarray(SLAB_BANDS)
    assert s.dfde is not None
    sub = dataclasses.replace(d["sub"], dfde=s.dfde[keep].copy())
    assert np.max(sub.dfde) > 1.0
    q0, qhat = np.zeros(3), np.array([1.0, 0.0, 0.0])
    ecut = wl.qpoints[0].ecut
    gm = rpa.gsphere(wl.A, wl.grid, q0, ecut)
    ref_g = oracle.gsphere(wl.A, q0, ecut)
    assert np.array_equal(gm, ref_g)
    NG = len(gm)
    zero = int(np.nonzero(np.all(ref_g == 0, axis=1))[0][0])
    sel = np.unique(np.concatenate([[zero], np.arange(64), np.linspace(0, NG - 1, 200).astype(np.int64),
                                    np.arange(NG - 64, NG)]))
    Q = synth.paw_q_table(wl.paw, wl.A, q0, ref_g)
    D = synth.paw_d_table(wl.paw)
    ref = oracle.chi0_q(wl.A, wl.grid, [sub], [sub], ref_g[sel], Q[:, sel], wl.paw.offsets, wl.omega,
                        optical=True, qhat=qhat, Dtab=D)
    qs = rpa.QSpec(q0, gm, Q, optical=True, qhat=qhat, Dpaw=D, device="cuda:0")
    st = rpa.States.from_synth(sub, wl.paw, "cuda:0")
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    idx = torch.as_tensor(sel, device="cuda:0")
    z = int(np.nonzero(sel == zero)[0][0])
    out = {}
    with rpa.Context(wl.A, wl.grid) as ctx:
        for prec in ("fp64", "split_bf16"):
            chi = ctx.chi0([st], [st], qs, fr, prec)
            ctx.check()
            out[prec] = chi.index_select(1, idx).index_select(2, idx).cpu().numpy()
            del chi
    # the intraband head outweighs the rest of the block by four orders: head, wings (G = 0 row and column)
    # and body are each compared with their own largest element
    body = np.ones(len(sel), dtype=bool)
    body[z] = False
    parts = {"head": lambda c: c[:, z, z], "wings": lambda c: np.concatenate([c[:, z, body], c[:, body, z]], axis=1),
             "body": lambda c: c[:, body][:, :, body]}
    for name, part in parts.items():
        r64, rs = _rel(part(out["fp64"]), part(ref)), _rel(part(out["split_bf16"]), part(ref))
        print(f"slab full optical {name}: NG={NG} block={len(sel)} max={np.max(np.abs(part(ref))):.3e} "
              f"fp64 rel={r64:.3e} split rel={rs:.3e}", flush=True)
        assert np.max(np.abs(part(ref))) > 0
        assert r64 < 1e-12
        assert rs < 2e-4
