"""rpa_ec_batched_sets through the C ABI: q-points with state-set lists of their own (Eq. rpa_c's q sum over
Eq. chi0's k sum) in one batched call, eager and from a replayed graph, against per-q rpa_ec calls with the
same sets (within 1e-13) and against the oracle (FP64 1e-10 Ha, split 1e-6 Ha)."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rpa():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1307_8052_amd as m
    return m


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_batched_sets_match_per_q_calls_and_oracle(rpa, prec):
    wl = synth.tiny(grid=(12, 12, 12), L=(8.0, 8.5, 9.0), n_occ=3, n_unocc=9, target_ng=40, extra_kq=True)
    s, t = wl.kpoints[0], wl.kq[0]
    Bm = oracle.reciprocal_rows(wl.A)
    qpts = [synth.QPoint(q=f * Bm[0] + g * Bm[1], ecut=synth.ecut_for_count(wl.A, f * Bm[0] + g * Bm[1], n),
                         weight=w)
            for f, g, n, w in ((0.1, 0.0, 40, 0.5), (0.25, 0.1, 25, 0.3), (0.0, 0.3, 60, 0.2))]
    # q 0: (s, t); q 1: (s, s) and (t, s), half weight each; q 2: (t, t)
    sh = dataclasses.replace(s, weight=0.5)
    th = dataclasses.replace(t, weight=0.5)
    oracle_sets = [([s], [t]), ([sh, th], [sh, s]), ([t], [t])]
    dev = "cuda:0"
    S = {id(x): rpa.States.from_synth(x, wl.paw, dev) for x in (s, t, sh, th)}
    sets = [([S[id(a)] for a in ks], [S[id(b)] for b in kqs]) for ks, kqs in oracle_sets]
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    qspecs = []
    for qp in qpts:
        gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
        qspecs.append(rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight, device=dev))
    with rpa.Context(wl.A, wl.grid) as ctx:
        per_q = [float(ctx.ec(ks, kqs, qs, fr, prec)[0].cpu()[0]) for (ks, kqs), qs in zip(sets, qspecs)]
        ec, _ = ctx.ec_batched_sets(sets, qspecs, fr, prec)
        eager = ec.cpu().numpy().copy()
        out = None
        for rep in range(2):
            out = ctx.ec_batched_sets(sets, qspecs, fr, prec, use_graph=True, out=out)
            got = out[0].cpu().numpy().copy()
            assert np.array_equal(got, eager), (rep, got, eager)
            e = float(ctx.ec(sets[1][0], sets[1][1], qspecs[1], fr, prec)[0].cpu()[0])
            assert e == per_q[1]
        ctx.check()
    print(f"{prec}: per-q {per_q} batched {eager}", flush=True)
    assert np.allclose(eager[:3], per_q, rtol=0, atol=1e-13)
    assert abs(eager[3] - sum(q.weight * e for q, e in zip(qpts, per_q))) < 1e-13
    for (ks, kqs), qp, e in zip(oracle_sets, qpts, per_q):
        gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
        Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
        E, _, _ = oracle.ec_q(wl.A, wl.grid, ks, kqs, gm, Q, wl.paw.offsets, qp.q, wl.omega, wl.omega_weight)
        assert abs(e - E) < (1e-10 if prec == "fp64" else 1e-6), (e, E)


@pytest.mark.parametrize("prec", ["fp64", "split_bf16"])
def test_shared_pair_transform_across_q(rpa, prec):
    """q-points that share every state set share each chunk's x-y pair transform (one box covering all
    spheres); with the same chunking as single-q calls the results agree with them to rounding (the wider
    box can switch the y pass from quads of lanes to whole lines), and each q-point matches the oracle. Spheres of 9, 42 and 60 G-vectors, chunks of 7 pairs (several chunks,
    a ragged last one)."""
    wl = synth.tiny(grid=(12, 12, 12), L=(8.0, 8.5, 9.0), n_occ=3, n_unocc=9, target_ng=40)
    Bm = oracle.reciprocal_rows(wl.A)
    qpts = [synth.QPoint(q=f * Bm[0] + g * Bm[1] + h * Bm[2],
                         ecut=synth.ecut_for_count(wl.A, f * Bm[0] + g * Bm[1] + h * Bm[2], n), weight=w)
            for f, g, h, n, w in ((0.1, 0.0, 0.0, 40, 0.5), (0.3, 0.2, 0.1, 9, 0.3), (0.0, 0.3, 0.2, 60, 0.2))]
    dev = "cuda:0"
    ks = [rpa.States.from_synth(wl.kpoints[0], wl.paw, dev)]
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    qspecs = []
    for qp in qpts:
        gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
        qspecs.append(rpa.QSpec(qp.q, gm, synth.paw_q_table(wl.paw, wl.A, qp.q, gm), weight=qp.weight, device=dev))
    ngs = sorted(q.NG for q in qspecs)
    assert ngs[0] < ngs[1] < ngs[2]
    with rpa.Context(wl.A, wl.grid) as ctx:
        ctx.set_chunk_pairs(7)
        per_q = [float(ctx.ec(ks, ks, qs, fr, prec)[0].cpu()[0]) for qs in qspecs]
        got = ctx.ec_batched(ks, ks, qspecs, fr, prec)[0].cpu().numpy()
        ctx.check()
    print(f"{prec}: per-q {per_q} batched {got[:3]}", flush=True)
    assert np.allclose(got[:3], per_q, rtol=1e-12 if prec == "fp64" else 1e-6, atol=0)
    for qp, e in zip(qpts, per_q):
        gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
        Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
        E, _, _ = oracle.ec_q(wl.A, wl.grid, wl.kpoints, wl.kpoints, gm, Q, wl.paw.offsets, qp.q, wl.omega,
                              wl.omega_weight)
        assert abs(e - E) < (1e-10 if prec == "fp64" else 1e-6), (e, E)
