"""Shared test helpers: run one synthetic workload through the oracle and through
the HIP library on the same inputs."""
import numpy as np

import oracle
import synth


def oracle_q(wl, iq=0, ik=None):
    """Oracle pieces for q-point iq: G-sphere, Q table, D table, chi0, F, E_c."""
    qp = wl.qpoints[iq]
    gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
    D = synth.paw_d_table(wl.paw)
    ks = wl.kpoints if ik is None else [wl.kpoints[ik]]
    kqs = wl.kq_sets() if ik is None else [wl.kq_sets()[ik]]
    E, F, chi = oracle.ec_q(wl.A, wl.grid, ks, kqs, gm, Q, wl.paw.offsets, qp.q, wl.omega, wl.omega_weight,
                            optical=qp.optical, qhat=qp.qhat, Dtab=D)
    return dict(gm=gm, Q=Q, D=D, E=E, F=F, chi=chi, qp=qp)


def gpu_inputs(rpa, wl, iq=0, device="cuda:0"):
    """Library-side inputs: the library's own G-sphere, the synthetic tables on it, device state sets."""
    qp = wl.qpoints[iq]
    gm = rpa.gsphere(wl.A, wl.grid, qp.q, qp.ecut)
    Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
    D = synth.paw_d_table(wl.paw)
    qs = rpa.QSpec(qp.q, gm, Q, optical=qp.optical, qhat=qp.qhat, Dpaw=D, weight=qp.weight, device=device)
    ks = [rpa.States.from_synth(s, wl.paw, device) for s in wl.kpoints]
    if wl.kq is None:
        kqs = ks
    else:
        kqs = [rpa.States.from_synth(s, wl.paw, device) for s in wl.kq]
    fr = rpa.Freq(wl.omega, wl.omega_weight)
    return ks, kqs, qs, fr, gm
