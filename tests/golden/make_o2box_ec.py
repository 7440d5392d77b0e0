"""Write the oracle's E_c(q) and F(w) for the full O2-in-box workload (12 x 12 x 13 bohr, 48^3 grid,
16 occupied + 800 unoccupied states, 2 atoms x 13 projectors, NG ~ 1500, 16 imaginary frequencies;
q = 0 optical, 0.1 and 0.2 x 2 pi/12 along x) to ``o2box_ec.json``.

The values come from the FP64 CPU oracle alone (``oracle.ec_q`` on the seeded inputs of
``synth.config1``); nothing here touches the HIP library. Takes a few minutes.

Usage: python tests/golden/make_o2box_ec.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    wl = synth.config1()
    out = {"workload": "synth.config1() defaults (seed 1, paw_model 'overlap')", "digest": wl.digest(),
           "qpoints": []}
    D = synth.paw_d_table(wl.paw)
    for iq, qp in enumerate(wl.qpoints):
        t = time.time()
        gm = oracle.gsphere(wl.A, qp.q, qp.ecut)
        Q = synth.paw_q_table(wl.paw, wl.A, qp.q, gm)
        E, F, chi = oracle.ec_q(wl.A, wl.grid, wl.kpoints, wl.kq_sets(), gm, Q, wl.paw.offsets, qp.q,
                                wl.omega, wl.omega_weight, optical=qp.optical, qhat=qp.qhat, Dtab=D)
        diag = np.real(np.einsum("wgg->wg", chi))
        out["qpoints"].append({"iq": iq, "q": qp.q.tolist(), "optical": bool(qp.optical), "NG": int(len(gm)),
                               "E_c": E, "F": [float(x) for x in F],
                               "chi0_diag_w0_first16": [float(x) for x in diag[0, :16]],
                               "chi0_fro": [float(np.linalg.norm(c)) for c in chi]})
        print(f"q{iq}: NG={len(gm)} E_c={E:.15f} ({time.time() - t:.0f} s)", flush=True)
    with open(os.path.join(HERE, "o2box_ec.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
