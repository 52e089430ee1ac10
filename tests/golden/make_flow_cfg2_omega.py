"""Write flow_cfg2_omega_dopri5_oracle.json: the oracle's adaptive
Dormand-Prince flow of the 24x24 / 96x96, N_ff = 13 workload (t' = -0.25,
filling 0.85, U = 3) with the Omega cutoff at zero temperature (Omega from 800
to 1e-3, stop at max|X| > 80).

Calls only oracle/ and the seeded workload definition in synth/.  The full
oracle flow takes many minutes on a CPU, too long for the test suite, so its
result is stored once and the GPU flow is compared with it.

    python tests/golden/make_flow_cfg2_omega.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import flow as oflow  # noqa: E402
from oracle.lattice import mu_from_filling  # noqa: E402


def main():
    w = synth.cfg2_omega()
    pt = w.points[0]
    pt.mu = mu_from_filling(pt.filling, pt.t, pt.tp, pt.mu_T, pt.mu_L)
    t0 = time.perf_counter()
    r = oflow.flow_dopri5(pt, w.T0, w.Tmin, w.Xmax, rtol=w.rtol, atol=w.atol, regulator="omega")
    el = time.perf_counter() - t0
    out = {
        "citation": "Sec. 3 (flow of the channel couplings from the bare interaction, with the Omega "
                    "cutoff as regulator) and Sec. 4 (start two orders of magnitude above the "
                    "bandwidth, stop at ten times the bandwidth; leading channel, ordering vector "
                    "and form-factor symmetry); written by the oracle only.",
        "workload": w.name,
        "point": {"t": pt.t, "tp": pt.tp, "U": pt.U, "Lq": pt.Lq, "Lk": pt.Lk, "shells": pt.shells,
                  "filling": pt.filling, "mu_T": pt.mu_T, "mu_L": pt.mu_L, "mu": pt.mu},
        "flow": {"scheme": "dopri5", "regulator": "omega", "Omega0": w.T0, "Omega_min": w.Tmin,
                 "Xmax": w.Xmax,
                 "rtol": w.rtol, "atol": w.atol},
        "status": {oflow.STATUS_DIVERGED: "diverged", oflow.STATUS_REACHED_TMIN: "reached_tmin",
                   oflow.STATUS_NONFINITE: "nonfinite"}[int(r.status)],
        "Omega_c": None if r.Tc is None else float(r.Tc), "channel": r.channel,
        "q_index": None if r.q_index is None else int(r.q_index), "irrep": r.irrep,
        "max_abs_X": float(r.max_abs_X), "n_rhs": int(r.n_rhs), "n_steps": int(r.n_steps),
        "oracle_seconds": el,
    }
    with open(os.path.join(HERE, "flow_cfg2_omega_dopri5_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
