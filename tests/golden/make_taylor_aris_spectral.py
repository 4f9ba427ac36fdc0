"""Writes taylor_aris_spectral.json: the scheme's asymptotic dispersion
coefficient K and drift U in every channel of the seeded 64-channel
Taylor-Aris ensemble (Sec. 3.2), from the oracle's one-step symbol
(oracle.lbm.channel_dispersion), next to D_m (1 + Pe^2/210).  Uses only the
oracle and the seeded workload parameters.

    python tests/golden/make_taylor_aris_spectral.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lbm as O                                   # noqa: E402
from paper_1404_2363_amd import workloads as W                # noqa: E402


def channel_row(m):
    wl = W.taylor_aris_channel(m["h"], m["Pe"], m["tau"], nx=64, steps=1)
    prob = O.problem_for(wl, idx=[np.arange(3), np.arange(m["h"])], heat_rule=[1 / m["tau"]] * 2)
    K, U = O.channel_dispersion(prob, k=1e-3)
    Pe = m["U_node_mean"] * m["h"] / m["D_m"]
    K_ta = m["D_m"] * (1.0 + Pe * Pe / 210.0)
    return {"h": m["h"], "Pe": Pe, "tau": m["tau"], "K_scheme": float(K), "U_scheme": float(U),
            "K_taylor_aris": K_ta, "rel": float(K / K_ta - 1.0)}


def main():
    rows = [channel_row(r.meta) for r in W.taylor_aris_batch()]
    out = {"source": "oracle.lbm.channel_dispersion, k = 1e-3 with Richardson at 2k; "
                     "seeded ensemble workloads.taylor_aris_batch()", "channels": rows}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "taylor_aris_spectral.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}: max |K/K_TA - 1| = {max(abs(r['rel']) for r in rows):.4%}")


if __name__ == "__main__":
    main()
