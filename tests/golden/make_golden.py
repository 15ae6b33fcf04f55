"""Write ``oracle_sphere_entries.txt``: a regression fixture of oracle values.

The paper prints no per-integral values, so the stored values here are the
oracle's own, written by this script (which calls only ``oracle`` and the
seeded input generators).  They guard the oracle's arithmetic against silent
drift; its correctness is pinned separately (tests/test_oracle_pins.py).

Cases, all on the 512-triangle octahedron sphere (Sec. 4 geometry):
  slp_tri7_ss3   Laplace SLP, 7-point rule regular, Sauter-Schwab order 3
  dlp_q4         Laplace DLP, Duffy/Gauss order 4, Sauter-Schwab order 4
  helm_slp_k2_q4 Helmholtz SLP, kappa = 2, orders 4/4
  helm_dlp_k8_q5 Helmholtz DLP, kappa = 8, orders 5/5
Each case lists 40 seeded pairs plus one pair of every singular class.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from bem_inputs import octahedron_sphere, sample_pairs  # noqa: E402

CASES = {
    "slp_tri7_ss3": dict(kernel=0, layer=0, kappa=0.0, rule=1, q_reg=3, q_sing=3),
    "dlp_q4": dict(kernel=0, layer=1, kappa=0.0, rule=0, q_reg=4, q_sing=4),
    "helm_slp_k2_q4": dict(kernel=1, layer=0, kappa=2.0, rule=0, q_reg=4, q_sing=4),
    "helm_dlp_k8_q5": dict(kernel=1, layer=1, kappa=8.0, rule=0, q_reg=5, q_sing=5),
}


def pairs(m):
    r, c = sample_pairs(m.nt, 40, seed=7)
    extra_r, extra_c = [], []
    for cls in (3, 2, 1):
        j = next(j for j in range(m.nt) if oracle.shared_vertices(m.tri, 5, j) == cls)
        extra_r.append(5)
        extra_c.append(j)
    return np.concatenate([r, extra_r]).astype(np.int32), np.concatenate([c, extra_c]).astype(np.int32)


def main():
    m = octahedron_sphere(8)
    r, c = pairs(m)
    lines = ["# case row col re im   (written by make_golden.py; oracle values)"]
    for name, op in CASES.items():
        g = oracle.entries(m.v, m.tri, r, c, **op)
        for k in range(r.size):
            lines.append(f"{name} {r[k]} {c[k]} {g[k].real:.17e} {g[k].imag:.17e}")
    with open(os.path.join(HERE, "oracle_sphere_entries.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
