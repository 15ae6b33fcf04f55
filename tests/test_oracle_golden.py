"""The oracle still reproduces its stored regression fixture (see
tests/golden/make_golden.py for what the fixture is and is not)."""
import os

import numpy as np

import oracle
from bem_inputs import octahedron_sphere
from golden.make_golden import CASES

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_matches_stored_fixture():
    m = octahedron_sphere(8)
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "oracle_sphere_entries.txt"))
            if not l.startswith("#")]
    assert len(rows) == 4 * 43
    for name, op in CASES.items():
        sel = [r for r in rows if r[0] == name]
        r = np.array([int(x[1]) for x in sel], dtype=np.int32)
        c = np.array([int(x[2]) for x in sel], dtype=np.int32)
        ref = np.array([float(x[3]) + 1j * float(x[4]) for x in sel])
        got = oracle.entries(m.v, m.tri, r, c, **op)
        assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-14, name
