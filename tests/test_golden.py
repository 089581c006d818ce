"""CPU: the oracle still gives the results stored in tests/golden/oracle_tiny.txt
(written by tests/golden/make_golden.py from the oracle itself): a guard
against silent drift of the oracle's arithmetic, not a pin of it (the pins
against mathematics are in test_oracle_pins.py)."""
import importlib.util
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _load(path):
    spec = importlib.util.spec_from_file_location("make_golden", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_oracle_matches_stored_results():
    mg = _load(os.path.join(HERE, "golden", "make_golden.py"))
    hits, nodes, dist = mg.compute()
    stored_hits, stored_nodes = {}, []
    for line in open(os.path.join(HERE, "golden", "oracle_tiny.txt")):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "hit":
            stored_hits.setdefault(float(f[1]), []).append((float(f[3]), int(f[4]), float(f[5]), float(f[6])))
        else:
            stored_nodes.append((int(f[1]), float(f[2])))
    assert sorted(stored_hits) == sorted(hits)
    for tau, rows in stored_hits.items():
        t, prim, u, v = hits[tau]
        assert len(rows) == len(t) == 128
        for i, (st, sp, su, sv) in enumerate(rows):
            assert prim[i] == sp, (tau, i)
            for a, b in ((t[i], st), (u[i], su), (v[i], sv)):
                assert (math.isinf(a) and math.isinf(b)) or abs(a - b) <= 1e-12 * max(1.0, abs(b)), (tau, i, a, b)
    assert [k for k, _ in stored_nodes] == [int(k) for k in nodes]
    assert np.allclose(dist, [d for _, d in stored_nodes], rtol=1e-12, atol=1e-15)
