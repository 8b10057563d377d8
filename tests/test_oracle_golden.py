"""The oracle against its own recorded outputs (tests/golden/oracle_values.json,
written by tests/golden/make_golden.py from oracle/ only): any change of the
oracle's arithmetic shows here and must name, in its commit, the passage of
the paper that justifies it.  Libm may differ between hosts by an ulp or two,
hence the 1e-13 relative tolerance.  CPU only."""
import json
import os

import numpy as np

from tests.golden import make_golden

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_matches_its_record():
    rec = json.load(open(os.path.join(HERE, "golden", "oracle_values.json")))["cases"]
    now = make_golden.cases()
    assert set(rec) == set(now)
    for k, (pix, vals) in now.items():
        assert np.array_equal(np.asarray(rec[k]["pixels"]), pix), k
        want = np.asarray(rec[k]["values"])
        got = np.ravel(vals)
        scale = np.maximum(np.abs(want), 1e-300)
        assert np.all(np.abs(got - want) <= 1e-13 * scale + 1e-13 * np.abs(want).max()), k
