"""Regression of the oracle against its committed fixture (tests/golden)."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_matches_committed_fixture():
    import sys
    sys.path.insert(0, os.path.join(HERE, "golden"))
    from make_golden import compute
    ref = json.load(open(os.path.join(HERE, "golden", "oracle_c1_sample.json")))
    got = compute()
    assert got["pairs"] == ref["pairs"]
    assert got["sel_id"] == ref["sel_id"]
    for k in ("rgb", "depth", "alpha", "feat_topk_0_4", "feat_full_0_4"):
        np.testing.assert_allclose(np.array(got[k]), np.array(ref[k]), rtol=1e-12, atol=1e-14, err_msg=k)
