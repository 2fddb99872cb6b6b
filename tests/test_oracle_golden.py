"""The oracle against its stored run on the 64x64 grid configuration
(tests/golden/grid64_oracle.json, written by tests/golden/make_golden.py from
the oracle alone): a change of the oracle's arithmetic shows up here and has
to be justified by the passage of the paper it follows."""
import importlib.util
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_matches_its_golden_run():
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    with open(os.path.join(HERE, "golden", "grid64_oracle.json")) as f:
        want = json.load(f)
    got = mg.run()
    assert got["status"] == want["status"]
    assert len(got["rounds"]) == len(want["rounds"])
    for l, (a, b) in enumerate(zip(got["rounds"], want["rounds"])):
        assert a["cg_iters"] == b["cg_iters"], l
        for f in mg.FIELDS:
            if f != "cg_iters":
                assert a[f] == pytest.approx(b[f], rel=1e-12, abs=1e-300), (l, f)
    for f in ("potentials_sum", "potentials_norm2"):
        assert got[f] == pytest.approx(want[f], rel=1e-12)
    assert got["sweep"] == want["sweep"]
