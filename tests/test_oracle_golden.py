"""The oracle reproduces its stored snapshots bit for bit
(tests/golden/oracle_snapshots.json, written by tests/golden/make_golden.py
from the oracle alone): time steps and sampled cells of small seeded runs
covering walls, outflow, friction laws, rain and Green-Ampt, imposed
boundaries, first order and the three fluxes.  A failure means the
oracle's arithmetic changed; such a change must be justified by the paper
and the snapshots rewritten by the script."""

import importlib.util
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _generator():
    spec = importlib.util.spec_from_file_location("make_golden",
                                                  os.path.join(GOLDEN, "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


GEN = _generator()
STORED = json.load(open(os.path.join(GOLDEN, "oracle_snapshots.json")))["cases"]


@pytest.mark.parametrize("name,wl,steps", GEN.cases(), ids=[c[0] for c in GEN.cases()])
def test_oracle_matches_snapshot(name, wl, steps):
    ref = STORED[name]
    got = GEN.snapshot(wl, steps)
    assert got["rc"] == ref["rc"] and got["steps"] == ref["steps"]
    assert got["cells"] == ref["cells"]
    assert got["dts"] == ref["dts"] and got["t"] == ref["t"]
    for k in ("h", "qx", "qy", "vinf"):
        assert (k in got) == (k in ref), k
        if k in ref:
            assert got[k] == ref[k], k
