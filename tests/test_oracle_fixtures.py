"""CPU checks of the stored oracle runs in tests/golden/ (written by
tests/golden/make_oracle_fixtures.py from the CPU oracle only): they were
made by the oracle sources as they are now (a change of the oracle's
arithmetic must be followed by regenerating them), and they are
internally consistent -- each run converged to its tolerance, its residual
history ends at the reported residual, and the samples have the stated
stride."""
import hashlib
import json
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def _sha(sources):
    h = hashlib.sha256()
    for src in sources:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


@pytest.mark.parametrize("name", ["oracle_c3_mgpcg_256.json",
                                  "oracle_c5_var7_128.json"])
def test_fixture_made_by_current_oracle(name):
    d = _load(name)
    assert d["written_by"].startswith("tests/golden/make_oracle_fixtures.py")
    assert d["oracle_sources_sha256"] == _sha(d["oracle_sources"]), \
        f"{name} predates the current oracle sources; regenerate it"


def test_c3_fixture_consistent():
    d = _load("oracle_c3_mgpcg_256.json")
    n = 256 ** 3
    for tag in ("fp64", "mixed"):
        r = d[tag]
        assert r["status"] == 0   # M2S_OK
        assert r["true_relres"] <= 1e-9
        h = np.asarray(r["hist"])
        assert len(h) == r["iters"] + 1 and h[0] == 1.0 and h[-1] <= 1e-9
        assert np.all(h[1:-1] > 1e-9)   # stopped at the first pass
        assert len(r["x_sample"]) == -(-n // d["sample_stride"])
    # the mixed run differs from the FP64 one only by the float V-cycle
    assert abs(d["fp64"]["iters"] - d["mixed"]["iters"]) <= 2


def test_c5_fixture_consistent():
    d = _load("oracle_c5_var7_128.json")
    n = 128 ** 3
    for tag in ("forward", "adjoint"):
        h = np.asarray(d[tag]["hist"])
        assert d[tag]["status"] == 0
        assert d[tag]["true_relres"] <= 1e-10
        assert len(h) == d[tag]["iters"] + 1 and h[-1] <= 1e-10
    for name in ("u_sample", "lam_sample"):
        assert len(d[name]) == -(-n // d["sample_stride"])
    for name, m in (("gkx_sample", 128 * 128 * 129),
                    ("gky_sample", 128 * 129 * 128),
                    ("gkz_sample", 129 * 128 * 128)):
        assert len(d[name]) == -(-m // d["sample_stride"])
    assert d["loss"] > 0
