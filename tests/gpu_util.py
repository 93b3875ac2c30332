"""Helpers for the GPU parity tests (tensor <-> numpy, error norms)."""
import numpy as np
import torch

DEV = "cuda:0"


def dev(a, dtype=None):
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV).contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_inf(a, ref):
    a, ref = np.asarray(a, np.float64), np.asarray(ref, np.float64)
    den = np.max(np.abs(ref))
    return np.max(np.abs(a - ref)) / (den if den > 0 else 1.0)


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def oracle_fixture(name):
    """A stored oracle result (tests/golden/, written by
    tests/golden/make_oracle_fixtures.py from the CPU oracle only)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    with open(path) as fh:
        return json.load(fh)


def strided(a, stride):
    """Flat C-order entries 0, stride, 2 stride, ... (the fixtures'
    samples)."""
    return np.ascontiguousarray(a).ravel()[::stride]


def rel_sample(a, ref):
    """max |a - ref| / max |ref| over a sample."""
    a, ref = np.asarray(a, np.float64), np.asarray(ref, np.float64)
    return float(np.max(np.abs(a - ref)) / np.max(np.abs(ref)))
