"""Write the oracle fixtures of the full-size solve configurations.

    python tests/golden/make_oracle_fixtures.py [c3] [c5]

Runs ONLY the CPU oracle (oracle/, single-threaded) on the seeded inputs of
paper_2204_13304_amd.inputs and stores what the GPU tests compare against:

  oracle_c3_mgpcg_256.json  HPCG-shaped 27-point operator at 256^3, b = A*1 +
                            N(0, 1e-3) (seed 3), x0 = 0, 4-level MG-PCG to
                            relative residual 1e-9: the FP64 run and the mixed
                            run (V-cycle in float, r replaced by the true
                            residual every 50 iterations).
  oracle_c5_var7_128.json   VAR7 diffusion at 128^3 (seed 5), 4-level MG-PCG
                            to 1e-10 for A u = f, the adjoint solve
                            A lam = u - u_t to 1e-10, and the face gradient
                            dL/dk of L = 0.5 |u - u_t|^2.

Each file holds the iteration counts, the residual histories, the final
true residuals, fixed strided samples of the solution vectors (flat C-order
indices 0, s, 2s, ...), and the SHA-256 of the oracle's C sources, so that a
change of the oracle's arithmetic is visible against the stored values.
The whole run takes about 15 minutes on one core.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2204_13304_amd import inputs  # noqa: E402

# the oracle's solver core (the microbenchmark routines live in
# oracle/m2s_oracle_micro.h and do not take part in these runs)
ORACLE_SOURCES = ("oracle/m2s_oracle.c", "oracle/m2s_oracle_impl.h")
C3_FILE = os.path.join(HERE, "oracle_c3_mgpcg_256.json")
C5_FILE = os.path.join(HERE, "oracle_c5_var7_128.json")


def oracle_sha256():
    h = hashlib.sha256()
    for src in ORACLE_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def sample(a, stride):
    """Flat C-order entries 0, stride, 2 stride, ... of a."""
    return [float(v) for v in np.ascontiguousarray(a).ravel()[::stride]]


def run_c3():
    n = 256
    shape = (n, n, n)
    b = oracle.spmv27(np.ones(shape)) + inputs.rhs_perturbation(3, shape)
    out = {"config": "const27 256^3, 4-level MG-PCG, b = A*1 + N(0,1e-3) "
                     "seed 3, x0 = 0, tol 1e-9",
           "sample_stride": 16411}
    for tag, pc, rep in (("fp64", "mg", 0), ("mixed", "mg_f32", 50)):
        t = time.perf_counter()
        r = oracle.pcg(b, precond=pc, levels=4, max_iter=1000, tol=1e-9,
                       replace_every=rep)
        dt = time.perf_counter() - t
        print(f"c3 {tag}: {r['iters']} iterations, true relres "
              f"{r['true_relres']:.3e}, {dt:.0f} s", flush=True)
        out[tag] = {"status": r["status"], "iters": r["iters"],
                    "replace_every": rep, "true_relres": r["true_relres"],
                    "hist": [float(v) for v in r["hist"]],
                    "x_sample": sample(r["x"], out["sample_stride"]),
                    "oracle_seconds": dt}
    return out


def run_c5():
    n = 128
    shape = (n, n, n)
    pr = inputs.var7_problem(5, shape)
    faces = (pr["kx"], pr["ky"], pr["kz"])
    stride = 2053
    t = time.perf_counter()
    fw = oracle.pcg(pr["f"], kind="var7", faces=faces, precond="mg",
                    levels=4, max_iter=1000, tol=1e-10)
    adj = oracle.pcg(fw["x"] - pr["u_t"], kind="var7", faces=faces,
                     precond="mg", levels=4, max_iter=1000, tol=1e-10)
    gx, gy, gz = oracle.var7_face_grad(fw["x"], adj["x"])
    dt = time.perf_counter() - t
    loss = 0.5 * float(np.sum((fw["x"] - pr["u_t"]) ** 2))
    print(f"c5: forward {fw['iters']} iterations, adjoint {adj['iters']}, "
          f"loss {loss:.6e}, {dt:.0f} s", flush=True)
    solve = lambda r: {"status": r["status"], "iters": r["iters"],  # noqa
                       "true_relres": r["true_relres"],
                       "hist": [float(v) for v in r["hist"]]}
    return {"config": "var7 128^3 seed 5 (faces exp(N(0,0.5^2)), f, u_t ~ "
                      "N(0,1)), 4-level MG-PCG to 1e-10, adjoint solve to "
                      "1e-10, loss 0.5 |u - u_t|^2",
            "sample_stride": stride, "loss": loss,
            "forward": solve(fw), "adjoint": solve(adj),
            "u_sample": sample(fw["x"], stride),
            "lam_sample": sample(adj["x"], stride),
            "gkx_sample": sample(gx, stride),
            "gky_sample": sample(gy, stride),
            "gkz_sample": sample(gz, stride),
            "oracle_seconds": dt}


def main(argv):
    which = argv or ["c3", "c5"]
    for tag, fn, path in (("c3", run_c3, C3_FILE), ("c5", run_c5, C5_FILE)):
        if tag not in which:
            continue
        d = fn()
        d["oracle_sources"] = list(ORACLE_SOURCES)
        d["oracle_sources_sha256"] = oracle_sha256()
        d["written_by"] = "tests/golden/make_oracle_fixtures.py (oracle only)"
        with open(path, "w") as fh:
            json.dump(d, fh, indent=0)
            fh.write("\n")
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
