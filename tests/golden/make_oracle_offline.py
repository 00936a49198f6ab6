"""Writes tests/golden/<workload>_oracle.npz: the oracle's offline stage (TT
greedy-cross, rounding, gauge) for a workload of synth.WORKLOADS, so the
full-size GPU parity tests need not rerun the free-running CPU cross.  The
cross does not depend on the points; the stored cores, ranks, index sets,
decision log and per-sweep errors are the oracle's alone (this script calls
only oracle/ and synth/).

usage: python tests/golden/make_oracle_offline.py matern32_d3   (about 30 s of CPU)
       python tests/golden/make_oracle_offline.py matern_batched (tens of minutes)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import driver, kernels  # noqa: E402


def main(name):
    w = synth.WORKLOADS[name]
    P = kernels.Problem(w.kind, w.d, w.box_s, w.box_t, w.box_theta, w.n_spatial, w.n_param, w.const or None)
    x0 = np.asarray(w.box_s, float)[:, :1].T
    y0 = np.asarray(w.box_t, float)[:, :1].T
    out = driver.offline(P, x0, y0, w.tol, seed=0, max_sweeps=w.extra.get("max_sweeps", 200))
    info = out["info"]
    arrays = {"ranks": np.array(out["ranks"]), "cross_ranks": np.array(info["ranks"]),
              "sweeps": np.array(info["sweeps"]), "error": np.array(info["error"])}
    for k, g in enumerate(out["cores"]):
        arrays[f"core{k}"] = g
    for k in range(1, P.D):
        arrays[f"left{k}"] = np.asarray(info["L"][k], dtype=np.int32)
        arrays[f"right{k}"] = np.asarray(info["R"][k], dtype=np.int32)
    margins = [min(r.get("sample_margin", np.inf), r.get("search_margin", np.inf)) for r in info["log"]]
    arrays["min_margin"] = np.array(min(margins) if margins else np.inf)
    # the decision log: pivot (row, col) of each step, whether it was added,
    # and the step's smaller top-2 margin (a tie within rounding when tiny)
    arrays["log_pivot"] = np.array([[r["pivot_row"], r["pivot_col"], int(r["added"])] for r in info["log"]],
                                   dtype=np.int64).reshape(-1, 3)
    arrays["log_margin"] = np.array(margins, dtype=np.float64)
    arrays["errors"] = np.array(info["errors"], dtype=np.float64)
    arrays["converged"] = np.array(bool(info["converged"]))
    path = os.path.join(HERE, f"{name}_oracle.npz")
    np.savez_compressed(path, **arrays)
    print(path, out["ranks"], info["ranks"], info["sweeps"])


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "matern32_d3")
