"""Write the FP64 oracle's full-size OS-LALM results that GPU parity tests
compare against (test infrastructure; calls only ``oracle/`` and ``synth/``).

The 3D workloads are too large for the oracle to run inside a test (one
subset step of the 512x512x64 axial scan takes about 40 s on 8 host cores),
so the oracle runs once here and its results are stored under
``tests/oracle_cache/<workload>.npz`` (not committed; rerun this script to
regenerate them).  Stored, from x0 = 0, M subsets, continuation (Sec. III):

* ``slices``: the sampled slice indices (8, evenly spaced, both end slices
  included);
* ``DL``: the SQS denominator A'WA1 (Sec. IV-A) at those slices;
* ``x_k<K>``: the image after K iterations (K M subset steps) at those
  slices, for every K requested;
* ``cost_k<K>``: Psi, its data term and R at that image (FP64, full volume);
* ``rho``, ``xi``, ``restart``: per-step rho used, restart indicator and
  restart decision of the run;
* ``beta``, ``delta``, ``M``.

The file is rewritten after every requested K, so shorter results are
usable while a long run continues.

Usage:
    OMP_NUM_THREADS=8 python tests/make_oracle_cache.py cone_axial_512x64 --iters 1 20
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle as ora  # noqa: E402
import synth  # noqa: E402

CACHE = os.path.join(ROOT, "tests", "oracle_cache")


def sample_slices(nz, n=8):
    """n evenly spaced slice indices including the first and the last."""
    return np.unique(np.round(np.linspace(0, nz - 1, min(n, nz))).astype(np.int64))


def cache_path(workload):
    return os.path.join(CACHE, workload + ".npz")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("workload")
    ap.add_argument("--iters", type=int, nargs="+", default=[1])
    args = ap.parse_args()
    os.makedirs(CACHE, exist_ok=True)
    cfg = synth.get_config(args.workload)
    M = cfg["M"]
    beta, delta = cfg["beta"], synth.configs.delta_mu(cfg)
    shape = ora.image_shape(cfg)
    sl = sample_slices(shape[0])
    t0 = time.time()

    def note(msg):
        print("[%7.1f s] %s: %s" % (time.time() - t0, args.workload, msg), flush=True)

    data = synth.make_problem_data(cfg)
    note("synthetic data")
    DL = ora.sqs_denom(cfg, data["w"])
    note("SQS denominator")
    out = dict(slices=sl, DL=DL[sl].astype(np.float64), beta=beta, delta=delta, M=M,
               workload=args.workload)
    ks = sorted(set(args.iters))
    hist = {}

    def save():
        n = len(hist.get("rho", []))
        rec = dict(out, rho=np.array(hist["rho"][:n]), xi=np.array(hist["xi"][:n]),
                   restart=np.array(hist["restart"][:n], dtype=np.uint8))
        tmp = cache_path(args.workload) + ".tmp.npz"
        np.savez_compressed(tmp, **rec)
        os.replace(tmp, cache_path(args.workload))

    def on_step(j, x):
        note("step %d" % j)
        k, rem = divmod(j + 1, M)
        if rem == 0 and k in ks:
            out["x_k%d" % k] = x[sl].copy()
            out["cost_k%d" % k] = np.array(ora.cost(cfg, x, data["y"], data["w"], beta, delta))
            save()
            note("saved K = %d" % k)

    ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=M, n_steps=ks[-1] * M, denom=DL,
                callback=on_step, history=hist)
    note("done")


if __name__ == "__main__":
    main()
