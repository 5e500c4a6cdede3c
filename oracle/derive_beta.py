"""Derive the regularization strength of each workload with the FP64 oracle.

The paper does not state beta.  The reading used: beta = BETA_REL x the
median over the ROI of the SQS denominator D_L = A'WA1 of the workload's own
data, with BETA_REL chosen once by a sweep on the 128^2 fan-beam workload
(minimum ROI RMSE of the converged image against the true phantom, on a seed
that is not used for evaluation).

Usage:
    python -m oracle.derive_beta --sweep            # choose BETA_REL
    python -m oracle.derive_beta fan2d_128 fan2d_512 ...   # D_L medians

The printed medians are pasted, rounded to 4 significant digits, into
``synth/configs.py`` (``DL_MEDIAN``).
"""
import argparse
import math
import sys
import time

import numpy as np

import synth
from . import oracle as ora


def dl_median(name):
    cfg = synth.get_config(name)
    data = synth.make_problem_data(cfg)
    DL = ora.sqs_denom(cfg, data["w"])
    return float(np.median(DL[synth.roi_mask(cfg)]))


def sweep(seed=1001, n_iter=300):
    cfg = synth.get_config("fan2d_128", seed=seed)
    data = synth.make_problem_data(cfg, with_truth=True)
    DL = ora.sqs_denom(cfg, data["w"])
    med = float(np.median(DL[synth.roi_mask(cfg)]))
    mask = synth.roi_mask(cfg)
    delta = synth.configs.delta_mu(cfg)
    best = None
    for e in range(-12, -3):
        beta = 2.0 ** e * med
        out = ora.os_lalm(cfg, data["y"], data["w"], beta, delta, M=1, n_steps=n_iter,
                          continuation=True, denom=DL)
        err = ora.rmsd_hu(out["x"], data["x_true"], mask, synth.HU_PER_MU)
        print("beta_rel = 2^%d  RMSE vs truth = %.3f HU" % (e, err), flush=True)
        if best is None or err < best[1]:
            best = (e, err)
    print("best beta_rel = 2^%d" % best[0])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--sweep", action="store_true")
    a = ap.parse_args(argv)
    if a.sweep:
        sweep()
    for n in a.names:
        t = time.time()
        m = dl_median(n)
        print("%s: median_ROI(D_L) = %.6g   (%.1f s)" % (n, m, time.time() - t), flush=True)


if __name__ == "__main__":
    main()
