"""Section 5.5 on the host: the FP64 oracle over the stability grid.

Writes stability_oracle_5000x5000.json beside this script: for each sparse
test matrix (standardized Bernoulli SB, sparse sign SS, sparse Gaussian SG,
Bernoulli B), p in {ln(n)/n, 2e-3, 1e-2} and d in {1, n/10, n} (V_A block
diagonal with d Haar blocks; Matrix 1's spectrum; the inputs of
paper_2506_03859_amd.synth with seed 11, as bench.py --stability uses), the
(status, blocks, true relative error ||A - U S V^T||_F / ||A||_F) of `trials`
oracle solves at tol 1e-4, P = 1, the default b and block cap, seeds 1..trials.

    python tests/golden/stability_oracle.py [--trials 10] [--n 5000]
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import FarpcaParams, farpca  # noqa: E402
from paper_2506_03859_amd import synth  # noqa: E402

SKETCHES = [("SB", "std_bernoulli"), ("SS", "sparse_sign"), ("SG", "sparse_gaussian"), ("B", "bernoulli")]


def grid(n):
    return [1, n // 10, n], [("ln(n)/n", math.log(n) / n), ("2e-3", 2e-3), ("1e-2", 1e-2)]


def cell(a, na, sk, pv, seed, tol=1e-4):
    r = farpca(a, FarpcaParams(tol=tol, power=1, sketch=sk, p=pv, seed=seed))
    err = float(np.linalg.norm(a - (r.U * r.S) @ r.V.T) / na)
    return [int(r.status), int(r.blocks), err]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trials", type=int, default=10)
    ap.add_argument("--n", type=int, default=5000)
    args = ap.parse_args()
    n = args.n
    ds, ps = grid(n)
    out = {"n": n, "tol": 1e-4, "power": 1, "trials": args.trials, "seed_matrix": 11, "cells": {}}
    path = os.path.join(HERE, f"stability_oracle_{n}x{n}.json")
    t0 = time.time()
    for d in ds:
        a = synth.spectral_blockdiag_v(n, synth.matrix1_sigma(n), d, seed=11)
        na = float(np.linalg.norm(a))
        for pname, pv in ps:
            for short, sk in SKETCHES:
                key = f"{short} p={pname} d={d}"
                rec = [cell(a, na, sk, pv, s) for s in range(1, args.trials + 1)]
                out["cells"][key] = rec
                stop = sum(1 for s, _, _ in rec if s == 0)
                q18 = sum(1 for s, _, e in rec if s == 0 and e <= 1e-4)
                print(f"{time.time() - t0:7.0f}s {key}: stopped {stop}/{args.trials}, true error <= tol "
                      f"{q18}/{args.trials}, blocks {np.mean([b for _, b, _ in rec]):.1f}", flush=True)
                with open(path, "w") as f:
                    json.dump(out, f)


if __name__ == "__main__":
    main()
