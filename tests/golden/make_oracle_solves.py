"""Writes tests/golden/oracle_solves.json: the CPU oracle's certified optimum
of eq (1) (its branch and bound, Algorithm 1, run to a zero gap) on seeded
instances of each workload family at sizes the oracle closes in minutes. The
GPU tests regenerate the same instances from the seeds and compare the
device's certified optimum with these values.

Only the oracle and the seeded generators are used here:
    python tests/golden/make_oracle_solves.py [--only NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import datagen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "oracle_solves.json")

# name -> (generator arguments of datagen.gaussian_mixture, K)
CASES = {
    # the 10^9-sample workload's family (3 Gaussians, std 0.05, D = 2), seed 0
    "mixture_d2_k3_n1e6": (dict(n=1_000_000, d=2, k=3, std=0.05, seed=0), 3),
    # the 10^7-sample workload's family (5 Gaussians, std 0.1, D = 4, 1% outliers)
    "mixture_d4_k5_outliers_n2000": (dict(n=2000, d=4, k=5, std=0.1, seed=0, outlier_frac=0.01), 5),
    # the learned-branching evaluation family at its K (8 Gaussians, std 0.1, D = 5)
    "mixture_d5_k8_n300": (dict(n=300, d=5, k=8, std=0.1, seed=10000), 8),
}


def _cpu():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.machine()


def instance(name):
    kw, k = CASES[name]
    return datagen.gaussian_mixture(**kw), k


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    a = ap.parse_args()
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    res.setdefault("about", "Certified optima of the CPU oracle (float64 branch and bound, "
                   "Algorithm 1, zero gap) on seeded instances; written by "
                   "tests/golden/make_oracle_solves.py, which calls only the oracle and "
                   "the seeded generators.")
    res.setdefault("cases", {})
    for name, (kw, k) in CASES.items():
        if a.only and name != a.only:
            continue
        X, k = instance(name)
        t = time.time()
        r = oracle.solve(X.astype(np.float64), k)
        sec = time.time() - t
        assert r["status"] == 0 and r["lb"] == r["obj"], r
        res["cases"][name] = dict(generator=dict(kw, function="datagen.gaussian_mixture"), k=k,
                                  obj=r["obj"], lb=r["lb"], fft_obj=r["fft_obj"],
                                  centers=[int(c) for c in r["centers"]], nodes=int(r["nodes"]),
                                  oracle_seconds=round(sec, 2), threads=1,
                                  host=_cpu())
        print(name, res["cases"][name], flush=True)
        with open(OUT, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
