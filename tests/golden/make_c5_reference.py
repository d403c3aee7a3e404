"""Write tests/golden/c5_stress_qoi.json: oracle QoIs of two 256^3 samples.

Workload: the 256^3 stress configuration (sigma^2 = 2, correlation length
0.1, M = 512 KL modes, f = 1, u0 = 0, domain-average QoI), samples 0 and 1 of
level 0.  Each value is the oracle's fp64 result: Philox xi, KLE kappa at the
element centroids, assembled CSR operator, Jacobi-PCG to true relative
residual 1e-10.  Calls only oracle/ (and the workload definitions).
Takes about 10 minutes and 25 GB of memory per sample.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mlmc  # noqa: E402
from workloads import C5  # noqa: E402

RTOL = 1e-10


def main():
    out = {"workload": C5.name, "n": C5.n0, "sigma2": C5.sigma2, "corr_len": C5.corr_len,
           "n_modes": C5.n_modes, "seed": C5.seed, "qoi": "domain average", "rtol": RTOL, "samples": []}
    for s in (0, 1):
        t = time.time()
        Y, Qf, Qc, its = mlmc.sample_level(C5, 0, s, 1, rtol=RTOL, max_iter=100000)
        out["samples"].append({"level": 0, "index": s, "q": float(Qf[0]), "iterations": int(its[0]),
                               "seconds": round(time.time() - t, 1)})
        print(out["samples"][-1], flush=True)
    with open(os.path.join(HERE, "c5_stress_qoi.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
