"""Write tests/golden/c2_batched_qoi.json: oracle QoIs of four 64^3 samples.

Workload: the batched 64^3 configuration (sigma^2 = 1, correlation length
0.3, M = 64 KL modes, f = 1, u0 = 0, QoI = mean of u over [1/4, 3/4]^3),
samples 0, 1, 511 and 1023 of level 0, i.e. spread over one 1024-sample
batch.  Each value is the oracle's fp64 result: Philox xi, KLE kappa at the
element centroids, assembled CSR operator, Jacobi-PCG to true relative
residual 1e-12.  Calls only oracle/ (and the workload definitions).
Takes about a minute per sample.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mlmc  # noqa: E402
from workloads import C2  # noqa: E402

RTOL = 1e-12
INDICES = (0, 1, 511, 1023)


def main():
    out = {"workload": C2.name, "n": C2.n0, "sigma2": C2.sigma2, "corr_len": C2.corr_len,
           "n_modes": C2.n_modes, "seed": C2.seed, "qoi": "subcube [1/4,3/4]^3 average", "rtol": RTOL,
           "samples": []}
    for s in INDICES:
        t = time.time()
        Y, Qf, Qc, its = mlmc.sample_level(C2, 0, s, 1, rtol=RTOL, max_iter=100000)
        out["samples"].append({"level": 0, "index": s, "q": float(Qf[0]), "iterations": int(its[0]),
                               "seconds": round(time.time() - t, 1)})
        print(out["samples"][-1], flush=True)
    with open(os.path.join(HERE, "c2_batched_qoi.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
