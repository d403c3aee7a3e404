"""The 256^3 stress workload against stored oracle values.

tests/golden/c5_stress_qoi.json holds the oracle's QoIs of samples 0 and 1
(level 0) of the 256^3 workload (sigma^2 = 2, correlation length 0.1, 512 KL
modes), computed by tests/golden/make_c5_reference.py with the assembled
operator and Jacobi-PCG to true relative residual 1e-10.  The GPU solves the
same samples (same Philox draw, KLE, mesh) with the mixed-precision GMG-PCG to
the same residual.
"""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2111_11788_amd as mm
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


# the tuning the bench's 256^3 leg pins (16 samples per call as four
# concurrent batches of 4, the prolongation fusion off)
C5_PINNED = {"zvar_fp32": 2, "zvar_fp64": 2, "vsmall_fp32": 16, "vsmall_fp64": 8, "cheb_degree": 1, "max_batch": 4,
             "graph_batch": 2, "fuse": 510, "field": 0, "lanes": 4}


@pytest.mark.parametrize("tuning,count", [(None, 2), (C5_PINNED, 16)], ids=["defaults", "bench-pinned"])
def test_256cube_samples_match_stored_oracle_values(tuning, count):
    gold = json.load(open(os.path.join(HERE, "golden", "c5_stress_qoi.json")))
    wl = workloads.C5
    assert gold["n"] == wl.n0 and gold["n_modes"] == wl.n_modes and gold["seed"] == wl.seed
    ctx = mm.Context(wl, max_batch=count, rtol=gold["rtol"], max_iter=2000)
    if tuning:
        ctx.set_tuning(**tuning)
    y, qf, qc, it = ctx.sample_level(0, 0, count)
    for g in gold["samples"]:
        q = float(qf[g["index"]])
        rel = abs(q - g["q"]) / abs(g["q"])
        print(f"256^3 sample {g['index']}: gpu {q!r} oracle {g['q']!r} rel {rel:.2e} iters {int(it[g['index']])}")
        assert rel <= 1e-7
    assert np.all(qc == 0.0) and np.array_equal(y, qf)
    ctx.close()
