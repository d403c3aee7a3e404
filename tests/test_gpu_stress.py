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


def test_256cube_samples_match_stored_oracle_values():
    gold = json.load(open(os.path.join(HERE, "golden", "c5_stress_qoi.json")))
    wl = workloads.C5
    assert gold["n"] == wl.n0 and gold["n_modes"] == wl.n_modes and gold["seed"] == wl.seed
    ctx = mm.Context(wl, max_batch=2, rtol=gold["rtol"], max_iter=2000)
    y, qf, qc, it = ctx.sample_level(0, 0, 2)
    for g in gold["samples"]:
        q = float(qf[g["index"]])
        rel = abs(q - g["q"]) / abs(g["q"])
        print(f"256^3 sample {g['index']}: gpu {q!r} oracle {g['q']!r} rel {rel:.2e} iters {int(it[g['index']])}")
        assert rel <= 1e-7
    assert np.all(qc == 0.0) and np.array_equal(y, qf)
    ctx.close()
