"""Serving (continuous batching) through the C-ABI: results against the
oracle, alone-vs-mixed bit equality, admission by budget."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2111_11788_amd as mm
from oracle import mlmc as omlmc
from workloads import Workload


def _wl(**kw):
    base = dict(name="serve", n0=8, levels=3, sigma2=1.0, corr_len=0.3, n_modes=32, qoi=0, rtol=1e-10,
                max_iter=400, solver=0, precision=1, batch=8)
    base.update(kw)
    return Workload(**base)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    return torch.device("cuda")


@pytest.mark.parametrize("fuse,deg", [(None, 2), (None, 1), (0, 2)])
def test_served_samples_match_oracle(dev, fuse, deg):
    # fuse None: the default fusions (direction fused into the apply; with
    # Chebyshev degree 1 also the on-the-fly pre-smoothing and the residual
    # update fused into the next V-cycle); 0: none
    wl = _wl()
    ctx = mm.Context(wl, arena_bytes=1 << 30, cheb_degree=deg)
    if fuse is not None:
        ctx.set_tuning(fuse=fuse)
    ctx.serve_start([8, 8, 4])
    reqs = [(0, 3), (1, 4), (2, 5), (2, 6), (1, 7), (0, 8)]
    tickets = {ctx.submit(l, s): (l, s) for l, s in reqs}
    res = ctx.wait(tickets.keys())
    ctx.serve_stop()
    for t, (l, s) in tickets.items():
        r = res[t]
        assert r["status"] == 0 and r["level"] == l and r["sample"] == s
        y, qf, qc, _ = omlmc.sample_level(wl, l, s, 1, rtol=1e-12, max_iter=20000)
        assert abs(r["q_fine"] - qf[0]) <= 1e-7 * abs(qf[0])
        if l > 0:
            assert abs(r["q_coarse"] - qc[0]) <= 1e-7 * abs(qc[0])
        assert abs(r["y"] - (r["q_fine"] - r["q_coarse"])) == 0.0
        assert r["latency_s"] >= r["queue_s"] >= 0.0


@pytest.mark.parametrize("deg", [2, 1])
def test_alone_and_in_the_mix_are_identical(dev, deg):
    wl = _wl()
    ctx = mm.Context(wl, arena_bytes=1 << 30, cheb_degree=deg)
    ctx.serve_start([16, 16, 6])
    alone = ctx.wait([ctx.submit(2, 11)])
    (a,) = alone.values()
    # a burst of mixed levels that keeps every pool busy, with the same sample inside
    rng = np.random.default_rng(5)
    burst = [(int(l), int(s)) for l, s in zip(rng.integers(0, 3, 60), rng.integers(0, 1000, 60))]
    burst.insert(17, (2, 11))
    tickets = [ctx.submit(l, s) for l, s in burst]
    res = ctx.wait(tickets)
    ctx.serve_stop()
    b = res[tickets[17]]
    for k in ("y", "q_fine", "q_coarse", "iters"):
        assert a[k] == b[k], k
    assert all(r["status"] == 0 for r in res.values())


def test_budget_refusal_and_stop(dev):
    wl = _wl()
    ctx = mm.Context(wl, arena_bytes=1 << 30)
    ctx.serve_start([4, 4, 0])          # no slots for the 32^3 mesh
    with pytest.raises(mm.MLMCError) as e:
        ctx.submit(2, 0)
    assert e.value.code == -3
    t = ctx.submit(1, 0)                # 16^3 + 8^3 still served
    assert ctx.wait([t])[t]["status"] == 0
    # batch entry points are refused while serving
    with pytest.raises(mm.MLMCError):
        ctx.sample_level(0, 0, 1)
    ctx.serve_stop()
    y, _, _, _ = ctx.sample_level(0, 0, 2)   # and work again afterwards
    assert np.all(np.isfinite(y))


def test_submit_batch_and_drain_array_match_single_submits(dev):
    wl = _wl()
    ctx = mm.Context(wl, arena_bytes=1 << 30)
    ctx.serve_start([8, 8, 4])
    levels = np.array([0, 1, 2, 1, 0, 2, 0], dtype=np.int32)
    samples = np.array([40, 41, 42, 43, 44, 45, 46], dtype=np.uint64)
    tk = ctx.submit_batch(levels, samples)
    assert len(set(int(t) for t in tk)) == len(tk)
    got = []
    while sum(len(g) for g in got) < len(tk):
        got.append(ctx.drain_array(timeout=0.05))
    arr = np.concatenate(got)
    assert sorted(int(t) for t in arr["ticket"]) == sorted(int(t) for t in tk)
    # the same samples one at a time give the same bits
    single = ctx.wait([ctx.submit(int(l), int(s)) for l, s in zip(levels, samples)])
    ctx.serve_stop()
    by_sample = {(int(r["level"]), int(r["sample"])): r for r in single.values()}
    for r in arr:
        s = by_sample[(int(r["level"]), int(r["sample"]))]
        assert r["status"] == 0 and s["status"] == 0
        assert r["y"] == s["y"] and r["q_fine"] == s["q_fine"] and r["iters"] == s["iters"]


def test_idle_region_lends_and_takes_back(dev):
    # 2 slots per mesh: a burst of 8^3 samples keeps the 8^3 pool full while
    # the larger meshes idle, so an idle region takes a guest 8^3 pool of 2
    # slots; a 32^3 request (whose coarse solve is on 16^3) makes the lender
    # take its region back.  Every 8^3 result has the bits of the same sample
    # served alone, the 32^3 one matches the oracle.
    import time
    wl = _wl()
    ctx = mm.Context(wl, arena_bytes=1 << 30)
    ctx.serve_start([2, 2, 2])
    alone = {s: next(iter(ctx.wait([ctx.submit(0, s)]).values())) for s in (3, 29)}
    assert ctx.serve_stats()["lends"] == 0
    tickets = [ctx.submit(0, s) for s in range(40)]
    t0 = time.time()
    while ctx.serve_stats()["lends"] == 0 and time.time() - t0 < 10.0:
        time.sleep(0.002)
    st = ctx.serve_stats()
    assert st["lends"] >= 1
    assert st["slots"][0] == 4 and (st["slots"][1] == 0 or st["slots"][2] == 0)
    t2 = ctx.submit(2, 5)
    res = ctx.wait(tickets + [t2])
    st = ctx.serve_stats()
    ctx.serve_stop()
    assert st["reclaims"] >= 1 and st["completed"] == 43
    assert all(r["status"] == 0 for r in res.values())
    for s in (3, 29):
        r = res[tickets[s]]
        for k in ("y", "q_fine", "iters"):
            assert r[k] == alone[s][k], (s, k)
    r = res[t2]
    y, qf, qc, _ = omlmc.sample_level(wl, 2, 5, 1, rtol=1e-12, max_iter=20000)
    assert abs(r["q_fine"] - qf[0]) <= 1e-7 * abs(qf[0]) and abs(r["q_coarse"] - qc[0]) <= 1e-7 * abs(qc[0])
