"""Sampling rounds on several lanes (concurrent streams), their scheduling
decisions against the scheduling oracle, the device level statistics against
Welford in sample order, and the error statuses of the whole-path calls."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2111_11788_amd as mm
from oracle import mlmc as omlmc, sched
from workloads import Workload


def _wl(**kw):
    base = dict(name="rounds", n0=4, levels=3, sigma2=1.0, corr_len=0.5, n_modes=8, qoi=0, rtol=1e-10,
                max_iter=3000, solver=0, precision=1, batch=8)
    base.update(kw)
    return Workload(**base)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    mm.lib()
    return torch.device("cuda")


def _oracle_stats(y):
    s = omlmc.RunningStats()
    for v in y:
        s.push(float(v))
    return s


def test_fold_matches_welford_and_does_not_depend_on_the_split(dev):
    y = np.random.default_rng(5).standard_normal(5000) * 2e-3 + 0.0137
    yt = torch.tensor(y, device=dev)
    ctx = mm.Context(_wl(), arena_bytes=64 << 20)
    got = []
    for cuts in ([5000], [1, 63, 64, 500, 4372], [4096, 904], [37] * 135 + [5]):
        ctx.reset_stats()
        o = 0
        for c in cuts:
            ctx.fold_stats(1, yt[o:o + c])
            o += c
        assert o == 5000
        got.append(ctx.get_estimate()["levels"][1])
    for g in got[1:]:
        assert g["mean"] == got[0]["mean"] and g["m2"] == got[0]["m2"] and g["n"] == 5000
    ref = _oracle_stats(y)
    assert abs(got[0]["mean"] - ref.mean) <= 1e-14 * abs(ref.mean)
    assert abs(got[0]["m2"] - ref.m2) <= 1e-12 * ref.m2
    assert got[0]["var"] == pytest.approx(np.mean((y - y.mean()) ** 2), rel=1e-12)   # 1/N variance


def test_fold_counts_nonfinite_apart(dev):
    y = np.random.default_rng(6).standard_normal(300)
    bad = y.copy()
    bad[[3, 64, 200]] = [np.nan, np.inf, -np.inf]
    ctx = mm.Context(_wl(), arena_bytes=64 << 20)
    rc = ctx.fold_stats(0, torch.tensor(bad, device=dev), allow_nonfinite=True)
    assert rc == -5
    lv = ctx.get_estimate()["levels"][0]
    ref = _oracle_stats(np.delete(y, [3, 64, 200]))
    assert lv["n"] == 297 and lv["nonfinite"] == 3
    assert abs(lv["mean"] - ref.mean) <= 1e-13 * abs(ref.mean) + 1e-16


def _fill(n):
    """Samples of an n^3 mesh that fill the device: 8192 waves of the fp32
    stencil launch geometry (a thread per 4 nodes of a row, workgroups of up to
    256 threads holding whole rows)."""
    g = n // 4
    if g < 1:
        return 8192
    rowthreads = (n - 1) * g
    threads = 256 if rowthreads >= 256 else -(-rowthreads // 64) * 64
    rows = max(1, threads // g)
    waves = -(-(n - 1) // rows) * (threads // 64)
    return -(-8192 // waves)


def test_fill_geometry_examples():
    # 64^3: 4 workgroups of 16 rows, 4 waves each -> 512 samples; 256^3: 64 x 4 -> 32
    assert _fill(64) == 512 and _fill(256) == 32 and _fill(8) == 8192


@pytest.mark.parametrize("lanes,pack", [(2, True), (4, True), (4, False)])
def test_lanes_give_the_same_bits_and_the_oracle_plan(dev, lanes, pack):
    # a round over three levels (plain MLMC with fixed N_l) on several lanes:
    # every sample's QoIs are the bits of the one-lane run, the estimator too,
    # and the tasks are the scheduling oracle's, part for part and lane for
    # lane, with and without packing two levels' solves on one mesh
    wl = _wl(levels=3, n0=8, n_modes=16, corr_len=0.3, batch=16)
    nfix = [5000, 70, 9]
    res = {}
    for k in (1, lanes):
        ctx = mm.Context(wl, arena_bytes=2 << 30)
        fuse = ctx.tuning()["fuse"]
        fuse = (fuse | mm.FUSE_PACK) if pack else (fuse & ~mm.FUSE_PACK)
        ctx.set_tuning(lanes=k, fuse=fuse)
        nl, est = ctx.estimate(0.0, n_fixed=nfix)
        assert [int(x) for x in nl] == nfix
        plan = ctx.last_plan()
        caps = [sched.level_cap(wl.n0, wl.levels, l, 16) for l in range(3)]
        fills = [_fill(wl.n(l)) for l in range(3)]
        want = sched.plan(wl.n0, [(l, 0, nfix[l]) for l in range(3)], k, caps, fills, pack=pack)
        if k > 1:
            assert len(set(t["lane"] for t in plan)) > 1
        if pack:
            assert any(len(t["parts"]) == 2 for t in want)
        assert [(t["level"], t["n"], t["first"], t["count"], t["lane"], t["task"]) for t in plan] == sched.flat(want)
        assert est["lanes"] == k and 0.0 < est["active_ratio"] <= 1.0 + 1e-9
        per = [ctx.sample_level(l, 1000, 40) for l in range(3)]
        res[k] = (est, per)
        ctx.close()
    e1, p1 = res[1]
    ek, pk = res[lanes]
    assert e1["qtilde"] == ek["qtilde"]
    for a, b in zip(e1["levels"], ek["levels"]):
        assert a["mean"] == b["mean"] and a["m2"] == b["m2"] and a["n"] == b["n"]
    for a, b in zip(p1, pk):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_packed_levels_match_the_oracle(dev):
    # the level samples of a packed round agree with the oracle's solves
    wl = _wl(levels=3, n0=4, rtol=1e-12, precision=0, batch=8)
    ctx = mm.Context(wl, arena_bytes=512 << 20)
    ctx.set_tuning(lanes=3)
    nl, est = ctx.estimate(0.0, n_fixed=[12, 6, 3])
    for l, cnt in enumerate((12, 6, 3)):
        yo, _, _, _ = omlmc.sample_level(wl, l, 0, cnt, rtol=1e-12, max_iter=20000)
        ref = _oracle_stats(yo)
        assert abs(est["levels"][l]["mean"] - ref.mean) <= 1e-8 * abs(ref.mean) + 1e-12


def test_estimate_reports_non_convergence(dev):
    # max_iter 2 cannot reach 1e-10: the estimate finishes, fills its outputs
    # and returns MLMC_E_NOCONV instead of success
    wl = _wl(max_iter=2, precision=0)
    ctx = mm.Context(wl, arena_bytes=256 << 20)
    with pytest.raises(mm.MLMCError) as e:
        ctx.estimate(1e-3, n_pilot=4, cost_model=1, max_rounds=1)
    assert e.value.code == -4
    nl, est = ctx.estimate(1e-3, n_pilot=4, cost_model=1, max_rounds=1, allow=(-4,))
    assert ctx.last_rc == -4 and all(int(x) >= 4 for x in nl)


@pytest.mark.parametrize("n,precision", [(8, 1), (16, 1), (16, 0)])
def test_nonfinite_coefficient_stops_the_solve(dev, n, precision):
    # a NaN in kappa: the sample's solve stops at once with MLMC_E_NONFINITE
    # (8^3 mixed: the whole-solve kernel; 16^3: the level-by-level path)
    wl = _wl(n0=n, levels=1, precision=precision, max_iter=500)
    ctx = mm.Context(wl, arena_bytes=512 << 20)
    kap = ctx.field(n, ctx.draw_xi(0, 0, 3))
    kap[1, 17] = float("nan")
    u = torch.zeros((3, mm.grid_stride(n)), dtype=torch.float64, device=dev)
    it = np.zeros(3, dtype=np.int32)
    rc = mm.lib().mlmc_solve(ctx.h, n, 3, mm._ptr(kap), mm._ptr(u), it.ctypes.data)
    assert rc == -5, rc
    assert it[1] < 100
    uc = u.cpu().numpy()
    assert np.all(np.isfinite(uc[0])) and np.all(np.isfinite(uc[2]))
