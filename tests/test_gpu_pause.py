"""Pause-model scheduler stress through the C-ABI against the oracle: the
drawn durations bit for bit, the schedule (steps, finishing step of every
sample, ideal active ratio) exactly, and the device-measured waiting time at
least the scheduled one (Sec. 5.1 benchmark; eq. active_ratio)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2111_11788_amd as mm
from oracle import pause
from workloads import Workload


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    wl = Workload(name="pause", n0=4, levels=3, sigma2=1.0, corr_len=0.5, n_modes=8, qoi=0, rtol=1e-8,
                  max_iter=100, solver=0, precision=1, batch=8)
    return mm.Context(wl, arena_bytes=64 << 20)


CASES = [
    # counts, widths, mu_us, sigma_us, capacity, batch, min_step_us
    ([40, 10, 3], [1, 8, 64], 50.0, 50.0 / 2 / np.sqrt(3), 128, 1, 0.0),
    ([40, 10, 3], [1, 8, 64], 50.0, 10.0, 128, 4, 0.0),
    ([64, 0, 5], [2, 4, 16], 20.0, 0.2, 32, 1, 15.0),
    ([7], [1], 5.0, 0.0, 1, 1, 0.0),
    ([0, 0], [1, 1], 5.0, 1.0, 4, 1, 0.0),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_pause_model_matches_oracle(ctx, case):
    counts, widths, mu, sigma, cap, batch, min_step = CASES[case]
    out, ticks, done = ctx.pause_model(counts, widths, mu, sigma, cap, batch, min_step)
    f = out["clock_mhz"]
    assert f > 0
    want_ticks = np.concatenate([pause.to_ticks(pause.durations_us(ctx.cfg.seed, lv, c, mu, sigma), f)
                                 for lv, c in enumerate(counts)]) if sum(counts) else np.zeros(0, np.int64)
    assert np.array_equal(ticks, want_ticks)
    s = pause.schedule(counts, widths, want_ticks, cap, batch, int(np.floor(min_step * f + 0.5)))
    assert out["steps"] == s["steps"] and out["tasks"] == s["tasks"]
    assert np.array_equal(done, s["done_step"])
    assert out["ideal_ratio"] == pytest.approx(s["ideal_ratio"], rel=1e-12, abs=0)
    assert out["active_slot_s"] == pytest.approx(s["active"] / f * 1e-6, rel=1e-12, abs=0)
    if s["steps"]:
        # every workgroup waits at least its share of a step; the wall time covers
        # the steps, so the measured ratio cannot beat the ideal one
        assert out["measured_slot_s"] >= out["active_slot_s"] * (1 - 1e-12)
        assert out["wall_s"] >= sum(s["step_lengths"]) / f * 1e-6 * (1 - 1e-9)
        assert 0 < out["ratio"] <= out["ideal_ratio"] * (1 + 1e-9)
    else:
        assert out["ratio"] == 0.0 and out["wall_s"] == 0.0


def test_pause_model_refuses_bad_options(ctx):
    for kw in (dict(counts=[4], widths=[9], capacity=8),        # wider than the device
               dict(counts=[4], widths=[1], sigma_us=10.0),     # mu - sqrt(3) sigma < 0
               dict(counts=[4], widths=[1], capacity=0),
               dict(counts=[4], widths=[1], batch=0),
               dict(counts=[-1], widths=[1])):
        args = dict(counts=[4], widths=[1], mu_us=10.0, sigma_us=1.0, capacity=8, batch=1, min_step_us=0.0)
        args.update(kw)
        with pytest.raises(mm.MLMCError) as e:
            ctx.pause_model(**args)
        assert e.value.code == -1
