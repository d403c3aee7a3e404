"""Degenerate and boundary cases of the HIP path through the C-ABI: constant
coefficient (sigma^2 = 0), the 2^3 mesh with its single unknown, empty
requests, refused arguments and non-convergence."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2111_11788_amd as mm
from oracle import mlmc as omlmc
from workloads import Workload


def _wl(**kw):
    base = dict(name="edge", n0=2, levels=3, sigma2=0.0, corr_len=0.5, n_modes=8, qoi=0, rtol=1e-12,
                max_iter=3000, solver=0, precision=0, batch=8)
    base.update(kw)
    return Workload(**base)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    mm.lib()
    return torch.device("cuda")


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_constant_coefficient_field_and_closed_form(dev, precision):
    # sigma^2 = 0: kappa = exp(0) = 1 exactly (fp64, fp32 copy and bf16 KLE);
    # on 2^3 elements the single unknown is u = 3 h^2 / sum kappa = 0.75 / 8
    # and the domain average h^3 u = 0.01171875 (closed form)
    wl = _wl(precision=precision)
    ctx = mm.Context(wl, arena_bytes=64 << 20)
    for n in (2, 4, 8):
        k, k32 = ctx.field(n, ctx.draw_xi(0, 0, 3), want32=True)
        assert np.all(k.cpu().numpy() == 1.0) and np.all(k32.cpu().numpy() == 1.0)
    y, qf, qc, it = ctx.sample_level(0, 0, 4)
    tol = 1e-15 if precision == 0 else 1e-7
    assert np.all(np.abs(qf - 0.01171875) <= tol * 0.01171875) and np.all(qc == 0.0)
    # every sample of a level sees the same problem: Y_l is one number per level
    y1, qf1, qc1, _ = ctx.sample_level(2, 0, 5)
    assert np.ptp(qf1) <= 1e-14 * abs(qf1[0]) + (0 if precision == 0 else 1e-7 * abs(qf1[0]))
    q8 = omlmc.solve_qoi(8, np.ones(8 ** 3), 0, 1e-12, 1000)[0]
    assert abs(qf1[0] - q8) <= (1e-8 if precision == 0 else 1e-7) * q8


def test_empty_request_changes_nothing(dev):
    ctx = mm.Context(_wl(sigma2=1.0), arena_bytes=64 << 20)
    ctx.sample_level(1, 0, 3)
    before = ctx.get_estimate()
    y, qf, qc, it = ctx.sample_level(1, 3, 0)
    assert len(y) == 0
    after = ctx.get_estimate()
    assert after == before


def test_refused_arguments(dev):
    ctx = mm.Context(_wl(sigma2=1.0, n0=4), arena_bytes=64 << 20)
    for bad in (lambda: ctx.sample_level(3, 0, 1),          # level out of range
                lambda: ctx.sample_level(-1, 0, 1),
                lambda: ctx.node_map(6),                     # not a power of two
                lambda: ctx.set_tuning(fuse=1 << 12),        # unknown fusion bit
                lambda: ctx.estimate(0.0),                   # eps must be > 0
                lambda: ctx.estimate_adaptive(1e-3, l0=0)):  # adaptive needs a difference level
        with pytest.raises(mm.MLMCError) as e:
            bad()
        assert e.value.code == -1
    # the context still works after the refusals
    y, qf, qc, it = ctx.sample_level(0, 0, 2)
    assert np.all(np.isfinite(qf))


@pytest.mark.parametrize("precision", [0, 1])
def test_non_convergence_is_reported(dev, precision):
    # a cap of 2 iterations cannot reach 1e-12: MLMC_E_NOCONV, finite last iterates
    wl = _wl(sigma2=1.0, n0=8, levels=1, max_iter=2, precision=precision)
    ctx = mm.Context(wl, arena_bytes=256 << 20)
    kap = ctx.field(8, ctx.draw_xi(0, 0, 3))
    u, it = ctx.solve(8, kap, allow_noconv=True)
    assert np.all(np.isfinite(u.cpu().numpy()))
    with pytest.raises(mm.MLMCError) as e:
        ctx.solve(8, kap)
    assert e.value.code == -4
