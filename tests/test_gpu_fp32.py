"""Element-by-element parity of the fp32 kernels of the mixed-precision path
(through mlmc_apply_f32 and mlmc_vcycle_f32) against the fp64 oracle, at the
sizes and launch geometry the batched 64^3 workload runs (512+ samples: one
plane chunk per sample, four row blocks of 16 rows), and an iteration bound on
the mixed solve (fp64 refinement would otherwise hide a defective fp32
preconditioner behind extra iterations).

Tolerances (fp32 unit roundoff u = 2^-24 ~ 6e-8):
  apply: each output sums 8 element contributions of 8 terms each in fp32;
         |y - y_exact| <= 64 u sum_terms |.|, tested as 64 u x (27 max|A| max|u|)
  V-cycle: an affine chain of about 3 + 4 degree stencil passes per level over
         log2(n) levels; tested at 2e-5 of max|z| (observed ~1e-6), far below
         the 1e-2 .. 1 differences a wrong coefficient, interval or index gives.
The oracle gets the fp32-rounded inputs, so only the arithmetic differs.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2111_11788_amd as mm
from oracle import fe, gmg, mlmc as omlmc
from workloads import Workload, element_field, grid_vector

CHEB_HI = 1.75
U32 = 2.0 ** -24


def _wl(**kw):
    base = dict(name="f32", n0=16, levels=1, sigma2=1.0, corr_len=0.3, n_modes=16, qoi=1, rtol=1e-8,
                max_iter=3000, solver=0, precision=1, batch=16)
    base.update(kw)
    return Workload(**base)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    mm.lib()
    return torch.device("cuda")


def _inputs(n, B, seed, check):
    kap = element_field(n, B, seed=seed, spread=1.5).astype(np.float32)
    u = grid_vector(n, B, seed=seed + 1).astype(np.float32)
    return kap, u


@pytest.mark.parametrize("zvar", [0, 2])
@pytest.mark.parametrize("n,B,check", [(16, 5, (0, 4)), (32, 3, (0, 2)), (64, 512, (0, 255, 511))])
def test_apply_f32_matches_csr(dev, n, B, check, zvar):
    kap, u = _inputs(n, B, 900 + n, check)
    ctx = mm.Context(_wl(n0=n), arena_bytes=64 << 20)
    ctx.set_tuning(zvar_fp32=zvar)
    ug = mm.to_grid(torch.tensor(u, device=dev), n)
    yg = ctx.apply_f32(n, torch.tensor(kap, device=dev), ug)
    mask = np.ones(yg.shape[1], dtype=bool)
    mask[mm.interior_positions(n)] = False
    assert np.all(yg.cpu().numpy()[:, mask] == 0.0)
    y = mm.from_grid(yg, n).cpu().numpy().astype(np.float64)
    worst = 0.0
    for b in check:
        A = fe.assemble(n, kap[b].astype(np.float64))
        want = A @ u[b].astype(np.float64)
        scale = np.abs(A).max() * 27 * np.abs(u[b]).max()
        err = np.abs(y[b] - want).max() / scale
        worst = max(worst, err)
        assert err <= 64 * U32, (b, err)
    print(f"apply f32 n={n} B={B} zvar={zvar}: max err / row scale {worst:.2e}")


_HIER = {}


def _vcycle_oracle(n, kap, r, deg):
    # the oracle's hierarchy of one sample, kept for the other degree (the
    # 128^3 assembly takes tens of seconds)
    key = (n, kap.tobytes())
    if key not in _HIER:
        _HIER.clear()
        _HIER[key] = gmg.Hierarchy(n, kap.astype(np.float64))
    return _HIER[key].vcycle(r.astype(np.float64), deg, 4.0, CHEB_HI)


# 64^3 x 512: the tiles of the 64^3 x 1024 step; 128^3: rows of 32 vectors
# (the extra residual row of a tile as one wave of two nodes per lane)
@pytest.mark.parametrize("n,B,check", [(16, 6, (0, 5)), (32, 4, (1, 3)), (64, 512, (0, 300, 511)), (128, 2, (1,))])
@pytest.mark.parametrize("deg", [1, 2])
def test_vcycle_f32_matches_oracle(dev, n, B, check, deg):
    # every fusion set the path uses (0 none, 63 the default set, 127 with the
    # fused residual update), both fp32 stencil engines (2 LDS planes, 6 also
    # for the corrected smoothing step) and the coarse single-kernel V-cycle
    # from 16^3 on and off
    kap, r = _inputs(n, B, 1300 + n + deg, check)
    want = {b: _vcycle_oracle(n, kap[b], r[b], deg) for b in check}
    kt = torch.tensor(kap, device=dev)
    rg = mm.to_grid(torch.tensor(r, device=dev), n)
    ctx = mm.Context(_wl(n0=n), cheb_degree=deg, arena_bytes=(8 << 30) if n == 64 else (1 << 30))
    worst = 0.0
    for fuse in (0, 63, 127):
        for zvar in (2, 6):
            for vsmall in (16, 0):
                ctx.set_tuning(fuse=fuse, zvar_fp32=zvar, vsmall_fp32=vsmall)
                z = mm.from_grid(ctx.vcycle_f32(n, kt, rg), n).cpu().numpy().astype(np.float64)
                for b in check:
                    err = np.abs(z[b] - want[b]).max() / np.abs(want[b]).max()
                    worst = max(worst, err)
                    assert err <= 2e-5, (fuse, zvar, vsmall, b, err)
    print(f"vcycle f32 n={n} B={B} deg={deg}: max rel err {worst:.2e}")


@pytest.mark.parametrize("n,B,deg", [(32, 8, 1), (32, 8, 2), (64, 512, 1)])
def test_mixed_solve_inner_iterations_are_bounded(dev, n, B, deg):
    # the fp32 inner solves of the mixed path need about as many iterations as
    # the fp64 GMG-PCG (refinement restarts add a few); a defective fp32
    # preconditioner would converge only through many more
    wl = _wl(n0=n, n_modes=64, batch=B)
    tune = dict(zvar_fp32=2, zvar_fp64=2, vsmall_fp32=16, vsmall_fp64=8, cheb_degree=deg, graph_batch=1, fuse=63)
    counts = {}
    for prec in (1, 0):
        ctx = mm.Context(wl, precision=prec, max_batch=B, arena_bytes=(24 << 30) if n == 64 else (1 << 30))
        ctx.set_tuning(**tune)
        y, qf, qc, it = ctx.sample_level(0, 0, B)
        counts[prec] = it
        ctx.close()
    print(f"n={n} B={B} deg={deg}: mixed inner iterations max {counts[1].max()} mean {counts[1].mean():.2f}, "
          f"fp64 max {counts[0].max()} mean {counts[0].mean():.2f}")
    assert counts[1].max() <= counts[0].max() + 4
    assert counts[1].max() <= 14


def test_vcycle_f32_256cube_fused_restriction_matches_unfused(dev):
    # 256^3 (rows of one wave of vectors, 4-row tiles whose extra residual
    # row takes a second pass): the fused residual restriction against the
    # separate residual and restriction kernels, Chebyshev degree 2 (no
    # on-the-fly pre-smoothing); the oracle's 256^3 hierarchy is too large
    # to assemble here
    n, B = 256, 2
    kap, r = _inputs(n, B, 4242, (0, 1))
    kt = torch.tensor(kap, device=dev)
    rg = mm.to_grid(torch.tensor(r, device=dev), n)
    ctx = mm.Context(_wl(n0=n), cheb_degree=2, arena_bytes=8 << 30)
    out = {}
    for fuse in (0, 8):
        ctx.set_tuning(fuse=fuse, zvar_fp32=2, vsmall_fp32=16)
        out[fuse] = mm.from_grid(ctx.vcycle_f32(n, kt, rg), n).cpu().numpy().astype(np.float64)
    for b in range(B):
        err = np.abs(out[8][b] - out[0][b]).max() / np.abs(out[0][b]).max()
        assert err <= 2e-5, (b, err)
