"""Random forcing (a random f in eq. model, Sec. 2.1) through the C-ABI
against the oracle: the forcing field and its load vector, and whole
level samples in fp64 and mixed precision."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2111_11788_amd as mm
from oracle import fe, field, rng
from oracle import mlmc as omlmc
from workloads import Workload


def _wl(**kw):
    base = dict(name="forcing", n0=4, levels=2, sigma2=1.0, corr_len=0.5, n_modes=8, qoi=0, rtol=1e-12,
                max_iter=3000, solver=0, precision=0, batch=8, forcing=1)
    base.update(kw)
    return Workload(**base)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    mm.lib()
    return torch.device("cuda")


@pytest.mark.parametrize("n,level,first,count", [(4, 0, 0, 5), (8, 1, 3, 9), (16, 1, 7, 3)])
def test_forcing_field_and_load_match_oracle(dev, n, level, first, count):
    wl = _wl(n0=4, levels=3, n_modes=16, corr_len=0.3)
    ctx = mm.Context(wl, arena_bytes=64 << 20)
    f, b = ctx.forcing(n, level, first, count)
    xif = rng.draw_xi(wl.seed, level, first, count, wl.n_modes, stream=2)
    want_f = field.kappa(n, wl.corr_len, wl.sigma2, wl.n_modes, xif)
    got_f = f.cpu().numpy()
    assert np.max(np.abs(got_f - want_f) / want_f) < 1e-13
    got_b = mm.from_grid(b, n).cpu().numpy()
    for s in range(count):
        want_b = fe.load_elements(n, want_f[s])
        assert np.max(np.abs(got_b[s] - want_b) / np.abs(want_b)) < 1e-13
    # every position that is not an interior node is 0
    mask = np.ones(b.shape[1], dtype=bool)
    mask[mm.interior_positions(n)] = False
    assert np.all(b.cpu().numpy()[:, mask] == 0.0)


@pytest.mark.parametrize("precision,tol,fuse", [(0, 1e-8, None), (1, 1e-7, None), (1, 1e-7, 63)])
def test_forced_samples_match_oracle(dev, precision, tol, fuse):
    # mixed precision on 4^3 and 8^3: by default the whole solve runs in one
    # workgroup per sample (fuse bit 128), with fuse 63 the level-by-level path
    wl = _wl(precision=precision, rtol=1e-12 if precision == 0 else 1e-10)
    ctx = mm.Context(wl, arena_bytes=256 << 20)
    if fuse is not None:
        ctx.set_tuning(fuse=fuse)
    q0 = None
    for level, count in ((0, 6), (1, 5)):
        y, qf, qc, it = ctx.sample_level(level, 1, count)
        yo, qfo, qco, _ = omlmc.sample_level(wl, level, 1, count, rtol=1e-12, max_iter=20000)
        assert np.all(np.abs(qf - qfo) <= tol * np.abs(qfo))
        if level:
            assert np.all(np.abs(qc - qco) <= tol * np.abs(qco))
        else:
            q0 = qf
    # the forcing changes the answer: not the f = 1 one of the same samples
    q1 = mm.Context(_wl(precision=precision, forcing=0), arena_bytes=256 << 20).sample_level(0, 1, 6)[1]
    assert np.all(np.abs(q0 - q1) > 1e-3 * np.abs(q1))


def test_forcing_refusals(dev):
    with pytest.raises(mm.MLMCError):
        mm.Context(_wl(forcing=2), arena_bytes=64 << 20)
    ctx = mm.Context(_wl(), arena_bytes=256 << 20)
    with pytest.raises(mm.MLMCError) as e:
        ctx.serve_start()
    assert e.value.code == -1
    with pytest.raises(mm.MLMCError):
        ctx.forcing(6, 0, 0, 1)       # not a level mesh
