"""The allocation-free QoI entry point (partial sums in the library's static
device scratch) against mlmc_qoi, through the C-ABI."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2111_11788_amd as mm
from workloads import Workload, grid_vector


def _wl(qoi, n0):
    return Workload("noalloc", n0=n0, levels=2, sigma2=1.0, corr_len=0.3, n_modes=8, qoi=qoi, rtol=1e-8,
                    solver=0, precision=1, batch=8)


@pytest.mark.parametrize("qoi", [0, 1])
def test_noalloc_qoi_matches_qoi_on_two_calls(qoi):
    assert torch.cuda.is_available()
    ctx = mm.Context(_wl(qoi, 16), arena_bytes=1 << 30)
    # two calls in a row, the second on a smaller input (other mesh, fewer
    # samples): the scratch keeps the first call's partial sums, which the
    # second must not see
    for n, B, seed in ((32, 300, 3), (16, 5, 4)):
        u = mm.to_grid(torch.tensor(grid_vector(n, B, seed=seed), device="cuda"), n)
        want = ctx.qoi(n, u).cpu().numpy()
        got = ctx.qoi_noalloc(n, u).cpu().numpy()
        assert np.array_equal(got, want), (n, B, np.abs(got - want).max())
        # the QoI is linear in u: also check one value against its definition
        # from the binding's layout (interior positions) on the host
        if qoi == 0:
            uh = mm.from_grid(u, n).cpu().numpy()
            assert abs(got[1] - uh[1].sum() / n ** 3) <= 1e-13 * np.abs(uh[1]).sum() / n ** 3
    ctx.close()


def test_noalloc_qoi_refuses_counts_beyond_the_scratch():
    assert torch.cuda.is_available()
    ctx = mm.Context(_wl(0, 8), arena_bytes=1 << 28)
    u = torch.zeros((4, mm.grid_stride(8)), dtype=torch.float64, device="cuda")
    q = torch.empty(1 << 22, dtype=torch.float64, device="cuda")
    # 8^3: one partial sum per sample, 2^21 fit in 16 MiB; ask for 2^21 + 1 (no
    # kernel runs, so the short u is never read)
    rc = mm.lib().mlmc_qoi_noalloc(ctx.h, 8, (1 << 21) + 1, u.data_ptr(), q.data_ptr())
    assert rc == -1
    assert b"static scratch" in mm.lib().mlmc_last_error(ctx.h)
    # the context still works
    got = ctx.qoi_noalloc(8, u, q[:4])
    assert np.all(got.cpu().numpy() == 0.0)
    ctx.close()
