"""CPU-side checks of the C-ABI library: it loads, exports every declared
symbol, and its host-only entry points behave (no device calls)."""
import ctypes
import os
import re

import pytest

import paper_2111_11788_amd as mm
from workloads import C1, C2, C3, C5

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mlmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlmc_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = mm.lib()
    decl = _declared()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(decl) == sorted(mm.SYMBOLS)


def test_grid_stride_holds_every_neighbourhood():
    for n in (2, 4, 8, 16, 64, 256):
        s = mm.grid_stride(n)
        assert s % 64 == 0
        # largest neighbour position of an interior node: (n, n, n)
        assert s > n + n * n + n ** 3


def test_workspace_bytes_scale_with_batch():
    cfg = mm.make_config(C2)
    a = mm.workspace_bytes(cfg, 0, 1)
    b = mm.workspace_bytes(cfg, 0, 1024)
    assert 0 < a < b
    # the 64^3 x 1024 mixed-precision batch fits comfortably in 288 GB of HBM
    assert b < 40 * 2**30
    assert mm.workspace_bytes(mm.make_config(C5), 0, 16) < 60 * 2**30


@pytest.mark.parametrize("field,value", [("n0", 3), ("levels", 0), ("corr_len", 0.0), ("n_modes", 0),
                                         ("qoi", 7), ("precision", 5), ("max_batch", 0), ("rtol", -1.0)])
def test_invalid_configs_rejected_on_host(field, value):
    cfg = mm.make_config(C1, **{field: value})
    h = ctypes.c_void_p()
    rc = mm.lib().mlmc_create(ctypes.byref(cfg), ctypes.byref(h))
    assert rc == -1 and not h.value
    assert mm.lib().mlmc_last_error(None)


def test_workspace_rejects_bad_level():
    cfg = mm.make_config(C3)
    assert mm.workspace_bytes(cfg, 5, 4) == 0
    assert mm.workspace_bytes(cfg, 4, 4) > 0


def test_interior_positions_layout():
    n = 8
    pos = mm.interior_positions(n)
    assert len(pos) == (n - 1) ** 3 and len(set(pos.tolist())) == len(pos)
    i, j, k = pos % n, (pos // n) % n, pos // (n * n)
    assert i.min() == 1 and j.min() == 1 and k.min() == 1 and max(i.max(), j.max(), k.max()) == n - 1


def test_workspace_of_the_2cube_mesh_in_mixed_precision():
    # host geometry of the fp32 kernels on meshes narrower than one 16-byte
    # vector per row (2^3: one unknown); it once divided by zero on the host
    for prec in (0, 1, 2):
        cfg = mm.make_config(C1, n0=2, levels=3, precision=prec, solver=0)
        for level in range(3):
            for batch in (1, 7, 4096):
                assert mm.workspace_bytes(cfg, level, batch) > 0


def test_binding_fuse_bits_match_the_header():
    text = open(os.path.join(ROOT, "include", "mlmc.h")).read()
    bits = dict((k, int(v)) for k, v in re.findall(r"\bMLMC_FUSE_([A-Z]+)\s*=\s*(\d+)", text))
    assert len(bits) == 9
    for k, v in bits.items():
        assert getattr(mm, "FUSE_" + k) == v, k
