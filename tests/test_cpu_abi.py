"""Host-side checks of the C ABI: the library loads on a machine without a GPU,
exports every declared entry point, validates arguments, and its parameter
layout matches the oracle's independently built layout."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "squint.h")
LIB = os.path.join(ROOT, "paper_2602_21203_amd", "libsquint.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsquint.so not built")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^SQ_API\s+(?:const\s+)?\w+\*?\s+(\w+)\(", text, re.M)))


def test_exports_every_declared_symbol():
    names = declared()
    assert len(names) >= 25
    lib = ctypes.CDLL(LIB)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_layout_matches_oracle():
    from oracle import layout
    from paper_2602_21203_amd import _lib, configs
    for name, cfg in configs.CONFIGS.items():
        t, blocks = _lib.param_table(cfg)
        d = layout.dims(**cfg)
        ot, total = layout.offsets(d)
        assert [(n, o, tuple(s)) for n, o, s in t] == [(n, o, tuple(s)) for n, (o, s) in ot.items()]
        assert blocks == layout.blocks(d)
    assert _lib.param_count(configs.FULL) == 1493335
    assert _lib.param_count(configs.TINY) == 90563


def test_invalid_dims_are_rejected_without_work():
    from paper_2602_21203_amd import _lib, configs
    bad = dict(configs.FULL, k=3)            # 64 is not a multiple of 3
    with pytest.raises(_lib.SquintError, match="frame dims"):
        _lib.param_count(bad)
    with pytest.raises(_lib.SquintError):
        _lib.param_count(dict(configs.FULL, atoms=0))
    with pytest.raises(_lib.SquintError, match="v_max"):
        _lib.param_count(dict(configs.FULL, v_min=1.0, v_max=1.0))
    assert _lib.param_count(dict(configs.FULL, atoms=1, v_min=0.0, v_max=0.0)) == 1493335 - 2 * 100 * 513
    with pytest.raises(_lib.SquintError):
        _lib.param_count(dict(configs.FULL, hidden=2048))
    with pytest.raises(_lib.SquintError):
        _lib.workspace_bytes(configs.FULL, 7, 10)
    # null pointers / negative sizes: EINVAL before anything touches the device
    d = _lib.make_dims(configs.FULL)
    assert _lib.LIB.squint_downsample(ctypes.byref(d), None, None, 4, 0, None, None) == _lib.SQ_EINVAL
    assert _lib.LIB.encoder_fwd(ctypes.byref(d), 0, None, None, -1, None, None, None) == _lib.SQ_EINVAL
    assert _lib.LIB.sq_sample_indices(1, 0, 0, 10, None, None) == _lib.SQ_EINVAL
    assert _lib.LIB.sac_update(None, None, 1, None, None) == _lib.SQ_EINVAL
    assert _lib.LIB.act(None, None, None, 1, 0, 0, None, None) == _lib.SQ_EINVAL
    assert b"NULL" in _lib.LIB.sq_last_error() or b"agent" in _lib.LIB.sq_last_error()
    h = ctypes.c_void_p()
    assert _lib.LIB.sq_ring_create(ctypes.byref(d), 0, ctypes.byref(h)) == _lib.SQ_EINVAL
    assert _lib.LIB.sq_ring_insert(None, None, None, None, None, None, None, None, 1, None) == _lib.SQ_EINVAL
    assert _lib.LIB.sq_ring_view(None, None) == _lib.SQ_EINVAL
    assert _lib.LIB.sq_ring_copy_out(None, 0, 0, 1, None, None) == _lib.SQ_EINVAL
    assert _lib.LIB.sq_env_create(ctypes.byref(d), 4, 10, 1, None, ctypes.byref(h)) == _lib.SQ_EINVAL
    assert _lib.LIB.sq_env_step(None, None, None) == _lib.SQ_EINVAL


def test_workspace_sizes_grow_with_rows():
    from paper_2602_21203_amd import _lib, configs
    for op in (0, 1, 2):
        a = _lib.workspace_bytes(configs.FULL, op, 16)
        b = _lib.workspace_bytes(configs.FULL, op, 512)
        assert b > a > 0


def test_missing_library_fails_loudly():
    code = "import paper_2602_21203_amd._lib"
    env = dict(os.environ, SQ_LIB_PATH="/nonexistent/libsquint.so")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True)
    assert r.returncode != 0 and "missing" in r.stderr


def test_ring_rows_in_64_bit():
    """The ring row (pos + i) mod capacity, computed by the same function the
    insert kernel uses, where pos + i passes 2^31 (capacity near 2^31 - 1)."""
    from paper_2602_21203_amd import _lib
    cap = 2 ** 31 - 1
    for pos, i in ((cap - 10, 20), (cap - 1, 2 ** 31 - 1), (2 ** 30, 2 ** 31 - 1), (5, 0), (0, cap)):
        row = ctypes.c_int()
        assert _lib.LIB.sq_ring_row(pos, i, cap, ctypes.byref(row)) == _lib.SQ_OK
        assert row.value == (pos + i) % cap, (pos, i, row.value)
    row = ctypes.c_int()
    assert _lib.LIB.sq_ring_row(cap, 1, cap, ctypes.byref(row)) == _lib.SQ_EINVAL
    assert _lib.LIB.sq_ring_row(0, -1, cap, ctypes.byref(row)) == _lib.SQ_EINVAL


def _tile_order(gx, gy, gz):
    from paper_2602_21203_amd import _lib
    t = (ctypes.c_int * 3)()
    out = []
    for b in range(gx * gy * gz):
        assert _lib.LIB.sq_gemm_tile_order(b, gx, gy, gz, t) == _lib.SQ_OK
        out.append(tuple(t))
    return out


def test_gemm_workgroup_order_is_a_bijection():
    """Every workgroup of a product grid computes a distinct output tile and every
    tile is computed, for grids with and without a tile count divisible by 8."""
    for gx, gy, gz in ((16, 16, 2), (16, 16, 4), (32, 16, 1), (16, 4, 2), (4, 16, 4), (32, 1, 1), (3, 5, 1),
                       (7, 9, 2), (17, 3, 4), (1, 1, 1), (9, 1, 8)):
        tiles = _tile_order(gx, gy, gz)
        assert sorted(tiles) == sorted((x, y, z) for x in range(gx) for y in range(gy) for z in range(gz)), (gx, gy, gz)


def test_gemm_workgroup_order_gives_each_xcd_a_block():
    """Workgroup b runs on XCD b % 8: for the twin-layer grid (16 x 16 tiles, 2
    batches) each XCD's 64 tiles are an 8 x 8 block of one batch, so its L2 reads
    half of that batch's A rows and half of its W rows."""
    tiles = _tile_order(16, 16, 2)
    for xcd in range(8):
        mine = [tiles[b] for b in range(xcd, len(tiles), 8)]
        assert len({z for _, _, z in mine}) == 1
        assert len({x for x, _, _ in mine}) == 8 and len({y for _, y, _ in mine}) == 8
    from paper_2602_21203_amd import _lib
    t = (ctypes.c_int * 3)()
    assert _lib.LIB.sq_gemm_tile_order(512, 16, 16, 2, t) == _lib.SQ_EINVAL
    assert _lib.LIB.sq_gemm_tile_order(0, 0, 16, 2, t) == _lib.SQ_EINVAL
