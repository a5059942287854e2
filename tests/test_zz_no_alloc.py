"""encoder_fwd_noalloc (the encoder forward for callers that cannot allocate)
against encoder_fwd through the C ABI: the same feature bits, on two calls in a
row (the second with fewer images), for the fused 16x16 encoder in both
precisions, the tiny geometry and the general-geometry 32x32 convolutions; and
the size limit is enforced before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2602_21203_amd import synthetic
from tests import helpers as H

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2602_21203_amd import _lib, api


@pytest.mark.parametrize("name,prec,sizes", [("full", 1, (700, 33)), ("full", 0, (512, 100)),
                                             ("tiny", 1, (300, 7)), ("full32", 1, (130, 2))])
def test_noalloc_encoder_equals_workspace_encoder(name, prec, sizes):
    print(f"noalloc encoder {name} prec={prec} sizes={sizes}", flush=True)
    cfg = H.cfg(name)
    p = torch.as_tensor(H.params(name)).cuda()
    _, blocks = _lib.param_table(cfg)
    enc = p[blocks["enc"][0]:blocks["enc"][1]].contiguous()
    nmax = api.encoder_noalloc_max_images(cfg)
    assert nmax >= max(sizes), (nmax, sizes)
    frames = synthetic.frames(max(sizes), cfg["H"], cfg["W"], cfg["C"], seed=21).cuda()
    x_all = api.squint_downsample(cfg, frames)
    for n in sizes:
        x = x_all[:n].contiguous()
        want, _ = api.encoder_fwd(cfg, prec, enc, x)
        got = api.encoder_fwd_noalloc(cfg, prec, enc, x)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (n, (got - want).abs().max().item())
        assert torch.isfinite(got).all()


def test_noalloc_encoder_rejects_too_many_images():
    cfg = H.cfg("full")
    nmax = api.encoder_noalloc_max_images(cfg)
    d = _lib.make_dims(cfg)
    st = _lib.LIB.encoder_fwd_noalloc(ctypes.byref(d), 1, None, None, nmax + 1, None, None)
    assert st == _lib.SQ_EINVAL        # NULL arguments are checked first
    x = torch.zeros((1, 1), device="cuda")
    st = _lib.LIB.encoder_fwd_noalloc(ctypes.byref(d), 1, _lib.ptr(x), _lib.ptr(x), nmax + 1, _lib.ptr(x), None)
    assert st == _lib.SQ_ENOMEM
    assert b"scratch" in _lib.LIB.sq_last_error()
