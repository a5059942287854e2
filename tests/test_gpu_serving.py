"""The continuous-batching act() server: results alone equal results in a mix
(bitwise), admission by memory, FIFO completion of every request."""
import time

import numpy as np
import pytest
import torch

from paper_2602_21203_amd import synthetic
from tests import helpers as H

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2602_21203_amd import _lib, api


@pytest.fixture(scope="module")
def setup():
    cfg = H.cfg("full")
    torch.manual_seed(0)
    frames = synthetic.frames(3000, cfg["H"], cfg["W"], cfg["C"], seed=9, device="cuda")
    prop = torch.randn(3000, cfg["proprio"], device="cuda")
    agent = api.Agent(cfg, H.params("full"), 32, prec=1)
    return cfg, frames, prop, agent


def test_alone_equals_mixed_bitwise(setup):
    cfg, frames, prop, agent = setup
    sizes = [1, 7, 300, 2, 1000, 64, 5, 900, 33, 17]
    offs = np.cumsum([0] + sizes)
    reqs = [(frames[offs[i]:offs[i + 1]], prop[offs[i]:offs[i + 1]], 1000 + i, i % 2 == 1) for i in range(len(sizes))]
    # alone: plain act() one request at a time
    alone = [agent.act(f, p, sample=s, request_id=rid) for f, p, rid, s in reqs]
    torch.cuda.synchronize()
    # admissions held while the ten requests queue, then released: with at most
    # 1100 rows per launch the scheduler fuses them into three launches, one per
    # slot ([1, 7, 300, 2], [1000, 64, 5], [900, 33, 17]), that run at once
    srv = api.Server(agent, mem_budget=8 << 30, max_batch_obs=1100, n_slots=3)
    srv.hold(True)
    outs = [srv.submit(f, p, rid, sample=s) for f, p, rid, s in reqs]
    srv.hold(False)
    srv.drain()
    torch.cuda.synchronize()
    for a, b in zip(alone, outs):
        assert torch.equal(a, b)
    assert sorted(srv.done) == [r[2] for r in reqs]
    st = srv.stats()
    print("  server stats:", st)
    assert st["batches"] == 3 and st["fused_batches"] == 3 and st["max_requests_per_batch"] == 4
    assert st["requests"] == 10 and st["rows"] == sum(sizes)
    assert st["max_slots_busy"] == 3
    # the three batches' device intervals overlap (timing events on the slot streams)
    assert st["overlapped_batches"] >= 1
    assert 0 < st["device_busy_s"] < 3 * st["device_span_s"]
    srv.close()


def test_memory_admission_and_limits(setup):
    cfg, frames, prop, agent = setup
    per_obs = _lib.workspace_bytes(cfg, _lib.SQ_OP_ACTOR, 1)  # order of magnitude only
    assert per_obs > 0
    # a budget that fits ~100 observations: a 2000-row request is refused up front
    srv = api.Server(agent, mem_budget=100 * 40 * 1024, max_batch_obs=2048, n_slots=2)
    with pytest.raises(_lib.SquintError, match="exceeds"):
        srv.submit(frames[:2000], prop[:2000], 1)
    # requests that fit alone but not together are serialised, and all complete
    outs = [srv.submit(frames[i * 60:(i + 1) * 60], prop[i * 60:(i + 1) * 60], 10 + i) for i in range(6)]
    srv.drain()
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        ref = agent.act(frames[i * 60:(i + 1) * 60], prop[i * 60:(i + 1) * 60])
        assert torch.equal(o, ref)
    t = [srv.done[10 + i] for i in range(6)]
    assert t == sorted(t)   # FIFO without skipping: completions in submit order
    srv.close()


def test_poisson_burst_completes(setup):
    cfg, frames, prop, agent = setup
    srv = api.Server(agent, mem_budget=8 << 30, max_batch_obs=8192, n_slots=4)
    rng = np.random.default_rng(3)
    sub = {}
    for i in range(40):
        n = int(rng.integers(1, 3000))
        s0 = int(rng.integers(0, 3000 - n + 1))
        sub[i] = time.perf_counter()
        srv.submit(frames[s0:s0 + n], prop[s0:s0 + n], i, sample=bool(i % 3 == 0))
    srv.drain()
    assert len(srv.done) == 40
    srv.close()
