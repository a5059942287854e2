"""GPU parity of the synthetic environment stub (sq_env_* through the C ABI)
against the oracle's, and of the environment -> ring data path of the
environment-step loop."""
import numpy as np
import pytest
import torch

from oracle import env as oenv
from oracle import ring as oring
from tests import helpers as H

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2602_21203_amd import api


def _actions(n, A, seed):
    return np.random.default_rng(seed).uniform(-1, 1, (n, A)).astype(np.float32)


@pytest.mark.parametrize("name,n,T", [("tiny", 37, 5), ("full", 64, 4)])
def test_env_matches_oracle(name, n, T):
    cfg = H.cfg(name)
    print(f"env {name} n={n} T={T}", flush=True)
    e_gpu = api.Env(cfg, n, episode_len=T, seed=9)
    e_ora = oenv.Env(n, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], T, seed=9)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(e_gpu.obs.cpu().numpy(), e_ora.obs)
    np.testing.assert_array_equal(e_gpu.proprio.cpu().numpy(), e_ora.s)
    for step in range(3 * T + 1):
        a = _actions(n, cfg["action"], 100 + step)
        e_gpu.step(torch.tensor(a, device="cuda"))
        tr = e_ora.step(a)
        torch.cuda.synchronize()
        obs_t, next_obs, prop_t, next_prop, _, reward, done = (x.cpu().numpy() for x in e_gpu.transition())
        np.testing.assert_array_equal(obs_t, tr["obs"])
        np.testing.assert_array_equal(next_obs, tr["next_obs"])
        np.testing.assert_array_equal(prop_t, tr["proprio"])
        np.testing.assert_array_equal(next_prop, tr["next_proprio"])
        np.testing.assert_allclose(reward, tr["reward"], rtol=1e-6, atol=1e-7)
        np.testing.assert_array_equal(done, tr["done"])
        np.testing.assert_array_equal(e_gpu.obs.cpu().numpy(), e_ora.obs)
        np.testing.assert_array_equal(e_gpu.proprio.cpu().numpy(), e_ora.s)
    e_gpu.close()


def test_env_to_ring_path_matches_oracle():
    """Environment steps stored by squint at insertion: the ring after several
    steps holds the oracle environment's transitions, squinted."""
    name, n, T, cap = "full", 48, 3, 100
    cfg = H.cfg(name)
    e_gpu = api.Env(cfg, n, episode_len=T, seed=4)
    e_ora = oenv.Env(n, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], T, seed=4)
    r_gpu = api.Ring(cfg, cap)
    r_ora = oring.Ring(cap, cfg["H"] // cfg["k"], cfg["C"], cfg["proprio"], cfg["action"])
    for step in range(5):
        a = _actions(n, cfg["action"], 200 + step)
        at = torch.tensor(a, device="cuda")
        e_gpu.step(at)
        obs_t, next_obs, prop_t, next_prop, act, reward, done = e_gpu.transition()
        r_gpu.insert(obs_t, next_obs, prop_t, next_prop, act, reward, done)
        tr = e_ora.step(a)
        # the oracle ring stores the oracle environment's FP64 reward rounded to FP32
        r_ora.insert(cfg["k"], tr["obs"], tr["next_obs"], tr["proprio"], tr["next_proprio"], tr["action"],
                     tr["reward"].astype(np.float32), tr["done"])
    torch.cuda.synchronize()
    for f in oring.FIELDS:
        got = r_gpu.read(f).cpu().numpy()
        if f == "reward":
            np.testing.assert_allclose(got, r_ora.reward, rtol=1e-6, atol=1e-7)
        else:
            np.testing.assert_array_equal(got, getattr(r_ora, f), err_msg=f)
    assert r_gpu.state() == (r_ora.pos, r_ora.size)
    r_gpu.close()
    e_gpu.close()
