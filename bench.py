#!/usr/bin/env python
"""Throughput of the fused Squint SAC update on one MI355X.

A step is one sac_update call of UTD (default 4) updates at batch 512 on the
full-size network (64x64x9 uint8 frames squinted 4x, 3 convs of 32 channels,
projection 256, twin 512-512 C51 critics with 101 atoms, 512-512 tanh-Gaussian
actor), replayed from a captured HIP graph; replay rows are seeded synthetic
frames resident in HBM (capacity 65,536 transitions).  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--prec bf16|fp32]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic counts per update at the full-size network, batch B (see design notes)
FULL = dict(C=9, H=64, W=64, k=4, n_conv=3, F=32, proj=256, hidden=512, atoms=101, proprio=12, action=6,
            v_min=-20.0, v_max=20.0)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--prec", choices=["bf16", "fp32"], default="bf16")
    ap.add_argument("--utd", type=int, default=4)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--capacity", type=int, default=65536)
    ap.add_argument("--frame", type=int, default=64, help="source frame side (64: k=4, 128: k=8)")
    ap.add_argument("--side", type=int, default=16, help="squinted side (16; 32 is the higher-resolution variant)")
    ap.add_argument("--serve-requests", type=int, default=2000, help="requests of the closed-loop serving point")
    ap.add_argument("--serve-rate", type=float, default=50000.0, help="Poisson point of the default line, obs/s")
    ap.add_argument("--serve-seconds-default", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the other-precision timing")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--no-insert", action="store_true", help="skip the insert-path (squint at insertion) timing")
    ap.add_argument("--cdq", action="store_true", help="clipped double-Q target instead of the twin average")
    ap.add_argument("--state", action="store_true",
                    help="state-based SAC (no image or encoder; a 40-float state in place of the features)")
    ap.add_argument("--env-loop", action="store_true",
                    help="environment-step loop with the synthetic environment stub (time breakdown)")
    ap.add_argument("--envs", type=int, default=1024)
    ap.add_argument("--loop-utd", type=int, default=256, help="updates per environment step in --env-loop")
    ap.add_argument("--loop-steps", type=int, default=8)
    ap.add_argument("--loop-warmup", type=int, default=2)
    ap.add_argument("--scalar-critic", action="store_true",
                    help="scalar critics on the squared Bellman error instead of C51")
    ap.add_argument("--sweep", action="store_true",
                    help="UTD sweep {1,4,8,16} at batch 1024 on 128x128x9 frames (prints one JSON line)")
    ap.add_argument("--serve", action="store_true",
                    help="Poisson act() load at 2k..50k obs/s, pools U{1..4096} (prints one JSON line)")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--report", action="store_true",
                    help="errors after 1 and N updates vs the FP64 oracle, BF16 and FP32 (prints one JSON line)")
    ap.add_argument("--report-updates", type=int, default=100)
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 256 MiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def cfg_for(frame, side=16):
    c = dict(FULL)
    c["H"] = c["W"] = frame
    c["k"] = frame // side
    return c


def side_of(cfg):
    return cfg["H"] // cfg["k"]


def squint_kernel_name(cfg, mode=""):
    if (cfg["C"], cfg["k"], side_of(cfg)) in ((9, 4, 16), (9, 8, 16), (9, 4, 32)):
        return f"k_squint_ck<9,{cfg['k']},{side_of(cfg)}>" + mode
    return "k_squint" + mode


def time_updates(agent, rep, utd, steps, warmup):
    import torch
    stats = torch.empty((utd, 8), dtype=torch.float32, device="cuda")
    # the training loop issues its updates on the agent's own stream
    for _ in range(warmup):
        agent.sac_update(rep, utd, stats=stats, stream=agent.stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(agent.stream)
    for _ in range(steps):
        agent.sac_update(rep, utd, stats=stats, stream=agent.stream)
    ev1.record(agent.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu = ev0.elapsed_time(ev1) / 1e3
    s = stats.cpu().numpy()
    return wall, gpu, s


def graph_time(fn, reps):
    """Average device time of one call of fn (a single library kernel launch):
    reps calls captured in one HIP graph on a side stream, the graph replayed
    five times between HIP events recorded on that same stream."""
    import torch
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        for _ in range(3):
            fn()
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(reps):
            fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(s):
        g.replay()
        e0.record(s)
        for _ in range(5):
            g.replay()
        e1.record(s)
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / (5 * reps)
    del g
    return t


def squint_kernel_time(cfg, rep, B, reps):
    """Average duration of the squint gather kernel (2B frames, as inside the
    update).  Every launch of the timed graph gathers its own random rows, so
    the frames come from HBM as in the update, not from a cache that a repeated
    gather of the same rows would keep warm."""
    import torch

    from paper_2602_21203_amd import api
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    idxs = [torch.randint(0, rep["obs"].shape[0], (2 * B,), generator=g, dtype=torch.int32, device="cuda")
            for _ in range(reps)]
    out = torch.empty((2 * B, cfg["C"], side_of(cfg), side_of(cfg)), dtype=torch.float32, device="cuda")
    calls = [0]

    def one():
        api.squint_downsample(cfg, rep["obs"], idxs[calls[0] % reps], out=out)
        calls[0] += 1
    return graph_time(one, reps)


def measured_traffic(kernel_key, source):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, each counter scaled by what it reads for a 256 MiB copy; None when
    the kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_counters_gemm_squint.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    fetch_f = float(re_search(r"copy FETCH_SIZE [\d.]+ KiB -> factor ([\d.]+)", text))
    write_f = float(re_search(r"copy WRITE_SIZE [\d.]+ KiB -> factor ([\d.]+)", text))
    m = re_search(kernel_key + r"\s+source=(\w+)\s+([\d.]+)\s+([\d.]+)", text, groups=True)
    if m is None:
        return None
    digest = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()[:16]
    if m[0] != digest:
        return None
    return round((float(m[1]) * fetch_f + float(m[2]) * write_f) * 1024)


def measured_mfma_busy(kernel_key, source):
    """MFMA busy share (%) of the kernel from the committed counter summary, None
    when the kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_counters_gemm_squint.txt")
    if not os.path.exists(path):
        return None
    m = re_search(kernel_key + r"\s+source=(\w+)\s+mfma_busy_pct=([\d.]+)", open(path).read(), groups=True)
    if m is None:
        return None
    digest = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()[:16]
    return float(m[1]) if m[0] == digest else None


def measured_profiled_us(kernel_key, source):
    """Mean kernel duration (us) of the standalone launches in the committed
    kernel trace, None when the kernel's source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_counters_gemm_squint.txt")
    if not os.path.exists(path):
        return None
    m = re_search(kernel_key + r"\s+source=(\w+)\s+profiled_us=([\d.]+)", open(path).read(), groups=True)
    if m is None:
        return None
    digest = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()[:16]
    return float(m[1]) if m[0] == digest else None


def profiled_figure(kernel_key, source, work, peak, scale):
    """The roofline figure from the committed profile's kernel duration: work
    (FLOP or bytes) per launch / profiled mean duration, against peak."""
    us = measured_profiled_us(kernel_key, source)
    if us is None:
        return None
    ach = work / (us * 1e-6) / scale
    return {"avg_us": us, "achieved": round(ach, 2), "frac": round(ach / peak, 5),
            "method": "the mean duration of the same standalone launches in the committed rocprofv3 kernel trace "
                      "(profiles/sac_update_full_b512_bf16_kernels.txt, profiler attached)"}


def re_search(pat, text, groups=False):
    import re
    m = re.search(pat, text)
    if m is None:
        return None
    return m.groups() if groups else m.group(1)


def gemm_kernel_time(prec, reps):
    """Average duration of the largest linear-layer product of the update -- the
    twin critics' second hidden layer, C[2, 512, 512] = A[2, 512, 512] W[2]^T + b
    -- launched alone with the same kernel, shapes and operand layouts (in the
    bfloat16 mode the update's forward products read bfloat16 copies of A and W)."""
    import torch

    from paper_2602_21203_amd import _lib, api
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    A = torch.rand((2, 512, 512), generator=g, device="cuda")
    W = torch.rand((2, 512, 512), generator=g, device="cuda") - 0.5
    b = torch.rand((2, 512), generator=g, device="cuda")
    C = torch.empty((2, 512, 512), device="cuda")
    if prec == _lib.SQ_BF16:
        Ah, Wh = A.to(torch.bfloat16), W.to(torch.bfloat16)
        return graph_time(lambda: api.gemm_bf16(Ah, Wh, C, bias=b), reps)
    return graph_time(lambda: api.gemm(prec, A, W, C, bias=b), reps)


def insert_path(cfg, rep, agent, a, n_env=1024):
    """The insert path: squint at insertion of n_env transitions per call (one
    environment step of n_env parallel envs) into a device FIFO ring of uint8
    block means, then UTD updates sampling the ring instead of raw frames."""
    import torch

    from paper_2602_21203_amd import api
    cap = a.capacity
    n_env = min(n_env, cap)
    ring = api.Ring(cfg, cap)
    names = ("obs", "next_obs", "proprio", "next_proprio", "action", "reward", "done")
    chunks = max(1, cap // n_env)

    # the per-chunk argument slices are made before timing, so the timed loop is
    # the library calls alone; the best of three passes discounts host hiccups
    # (each call is submitted from the host, so a stalled host shows as idle GPU)
    args = [tuple(rep[f][i * n_env:(i + 1) * n_env] for f in names) for i in range(chunks)]

    def insert(i):
        ring.insert(*args[i % chunks], stream=agent.stream)

    for i in range(4):
        insert(i)
    torch.cuda.synchronize()
    calls = 2 * chunks
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_call = float("inf")
    for _ in range(3):
        e0.record(agent.stream)
        for i in range(calls):
            insert(i)
        e1.record(agent.stream)
        torch.cuda.synchronize()
        t_call = min(t_call, e0.elapsed_time(e1) / 1e3 / calls)
    P, A = cfg["proprio"], cfg["action"]
    frame_bytes = 2 * (cfg["H"] * cfg["W"] * cfg["C"] + side_of(cfg) ** 2 * cfg["C"])
    field_bytes = 2 * (4 * (2 * P + A + 1) + 1)
    per_call = n_env * (frame_bytes + field_bytes)
    ach = per_call / t_call / 1e9
    wall, gpu, _ = time_updates(agent, ring, a.utd, a.steps, a.warmup)
    out = {"transitions_per_insert": n_env, "ring_rows": cap,
           "insert_transitions_per_s": round(n_env / t_call, 1), "insert_us": round(t_call * 1e6, 3),
           "roofline_insert": {"kernel": squint_kernel_name(cfg, " in uint8-ring mode (one insert call: frames and fields)"),
                               "bound": "hbm", "achieved": round(ach, 1), "peak": 8000.0, "unit": "GB/s",
                               "frac": round(ach / 8000.0, 4),
                               "traffic": measured_traffic("squint_insert_1024",
                                                           "paper_2602_21203_amd/csrc/kernels/squint.hip")
                               if (n_env, cfg["H"], side_of(cfg)) == (1024, 64, 16) else None,
                               "algorithmic_bytes": per_call},
           "ring_updates_per_s": round(a.utd * a.steps / wall, 2),
           "ring_gpu_event_updates_per_s": round(a.utd * a.steps / gpu, 2)}
    ring.close()
    return out


def _serve_pool(cfg):
    import torch

    from paper_2602_21203_amd import synthetic
    pool = synthetic.frames(4096, cfg["H"], cfg["W"], cfg["C"], seed=11, device="cuda")
    prop = torch.randn(4096, cfg["proprio"], device="cuda")
    torch.cuda.synchronize()
    return pool, prop


def _latency_summary(srv, t_sub, sizes, t0, t1):
    lat = sorted(srv.done[j] - t_sub[j] for j in range(len(sizes)))
    st = srv.stats()
    pct = lambda q: lat[min(len(lat) - 1, int(q * len(lat)))] * 1e3
    return {"requests": len(sizes), "p50_ms": round(pct(0.5), 3), "p99_ms": round(pct(0.99), 3),
            "achieved_obs_per_s": round(float(sum(sizes)) / (t1 - t0), 1),
            "gpu_busy_frac": round(st["device_busy_s"] / (t1 - t0), 4),
            "batches": st["batches"], "fused_batches": st["fused_batches"],
            "max_requests_per_batch": st["max_requests_per_batch"], "max_slots_busy": st["max_slots_busy"],
            "overlapped_batches": st["overlapped_batches"]}


def serve_poisson(agent, cfg, pool, prop, rate, seconds, max_requests, seed=3):
    """Poisson arrivals of pools U{1..4096} at `rate` observations/s (request rate
    rate / 2048.5) through the continuous-batching server, for `seconds` or
    max_requests requests, whichever comes first.  Latency = completion (host
    steady clock, in the server's callback) - scheduled arrival."""
    import numpy as np

    from paper_2602_21203_amd import api
    rng = np.random.default_rng(seed)
    srv = api.Server(agent, mem_budget=16 << 30, max_batch_obs=8192, n_slots=4)
    lam = rate / 2048.5
    t_sub, sizes = {}, []
    t0 = time.monotonic()
    t_next = t0
    while len(sizes) < max_requests and time.monotonic() - t0 < seconds:
        t_next += rng.exponential(1.0 / lam)
        while True:
            now = time.monotonic()
            if now >= t_next:
                break
            time.sleep(min(0.0005, t_next - now))
        n = int(rng.integers(1, 4097))
        t_sub[len(sizes)] = t_next
        sizes.append(n)
        srv.submit(pool[:n], prop[:n], len(sizes) - 1, sample=True)
    srv.drain()
    out = dict(offered_obs_per_s=rate, **_latency_summary(srv, t_sub, sizes, t0, time.monotonic()))
    srv.close()
    return out


def serve_closed_loop(agent, cfg, pool, prop, n_req=2000, in_flight=8, seed=4):
    """Closed-loop saturation: n_req pools U{1..4096}, a new request submitted as
    soon as fewer than `in_flight` are outstanding."""
    import threading

    import numpy as np

    from paper_2602_21203_amd import api
    rng = np.random.default_rng(seed)
    srv = api.Server(agent, mem_budget=16 << 30, max_batch_obs=8192, n_slots=4)
    cv = threading.Condition()
    base_cb = srv._on_done

    def on_done(rid, t, user):
        base_cb(rid, t, user)
        with cv:
            cv.notify()
    srv._cb = api.L.DONE_CB(on_done)
    t_sub, sizes = {}, []
    t0 = time.monotonic()
    for i in range(n_req):
        with cv:
            cv.wait_for(lambda: i - len(srv.done) < in_flight)
        n = int(rng.integers(1, 4097))
        t_sub[i] = time.monotonic()
        sizes.append(n)
        srv.submit(pool[:n], prop[:n], i, sample=True)
    srv.drain()
    out = dict(in_flight=in_flight, **_latency_summary(srv, t_sub, sizes, t0, time.monotonic()))
    srv.close()
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, B, budget_s=12.0):
    """The FP64 oracle timed on the host cores on a bounded sample of updates,
    with the BLAS pool at all its threads and at one thread."""
    import numpy as np
    import torch
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import layout as olayout
    from oracle import sac
    from paper_2602_21203_amd import synthetic
    d = olayout.dims(**cfg)
    table = [(n, o, s) for n, (o, s) in olayout.offsets(d)[0].items()]
    params = synthetic.init_params(table, seed=1).astype(np.float64)
    cpu = synthetic.replay(2048, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], seed=0)
    rep = {k: (v.numpy() if torch.is_tensor(v) else v) for k, v in cpu.items()}
    hp = sac.hparams(d)

    def rate(budget):
        st = sac.new_state(d, params)
        sac.sac_update(st, rep, d, hp, B)          # warm-up (not timed)
        n, t0 = 0, time.perf_counter()
        while n < 2 or (time.perf_counter() - t0 < budget and n < 100):
            sac.sac_update(st, rep, d, hp, B)
            n += 1
        return n, n / (time.perf_counter() - t0)

    n_all, r_all = rate(budget_s)
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    with threadpool_limits(limits=1):
        n_one, r_one = rate(budget_s)
    return dict(value=r_all, unit="updates/s", cores=int(threads), kind="oracle",
                sample=f"{n_all} FP64 oracle updates at batch {B} (full network, 64x64x9 frames) after 1 warm-up, "
                       f"BLAS pool of {threads} threads; one thread: {n_one} updates",
                cpu_model=cpu_model(), host_cpus=os.cpu_count(), one_thread_value=r_one)


def run_sweep(a):
    import torch

    from paper_2602_21203_amd import _lib, api, synthetic
    cfg = cfg_for(128)
    B = 1024
    rep = synthetic.replay(32768, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], seed=0,
                           device="cuda")
    table, _ = _lib.param_table(cfg)
    params = synthetic.init_params(table, seed=1)
    out = {"mode": "utd_sweep", "workload": "full network, batch 1024, 128x128x9 frames squinted 8x, "
                                            "replay 32768 rows", "unit": "updates/s", "points": []}
    for prec_name, prec in (("bf16", _lib.SQ_BF16), ("fp32", _lib.SQ_F32)):
        for utd in (1, 4, 8, 16):
            ag = api.Agent(cfg, params, B, prec=prec)
            steps = max(4, 64 // utd)
            wall, gpu, _ = time_updates(ag, rep, utd, steps, 2)
            out["points"].append({"precision": prec_name, "utd": utd, "updates_per_s": round(utd * steps / wall, 2),
                                  "ms_per_launch": round(wall / steps * 1e3, 3)})
            ag.close()
    print(json.dumps(out))


def run_env_loop(a):
    """Alg. 1's environment-step loop end to end on the device, with the synthetic
    environment stub in place of the simulator: per environment step, act() on
    every environment (tanh-Gaussian samples), step the environments, store the
    transitions by squint at insertion, then UTD updates sampling the ring.  HIP
    events between the phases give the time breakdown."""
    import torch

    from paper_2602_21203_amd import _lib, api, synthetic
    cfg = cfg_for(a.frame, a.side)
    n_env, utd, B = a.envs, a.loop_utd, a.batch
    table, _ = _lib.param_table(cfg)
    params = synthetic.init_params(table, seed=1)
    prec = _lib.SQ_BF16 if a.prec == "bf16" else _lib.SQ_F32
    agent = api.Agent(cfg, params, B, prec=prec)
    env = api.Env(cfg, n_env, episode_len=50, seed=3)
    ring = api.Ring(cfg, a.capacity)
    st = agent.stream
    stats = torch.empty((utd, 8), dtype=torch.float32, device="cuda")
    act_out = torch.empty((n_env, cfg["action"]), dtype=torch.float32, device="cuda")
    phases = ("act", "env_step", "insert", "updates")
    tot = dict.fromkeys(phases, 0.0)

    def env_step(t, timed):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(st)
        agent.act(env.obs, env.proprio, sample=True, request_id=t, out=act_out, stream=st)
        ev[1].record(st)
        env.step(act_out, stream=st)
        ev[2].record(st)
        ring.insert(*env.transition(), stream=st)
        ev[3].record(st)
        agent.sac_update(ring, utd, stats=stats, stream=st)
        ev[4].record(st)
        return ev

    for t in range(a.loop_warmup):
        env_step(t, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [env_step(a.loop_warmup + t, True) for t in range(a.loop_steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for ev in evs:
        for i, ph in enumerate(phases):
            tot[ph] += ev[i].elapsed_time(ev[i + 1]) / 1e3
    dev = sum(tot.values())
    out = {"mode": "env_loop",
           "workload": f"Alg. 1 outer loop with the synthetic environment stub: {n_env} environments, "
                       f"{cfg['H']}x{cfg['W']}x{cfg['C']} frames squinted at insertion to {side_of(cfg)}x{side_of(cfg)}, "
                       f"{utd} updates of batch {B} ({a.prec}) per environment step, ring {a.capacity} rows",
           "env_steps": a.loop_steps, "env_steps_per_s": round(a.loop_steps / wall, 3),
           "transitions_per_s": round(a.loop_steps * n_env / wall, 1),
           "updates_per_s": round(a.loop_steps * utd / wall, 2),
           "ms_per_env_step": {ph: round(tot[ph] / a.loop_steps * 1e3, 4) for ph in phases},
           "share": {ph: round(tot[ph] / dev, 5) for ph in phases},
           "final_stats": {n: float(v) for n, v in zip(_lib.STAT_NAMES, stats[-1].cpu().numpy())}}
    ring.close()
    env.close()
    agent.close()
    print(json.dumps(out))


def run_serve(a):
    from paper_2602_21203_amd import _lib, api, synthetic
    cfg = cfg_for(64)
    table, _ = _lib.param_table(cfg)
    params = synthetic.init_params(table, seed=1)
    agent = api.Agent(cfg, params, 32, prec=_lib.SQ_BF16)
    pool, prop = _serve_pool(cfg)
    out = {"mode": "act_serving", "workload": "act() of BF16 full network on 64x64x9 frames, pools U{1..4096}, "
                                              "Poisson arrivals, 4 stream slots, weights resident",
           "points": []}
    # the configured rates (a few requests per second: each point holds what
    # arrives in --serve-seconds), then rates that load the device, where 2000
    # requests arrive within seconds
    for rate in (2000, 5000, 10000, 20000, 50000, 500000, 2000000, 8000000):
        p = serve_poisson(agent, cfg, pool, prop, rate, a.serve_seconds, 2000)
        print(json.dumps(p), file=sys.stderr, flush=True)
        out["points"].append(p)
    out["closed_loop"] = [serve_closed_loop(agent, cfg, pool, prop, 2000, k) for k in (1, 4, 8, 16)]
    agent.close()
    print(json.dumps(out))


def run_report(a):
    """Precision report: GPU BF16 and FP32 updates against three references over
    the same N updates -- the FP64 oracle, the oracle's bfloat16-operand mode, and
    the FP32 GPU path -- on the loss statistics, the first update's gradients and
    the parameters after N updates."""
    import numpy as np
    import torch

    from oracle import layout as olayout
    from oracle import sac
    from paper_2602_21203_amd import _lib, api, synthetic
    cfg = cfg_for(64)
    B = a.batch
    d = olayout.dims(**cfg)
    table = [(n, o, s) for n, (o, s) in olayout.offsets(d)[0].items()]
    params = synthetic.init_params(table, seed=1)
    cpu = synthetic.replay(8192, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], seed=0)
    gpu = {k: (v.cuda() if torch.is_tensor(v) else v) for k, v in cpu.items()}
    npr = {k: (v.numpy() if torch.is_tensor(v) else v) for k, v in cpu.items()}
    N = a.report_updates
    blk = olayout.blocks(d)

    def flat_grads(o):
        g = np.zeros(blk["total"])
        g[:blk["critic"][1]] = o["g_enc_critic"]
        g[blk["actor"][0]:blk["actor"][1]] = o["g_actor"]
        g[blk["log_alpha"][0]] = o["g_log_alpha"][0]
        return g

    refs = {}
    for name, bf in (("oracle_fp64", False), ("oracle_bf16_operands", True)):
        st = sac.new_state(d, params.astype(np.float64))
        hp = sac.hparams(d)
        stats, g1 = [], None
        for u in range(N):
            if u % 10 == 0:
                print(f"{name} update {u}/{N}", file=sys.stderr, flush=True)
            o = sac.sac_update(st, npr, d, hp, B, bf=bf)
            stats.append(o["stats"])
            if u == 0:
                g1 = flat_grads(o)
        refs[name] = dict(stats=np.array(stats), g1=g1, pN=st.params.copy())
    runs = {}
    for name, prec in (("bf16", _lib.SQ_BF16), ("fp32", _lib.SQ_F32)):
        ag = api.Agent(cfg, params, B, prec=prec)
        s1 = ag.sac_update(gpu, 1, graph=False).cpu().numpy()
        torch.cuda.synchronize()
        g1 = ag.grads.double().cpu().numpy()
        sN = ag.sac_update(gpu, N - 1, graph=True).cpu().numpy() if N > 1 else s1[:0]
        torch.cuda.synchronize()
        runs[name] = dict(stats=np.concatenate([s1, sN]).astype(np.float64), g1=g1,
                          pN=ag.params.double().cpu().numpy())
        ag.close()
    refs["gpu_fp32"] = runs["fp32"]
    rel = lambda x, y: float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-30))

    def worst_tensor(g, r):
        w = (0.0, "")
        for n, (o, shp) in olayout.offsets(d)[0].items():
            k = int(np.prod(shp))
            w = max(w, (rel(g[o:o + k], r[o:o + k]), n))
        return {"rel_err": w[0], "tensor": w[1]}

    out = {"mode": "precision_report", "batch": B, "updates": N, "workload": "full network, 64x64x9 frames",
           "results": {}}
    for name, run in runs.items():
        res = {}
        for rname, ref in refs.items():
            if rname == "gpu_fp32" and name == "fp32":
                continue
            S, R = run["stats"], ref["stats"]
            cl = np.abs(S[:, 0] - R[:, 0]) / np.abs(R[:, 0])
            res["vs_" + rname] = {
                "critic_loss_rel_err_update1": float(cl[0]), "critic_loss_rel_err_last": float(cl[-1]),
                "critic_loss_rel_err_max": float(cl.max()),
                "critic_loss_rel_err_by_update": [float(cl[i]) for i in (0, 1, 3, 9, 29, N - 1) if i < N],
                "actor_loss_abs_err_update1": float(abs(S[0, 1] - R[0, 1])),
                "actor_loss_abs_err_last": float(abs(S[-1, 1] - R[-1, 1])),
                "grad_rel_err_update1": rel(run["g1"], ref["g1"]),
                "grad_worst_tensor_update1": worst_tensor(run["g1"], ref["g1"]),
                "param_rel_err_last": rel(run["pN"], ref["pN"]),
            }
        out["results"][name] = res
    print(json.dumps(out))


def main():
    a = parse()
    if a.sweep or a.serve or a.report or a.env_loop:
        if a.gpus != 1:
            print(json.dumps({"error": "this implementation runs on one GPU", "n_gpus": a.gpus}))
            sys.exit(2)
        (run_sweep if a.sweep else run_serve if a.serve else run_report if a.report else run_env_loop)(a)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    from paper_2602_21203_amd import _lib, api, synthetic
    cfg = cfg_for(a.frame, a.side)
    if a.state:
        # state-based SAC: no image or encoder; a 40-float state vector feeds the
        # projections (the replay's frames are tiny and never read)
        cfg = dict(cfg, n_conv=0, H=8, W=8, C=3, k=1, proprio=40)
    if a.scalar_critic:
        cfg["atoms"] = 1
    B = a.batch
    torch.cuda.init()
    rep = synthetic.replay(a.capacity, cfg["H"], cfg["W"], cfg["C"], cfg["proprio"], cfg["action"], seed=0,
                           device="cuda")
    table, _ = _lib.param_table(cfg)
    params = synthetic.init_params(table, seed=1)
    prec = _lib.SQ_BF16 if a.prec == "bf16" else _lib.SQ_F32
    agent = api.Agent(cfg, params, B, prec=prec, cdq=a.cdq)
    wall, gpu, stats = time_updates(agent, rep, a.utd, a.steps, a.warmup)
    ups = a.utd * a.steps / wall
    result = {
        "metric": "SAC updates/sec at batch 512 (BF16 vs FP32, 1 GPU); act() p50/p99 latency",
        "value": round(ups, 2), "unit": "updates/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": a.prec, "data": "synthetic",
        "config": {"workload": f"{'state-based' if a.state else 'visual'} SAC update, full network"
                               f"{' (scalar critics)' if a.scalar_critic else ''}"
                               f"{' (clipped double-Q target)' if a.cdq else ''}, batch {B}, "
                               + ("40-float state vectors" if a.state else
                                  f"{a.frame}x{a.frame}x9 uint8 frames squinted to {side_of(cfg)}x{side_of(cfg)}")
                               + f", UTD {a.utd} per HIP-graph launch, replay {a.capacity} rows",
                   "global_batch": B, "utd": a.utd, "precision": a.prec},
        "gpu_event_updates_per_s": round(a.utd * a.steps / gpu, 2),
        "final_stats": {n: float(v) for n, v in zip(_lib.STAT_NAMES, stats[-1])},
    }
    if not a.no_compare:
        other = _lib.SQ_F32 if prec == _lib.SQ_BF16 else _lib.SQ_BF16
        ag2 = api.Agent(cfg, params, B, prec=other, cdq=a.cdq)
        w2, _, _ = time_updates(ag2, rep, a.utd, max(5, a.steps // 2), max(2, a.warmup // 2))
        result["fp32_updates_per_s" if other == _lib.SQ_F32 else "bf16_updates_per_s"] = \
            round(a.utd * max(5, a.steps // 2) / w2, 2)
        ag2.close()
    # dominant kernel (most device time per update): the linear-layer MFMA product
    t_g = gemm_kernel_time(prec, a.kernel_reps)
    flops = 2 * 2 * 512 * 512 * 512
    peak = 2500.0 if a.prec == "bf16" else 157.3
    ach = flops / t_g / 1e12
    bf = a.prec == "bf16"
    result["roofline"] = {"kernel": "k_gemm_h (twin critic layer 2 forward on bfloat16 operand copies, "
                                    "2 x 512x512x512)" if bf else
                                    "k_gemm_r (twin critic layer 2 forward, 2 x 512x512x512)", "bound": "mfma",
                          "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 5),
                          "traffic": measured_traffic("gemm_twin_l2_fwd_bf16", "paper_2602_21203_amd/csrc/kernels/gemm.hip")
                          if a.prec == "bf16" else None,
                          "mfma_busy_pct": measured_mfma_busy("gemm_twin_l2_fwd_bf16",
                                                              "paper_2602_21203_amd/csrc/kernels/gemm.hip")
                          if a.prec == "bf16" else None,
                          "avg_us": round(t_g * 1e6, 3), "algorithmic_flops": flops,
                          "method": "achieved = algorithmic FLOP per launch / avg_us, the start-to-start period of "
                                    "back-to-back launches replayed from a HIP graph (HIP events on the launch stream)",
                          # A and W (bfloat16 copies, or FP32), C in FP32, the bias
                          "algorithmic_bytes": 2 * 2 * 512 * 512 * (2 if bf else 4) + 2 * 512 * 512 * 4 + 2 * 512 * 4,
                          "profiled": profiled_figure("gemm_twin_l2_fwd_bf16",
                                                      "paper_2602_21203_amd/csrc/kernels/gemm.hip", flops, peak, 1e12)
                          if a.prec == "bf16" else None}
    if a.state:
        agent.close()
        print(json.dumps(result))
        return
    # the HBM-bound step: squint gather of 2B frames (frames read + FP32 images written)
    t_k = squint_kernel_time(cfg, rep, B, a.kernel_reps)
    bytes_per_launch = 2 * B * (cfg["H"] * cfg["W"] * cfg["C"] + cfg["C"] * side_of(cfg) ** 2 * 4)
    achieved = bytes_per_launch / t_k / 1e9
    result["roofline_squint"] = {"kernel": squint_kernel_name(cfg, f" (gather + {cfg['k']}x{cfg['k']} area sum of 2B frames)"),
                                 "bound": "hbm",
                                 "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                                 "frac": round(achieved / 8000.0, 4),
                                 "traffic": measured_traffic("squint_2B_frames",
                                                             "paper_2602_21203_amd/csrc/kernels/squint.hip")
                                 if (B, cfg["H"], side_of(cfg)) == (512, 64, 16) else None,
                                 "avg_us": round(t_k * 1e6, 3), "algorithmic_bytes": bytes_per_launch,
                                 "profiled": profiled_figure("squint_2B_frames",
                                                             "paper_2602_21203_amd/csrc/kernels/squint.hip",
                                                             bytes_per_launch, 8000.0, 1e9)
                                 if (B, cfg["H"], side_of(cfg)) == (512, 64, 16) else None}
    if a.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = src.clone()
        torch.cuda.synchronize()
        del src, dst
    if not a.no_insert:
        result["insert_path"] = insert_path(cfg, rep, agent, a)
    if a.serve_requests > 0:
        pool, prop = _serve_pool(cfg)
        result["act_serving"] = {
            "workload": "act() of the full network (agent precision) on 64x64x9 frames, pools U{1..4096}, "
                        "4 stream slots, weights resident",
            "poisson": serve_poisson(agent, cfg, pool, prop, a.serve_rate, a.serve_seconds_default, 2000),
            "closed_loop": serve_closed_loop(agent, cfg, pool, prop, a.serve_requests, 8)}
    agent.close()
    if not a.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(cfg, B)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
