"""Throughput benchmark: rendered env-steps/s of the batched step + raycast render.

Headline workload: 4096 envs, 16x16 seeded mazes with loops, 8 wall colours,
goal billboard, 6 uniform-random actions, 64x64 RGB frames, 512-step episodes
with auto-reset.  Warm-up steps are untimed; the timed region runs K steps with
every frame written into a 128-slot rollout ring (6.4 GB), so the 256 MB
last-level cache cannot absorb the observation writes.  Inputs (maps, state,
actions) are resident in HBM before timing starts.

    python bench.py [--steps K] [--warmup W] [--form graph|eager|persistent]

Prints one JSON line.  Only N = 1 GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
RING = 128


def progress(msg: str) -> None:
    """One progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(cfg: dict, steps_per_launch: int = 1) -> dict:
    """HBM bytes one env must move at minimum, per env-step, when one launch
    advances it `steps_per_launch` steps.  Frames, actions, rewards and done
    flags move every step; the layout and the state are read once and the
    state written once per launch."""
    N = cfg["side"]
    T = max(1, steps_per_launch)
    obs = cfg["obs_h"] * cfg["obs_w"] * 3
    map_read = (N * N + 15) // 16 * 16
    # x y theta t episode goal door key (8 x 4) + decor (8) + flags, n_decor (2)
    # + seed (8) + cfg index, map offset (8) + frame offset (8)
    state_read = 32 + 8 + 2 + 8 + 8 + 8
    # x y theta t episode goal door key (32) + decor (8) + flags, n_decor, events (3)
    state_write = 32 + 8 + 3
    per_step = obs + 1 + 4 + 1  # frame, action, reward, done
    once = map_read + state_read + state_write
    return {"obs": obs, "map": map_read, "state_read": state_read, "state_write": state_write,
            "per_step": per_step, "per_launch_once": once, "steps_per_launch": T,
            "total": per_step + once / T}


def _kernel_source_digest(text: str | None = None) -> str:
    """sha256 (first 16 hex digits) of the kernel source's code, with comments
    removed and white space collapsed: a comment edit keeps the digest, any
    code edit changes it."""
    import hashlib
    import re
    if text is None:
        with open(os.path.join(ROOT, "paper_2605_19926_amd", "csrc", "jx_kernels.hip")) as f:
            text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256(" ".join(text.split()).encode()).hexdigest()[:16]


def measured_traffic(form: str, digest: str):
    """HBM bytes per env-step of the headline kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or
    None when there is none for this form or the kernel source has changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{form}_scale.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256_16") != digest:
        return None
    try:
        return float(vals["hbm_bytes_per_env_step"])
    except (KeyError, ValueError):
        return None


def store_pattern_ceilings():
    """GB/s that constant-data store patterns reach on this device (the
    library's jx_store_ceiling program, run in its own process): the fastest
    linear fill pattern, and the renderer's own pattern of one frame per wave
    and step at 64x64 and at 84x84.  None if the program is missing or fails."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2605_19926_amd", "jx_store_ceiling")
    if not os.path.exists(exe):
        return None
    try:
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    except subprocess.TimeoutExpired:
        return None
    if r.returncode != 0:
        progress(f"store ceiling calibration failed: {r.stderr.strip()[-200:]}")
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def _oracle_chunk(args):
    cfg_d, seeds, acts = args
    import oracle
    c = oracle.make_cfg(cfg_d)
    done, _, counts = oracle.rollout(c, seeds, acts, counts=True)
    return done, counts


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl: dict, tiny: dict, envs_per_worker: int = 64, cpu_seconds: float = 18.0) -> dict:
    """The oracle as it stands, on the host cores: the tiny workload in full
    (16 envs x 1000 steps) and a sample of the headline workload on one pinned
    core, then the headline sample split over every core of this process's
    affinity set (about `cpu_seconds` of CPU work in all).  The oracle's own
    column flags over the sample give the flagged fractions of the workload."""
    import oracle
    oracle.build()
    cfg = wl["cfg"]
    cores = sorted(os.sched_getaffinity(0))
    n_workers = len(cores)
    prev = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {cores[0]})
    try:
        # the tiny workload in full, one core
        tn, ts = tiny["n_envs"], tiny["steps"]
        t0 = time.perf_counter()
        tdone, _ = _oracle_chunk((tiny["cfg"], W.seeds(tiny["number"], tn),
                                  W.actions(tiny["number"], ts, tn, tiny["cfg"]["n_actions"])))
        dt_tiny = time.perf_counter() - t0
        # a one-core sample of the headline workload (also sizes the all-core sample)
        probe_steps = 300
        seeds1 = W.seeds(wl["number"], envs_per_worker)
        acts1 = W.actions(wl["number"], probe_steps, envs_per_worker, cfg["n_actions"])
        t0 = time.perf_counter()
        one, _ = _oracle_chunk((cfg, seeds1, acts1))
        dt1 = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, prev)
    one_core = one / dt1
    steps = max(100, int(cpu_seconds * one_core / (n_workers * envs_per_worker)))
    seeds = W.seeds(wl["number"], envs_per_worker * n_workers)
    acts = W.actions(wl["number"], steps, envs_per_worker * n_workers, cfg["n_actions"])
    chunks = [(cfg, seeds[k * envs_per_worker:(k + 1) * envs_per_worker],
               np.ascontiguousarray(acts[:, k * envs_per_worker:(k + 1) * envs_per_worker]))
              for k in range(n_workers)]
    # one host thread per core of the affinity set: the oracle runs each chunk
    # in one C call (ctypes releases the interpreter lock, and the oracle keeps
    # no mutable global state), so the threads run in parallel and no helper
    # process outlives the bench
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=n_workers) as pool:
        list(pool.map(_oracle_chunk, chunks[:1]))    # library load outside the timing
        t0 = time.perf_counter()
        res = list(pool.map(_oracle_chunk, chunks))
        dtn = time.perf_counter() - t0
    tot = sum(r[0] for r in res)
    cnt = {k: sum(r[1][k] for r in res) for k in res[0][1]}
    flags = {"columns": cnt["columns"], "flagged_frac": cnt["flagged"] / max(1, cnt["columns"]),
             "f1_frac": cnt["f1"] / max(1, cnt["columns"]),
             "steps_flagged_frac": cnt["steps_flagged"] / max(1, tot),
             "sample": f"the oracle's own trajectories of {n_workers * envs_per_worker} envs x "
                       f"{steps} steps of {wl['name']}"}
    return {"value": tot / dtn, "unit": "env-steps/s", "cores": n_workers, "kind": "oracle",
            "sample": (f"{wl['name']}: {envs_per_worker} envs x {steps} steps per thread, one thread on each of "
                       f"{n_workers} cores (step + full render, FP64 C oracle, gcc -O2); one pinned "
                       f"core: {one_core:.0f} env-steps/s ({envs_per_worker} envs x {probe_steps} "
                       f"steps); {tiny['name']} in full on one core: {tdone / dt_tiny:.0f} "
                       f"env-steps/s; cpu: {_cpu_model()}"),
            "one_core": one_core, "tiny_one_core": tdone / dt_tiny, "flags": flags}


def batch_form(jx, torch, launches: list[dict], rollouts: int = 2) -> dict:
    """Mixed-shape batch (16384 envs: map side {8,16,32,64}, frames {32,64,128}
    square, key-door on half) stepped by 128-step hipGraph rollouts; env-steps/s
    per launch mapping, the given ones and the one the library's autotuner picks
    (every candidate checked bit-identical to the default mapping)."""
    n, T = W.BATCH["n_envs"], W.BATCH["rollout"]
    cfgs, idx = W.batch_cfgs(n)
    env = jx.Env(W.seeds(W.BATCH["number"], n), cfgs, idx)
    env.reset()
    ob = env.obs_bytes
    obs = torch.empty(T * ob, dtype=torch.uint8, device=env.dev)
    rew = torch.empty(T * n, dtype=torch.float32, device=env.dev)
    done = torch.empty(T * n, dtype=torch.uint8, device=env.dev)
    acts = torch.from_numpy(W.actions(W.BATCH["number"], T, n, 6)).to(env.dev)
    out = {"workload": W.BATCH["name"], "n_envs": n, "rollout": T,
           "obs_bytes_per_step": ob, "results": []}
    for launch in list(launches) + ["autotune"]:
        tuned = launch == "autotune"
        if tuned:
            launch = env.autotune(acts, 16, obs[:ob])
        launch = dict(launch)
        fused = launch.pop("fused", False)
        env.set_launch(**launch)
        env.rollout(acts, obs, rew, done, T, obs_stride=ob, graph=not fused, fused=fused)  # warm
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(rollouts):
            env.rollout(acts, obs, rew, done, T, obs_stride=ob, graph=not fused, fused=fused)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        steps = rollouts * T
        out["results"].append({"launch": launch, "rollout": "fused" if fused else "graph",
                               "autotuned": tuned,
                               "env_steps_per_s": n * steps / sec,
                               "ms_per_step": sec / steps * 1e3,
                               "obs_gbs": ob * steps / sec / 1e9})
    env.close()
    return out


def serve_form(jx, n_requests: int, mode: int, rate: float = W.SERVE["rate"],
               budget: int = int(64e9), n_streams: int = 4, device_results: bool = False) -> dict:
    """Serving workload: Poisson arrivals over 256 client slots, clients of
    1-512 envs (log-uniform), side 8-64, frames 64 or 84 square.  Every client is
    opened before the clock starts (with a tight budget most of them queue for
    admission).  The library's native load generator (jx_server_replay) submits
    each request at its trace time, closes a client right after its last
    request, and collects completed requests in completion order from four
    threads, copying their frames, rewards and dones to host memory (or, with
    device_results, leaving them in each client's device rings of two slots,
    as a learner on the same GPU would read them).  Latency is submit-to-ready
    as measured by the server."""
    tr = W.serve_trace(n_requests, rate=rate)
    srv = jx.Server(hbm_budget=budget, n_streams=n_streams, mode=mode)
    sessions = {}
    ring_keep = []   # device result rings, alive until the server is closed
    last_of = {}
    for k, sid in enumerate(tr["session"]):
        last_of[int(sid)] = k
    queued = 0
    for k in range(n_requests):
        sid = int(tr["session"][k])
        if sid not in sessions:
            n = int(tr["n_envs"][sid])
            side = int(tr["side"][sid])
            ob = int(tr["obs"][sid])
            cfg = W.env_cfg(side=side, loop_frac=0.1, goal_sprite=1, obs_h=ob, obs_w=ob)
            seeds = tr["seed_base"][sid] + np.arange(n, dtype=np.uint64)
            if device_results:
                import torch
                rings = (torch.empty(2 * n * ob * ob * 3, dtype=torch.uint8, device="cuda"),
                         torch.empty(2 * n, dtype=torch.float32, device="cuda"),
                         torch.empty(2 * n, dtype=torch.uint8, device="cuda"))
                ring_keep.append(rings)
                cid, admitted = srv.open_dev(seeds, cfg, *rings, slots=2)
            else:
                cid, admitted = srv.open(seeds, cfg)
            queued += 0 if admitted else 1
            sessions[sid] = (cid, n)
    # everything the replay needs is prepared before the clock
    rng = np.random.default_rng(11)
    cids = np.array([sessions[int(s)][0] for s in tr["session"]], np.int32)
    acts = [rng.integers(0, 6, size=sessions[int(s)][1], dtype=np.uint8) for s in tr["session"]]
    close_after = np.array([last_of[int(s)] == k for k, s in enumerate(tr["session"])], np.uint8)
    lat, t_submitted, wall = srv.replay(tr["t"], cids, acts, close_after, n_collectors=4, timeout=600.0)
    progress(f"serving {'coalesced' if mode == jx.JX_SERVE_COALESCE else 'plain'} "
             f"rate {rate:g}/s budget {budget}{' device results' if device_results else ''} done")
    st = srv.stats()
    srv.close()
    lat_ms = lat * 1e3
    env_steps = int(sum(sessions[int(s)][1] for s in tr["session"]))
    del ring_keep
    return {"mode": "coalesced" if mode == jx.JX_SERVE_COALESCE else "plain-per-request",
            "results": "device rings" if device_results else "host copies",
            "driver": "native replay (jx_server_replay), 4 collector threads",
            "streams": n_streams if mode == jx.JX_SERVE_COALESCE else 1,
            "offered_req_per_s": rate, "submitted_req_per_s": n_requests / t_submitted,
            "hbm_budget_bytes": budget,
            "requests": n_requests, "clients": len(sessions),
            "clients_queued_for_admission": queued,
            "p50_ms": float(np.percentile(lat_ms, 50)),
            "p99_ms": float(np.percentile(lat_ms, 99)), "mean_ms": float(lat_ms.mean()),
            "env_steps_per_s": env_steps / wall, "launches": int(st["launches"]),
            "wall_s": wall}


def shape_sweep(jx, torch) -> list[dict]:
    """Fused 128-step rollouts of one configuration (16x16 mazes) over frame
    size x env count, under the static-stride and persistent mappings with one
    wave per env and the static stride with 2 or 4 waves per env: how many envs
    one wave per env needs before the frame writes saturate, and what several
    waves per env give below that."""
    T = 128
    out = []
    for side_px in (32, 64, 128):
        for n in (256, 512, 1024, 2048, 4096, 8192, 16384):
            cfg = W.env_cfg(side=16, loop_frac=0.1, goal_sprite=1, obs_h=side_px, obs_w=side_px,
                            n_actions=6, episode_cap=512)
            env = jx.Env(W.seeds(3, n), cfg)
            env.reset()
            ob = env.obs_bytes
            o = torch.empty(T * ob, dtype=torch.uint8, device=env.dev)
            rew = torch.empty(T * n, dtype=torch.float32, device=env.dev)
            dn = torch.empty(T * n, dtype=torch.uint8, device=env.dev)
            acts = torch.from_numpy(W.actions(3, T, n, 6)).to(env.dev)
            for launch in (dict(form=0, waves_per_group=4, groups_per_cu=1, store_mode=0),
                           dict(form=0, waves_per_group=8, groups_per_cu=1, store_mode=0),
                           dict(form=1, waves_per_group=4, groups_per_cu=2, store_mode=0),
                           dict(form=0, waves_per_group=8, groups_per_cu=1, store_mode=0, waves_per_env=2),
                           dict(form=0, waves_per_group=8, groups_per_cu=1, store_mode=0, waves_per_env=4)):
                env.set_launch(**launch)
                env.rollout(acts, o, rew, dn, T, obs_stride=ob, graph=False, fused=True)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(3):
                    env.rollout(acts, o, rew, dn, T, obs_stride=ob, graph=False, fused=True)
                e1.record()
                torch.cuda.synchronize()
                sec = e0.elapsed_time(e1) / 1e3
                out.append({"frame": f"{side_px}x{side_px}", "n_envs": n, "launch": launch,
                            "env_steps_per_s": n * T * 3 / sec, "obs_gbs": ob * T * 3 / sec / 1e9})
            env.close()
            del o
        progress(f"shape sweep {side_px}x{side_px} done")
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10_240)
    ap.add_argument("--warmup", type=int, default=128)
    ap.add_argument("--form", choices=["fused", "graph", "eager", "persistent", "pipeline"],
                    default="fused")
    ap.add_argument("--waves", type=int, default=0, help="waves per workgroup (0: the form's default)")
    ap.add_argument("--groups", type=int, default=4, help="persistent form: workgroups per CU")
    ap.add_argument("--store", type=int, default=-1, help="0 normal, 1 non-temporal (-1: default)")
    ap.add_argument("--single-slot", action="store_true", help="write every frame to one slot")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batching and serving forms")
    ap.add_argument("--serve-requests", type=int, default=20_000)
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--shape-sweep", action="store_true",
                    help="only time fused rollouts over frame size x env count and print them")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 launches), to scale "
                         "HBM traffic counters, and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the envs are "
              "independent, so a multi-GPU job would give each GPU its own env range, "
              "workspace and stream, and exchange nothing per step", file=sys.stderr)
        return 2

    import torch
    from paper_2605_19926_amd import jx

    if args.calib_copy_mib:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb, "launches": 5}))
        return 0

    if args.shape_sweep:
        print(json.dumps({"shape_sweep": shape_sweep(jx, torch)}))
        return 0

    wl = W.SCALE
    cfg, n = wl["cfg"], wl["n_envs"]
    K, Wu = args.steps, args.warmup
    seeds = W.seeds(wl["number"], n)
    env = jx.Env(seeds, cfg)
    env.reset()
    ob = env.obs_bytes
    slots = 1 if args.single_slot else RING
    obs = torch.empty(slots * ob, dtype=torch.uint8, device=env.dev)
    env.reset(obs[:ob])
    # Episode clocks staggered (env i starts at t = i mod cap): the envs then
    # reach the cap evenly, n / cap of them reset in every step, as in the
    # steady state of a long run, so resets fall inside the timed steps at any
    # step count.
    cap = cfg["episode_cap"]
    env.set_state({"t": (np.arange(n) % cap).astype(np.uint32)})
    acts = torch.from_numpy(W.actions(wl["number"], Wu + K, n, cfg["n_actions"])).to(env.dev)
    rew = torch.empty(RING * n, dtype=torch.float32, device=env.dev)
    done = torch.empty(RING * n, dtype=torch.uint8, device=env.dev)
    launch = {"form": {"persistent": jx.JX_FORM_PERSISTENT,
                       "pipeline": jx.JX_FORM_PIPELINE}.get(args.form, jx.JX_FORM_PLAIN),
              "waves_per_group": args.waves or {"persistent": 2, "fused": 8}.get(args.form, 4),
              "groups_per_cu": args.groups, "store_mode": max(args.store, 0)}
    env.set_launch(**launch)
    if args.autotune:
        launch = env.autotune(acts, 20, obs[:ob])
    def plan(first: int, count: int):
        t, end, out = first, first + count, []
        while t < end:
            slot = t % RING
            chunk = min(RING - slot, end - t)
            out.append((t, slot, chunk))
            t += chunk
        return out

    def run(first: int, count: int):
        for t, slot, chunk in plan(first, count):
            if args.form == "eager":
                for k in range(chunk):
                    s = slot + k
                    o = obs[s * ob:(s + 1) * ob] if slots > 1 else obs
                    env.step(acts[t + k], o, rew[s * n:(s + 1) * n], done[s * n:(s + 1) * n])
            else:
                o = obs[slot * ob:] if slots > 1 else obs
                env.rollout(acts[t:t + chunk], o, rew[slot * n:], done[slot * n:], chunk,
                            obs_stride=ob if slots > 1 else 0, graph=args.form != "fused",
                            fused=args.form == "fused")

    # capture every graph length the timed region will use before timing
    if args.form not in ("eager", "fused"):
        for T in sorted({c for _, _, c in plan(Wu, K)}):
            env.rollout(acts[:T], obs, rew, done, T, obs_stride=ob if slots > 1 else 0, graph=True)
    run(0, Wu)
    torch.cuda.synchronize()
    ep_before = int(env.get_state()["episode"].astype(np.int64).sum())
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    run(Wu, K)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1)
    episodes_timed = int(env.get_state()["episode"].astype(np.int64).sum()) - ep_before
    sec = ms / 1e3
    rate = n * K / sec
    # The fused form runs one kernel per ring chunk (up to 128 steps); the
    # other forms run one kernel per step.  Layout and state move once per
    # launch, frames, actions, rewards and dones once per step.
    chunks = plan(Wu, K)
    launches = len(chunks) if args.form == "fused" else K
    ab = algorithmic_bytes(cfg, K // launches)
    total_bytes = n * (K * ab["per_step"] + launches * ab["per_launch_once"])
    per_launch = total_bytes / launches
    bytes_per_env_step = total_bytes / (n * K)
    kern_s = sec / launches  # average launch duration over the timed region
    achieved = per_launch / kern_s / 1e9
    tr = measured_traffic(args.form, _kernel_source_digest())
    traffic = None if tr is None else tr * n * K / launches
    # store-pattern ceilings on this machine: constant-data store patterns timed by
    # the library's calibration program (its own process and buffer)
    pattern_ceilings = store_pattern_ceilings()
    # write-only ceiling on this machine: a plain fill of the whole frame ring
    fills = 3
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    obs.fill_(1)
    f0.record(stream)
    for _ in range(fills):
        obs.fill_(0)
    f1.record(stream)
    torch.cuda.synchronize()
    write_ceiling = obs.numel() * fills / (f0.elapsed_time(f1) / 1e3) / 1e9
    # single-slot variant (every frame to slot 0: the last-level cache can
    # absorb the frame writes), same form, fewer steps
    single = None
    if slots > 1 and args.form in ("fused", "graph"):
        Ks = min(K, 1024)
        o0 = obs[:ob]
        c0 = min(128, Ks)
        env.rollout(acts[:c0], o0, rew, done, c0, obs_stride=0, graph=args.form == "graph",
                    fused=args.form == "fused")
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for t in range(0, Ks, 128):
            c = min(128, Ks - t)
            env.rollout(acts[t:t + c], o0, rew, done, c, obs_stride=0,
                        graph=args.form == "graph", fused=args.form == "fused")
        s1.record(stream)
        torch.cuda.synchronize()
        ss = s0.elapsed_time(s1) / 1e3
        single = {"steps": Ks, "env_steps_per_s": n * Ks / ss, "ms_per_step": ss / Ks * 1e3}
    def variant_rate(vcfg, vseeds, name):
        """Fused 128-step rollouts of a variant configuration into the same
        frame ring (same frame size), timed like the headline."""
        venv = jx.Env(vseeds, vcfg)
        venv.reset(obs[:ob])
        venv.set_launch(**launch)   # the headline's mapping
        Kv = min(K, 2560)

        def vrun(first, count):
            for t, slot, chunk in plan(first, count):
                venv.rollout(acts[t:t + chunk], obs[slot * ob:], rew[slot * n:], done[slot * n:],
                             chunk, obs_stride=ob, graph=False, fused=True)
        vrun(0, Wu)
        torch.cuda.synchronize()
        v0, v1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        v0.record(stream)
        vrun(Wu, Kv)
        v1.record(stream)
        torch.cuda.synchronize()
        vs = v0.elapsed_time(v1) / 1e3
        venv.close()
        progress(f"{name}: {n * Kv / vs:.4g} env-steps/s")
        return {"steps": Kv, "env_steps_per_s": n * Kv / vs, "ms_per_step": vs / Kv * 1e3}

    def buffer_rate(layout, dtype):
        """Fused 128-step rollouts writing a learner's rollout buffer in a
        training format (frames [128][n][frame], previous actions beside),
        the buffer reused by every rollout, same workload; one 128-step window
        of actions serves every rollout."""
        bcfg = dict(cfg, obs_layout=layout, obs_dtype=dtype)
        benv = jx.Env(seeds, bcfg)
        benv.reset()
        fb = benv.obs_bytes
        T = 128
        dev = benv.dev
        bacts = torch.from_numpy(W.actions(wl["number"] + 100, T, n, cfg["n_actions"])).to(dev)
        buf = torch.empty(T * fb, dtype=torch.uint8, device=dev)
        brew = torch.empty(T * n, dtype=torch.float32, device=dev)
        bdone = torch.empty(T * n, dtype=torch.uint8, device=dev)
        bprev = torch.empty(T * n, dtype=torch.uint8, device=dev)
        Kb = max(T, min(K, 1280) // T * T)

        def brun(first, count):
            for _ in range(first, first + count, T):
                benv.rollout(bacts, buf, brew, bdone, T, obs_stride=fb, graph=False, fused=True, prev=bprev)
        brun(0, T)
        torch.cuda.synchronize()
        b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        b0.record(stream)
        brun(T, Kb)
        b1.record(stream)
        torch.cuda.synchronize()
        bs = b0.elapsed_time(b1) / 1e3
        benv.close()
        del buf
        r = n * Kb / bs
        name = f"{['NHWC', 'NCHW'][layout]}-{['u8', 'bf16', 'f32'][dtype]}"
        progress(f"training buffer {name}: {r:.4g} env-steps/s")
        return {"format": name, "steps": Kb, "env_steps_per_s": r, "ms_per_step": bs / Kb * 1e3,
                "frame_bytes": fb // n, "obs_gbs": fb * Kb / bs / 1e9,
                "frac_of_hbm_peak": fb * Kb / bs / 1e9 / HBM_PEAK_GBS}

    def keydoor_rate():
        """The key-door workload (8192 envs, 32x32 loop-free mazes with door,
        key, goal and decor sprites, 84x84 frames) in fused 128-step rollouts
        into its own 128-slot ring, with the headline's launch mapping."""
        kwl = W.KEYDOOR
        kn = kwl["n_envs"]
        kenv = jx.Env(W.seeds(kwl["number"], kn), kwl["cfg"])
        kenv.reset()
        kenv.set_launch(**launch)
        kob = kenv.obs_bytes
        T = 128
        dev = kenv.dev
        kacts = torch.from_numpy(W.actions(kwl["number"], T, kn, kwl["cfg"]["n_actions"])).to(dev)
        kobs = torch.empty(T * kob, dtype=torch.uint8, device=dev)
        krew = torch.empty(T * kn, dtype=torch.float32, device=dev)
        kdone = torch.empty(T * kn, dtype=torch.uint8, device=dev)
        launches = 4

        def krun(count):
            for _ in range(count):
                kenv.rollout(kacts, kobs, krew, kdone, T, obs_stride=kob, graph=False, fused=True)
        krun(1)
        torch.cuda.synchronize()
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k0.record(stream)
        krun(launches)
        k1.record(stream)
        torch.cuda.synchronize()
        ks = k0.elapsed_time(k1) / 1e3
        kenv.close()
        del kobs
        r = kn * T * launches / ks
        progress(f"key-door workload: {r:.4g} env-steps/s")
        gbs = kob * T * launches / ks / 1e9
        ceil84 = (pattern_ceilings or {}).get("env_frames_84px_12B")
        return {"workload": kwl["name"], "steps": T * launches, "env_steps_per_s": r,
                "ms_per_step": ks / (T * launches) * 1e3, "frame_bytes": kob // kn,
                "obs_gbs": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS,
                "frac_of_frame_pattern_ceiling": gbs / ceil84 if ceil84 else None}

    shaded = ascii_maps = buffers = keydoor = None
    if args.form == "fused" and slots > 1:
        # distance-shaded walls (render option), same workload
        shaded = dict(shade_levels=8, shade_dist=12.0,
                      **variant_rate(dict(cfg, shade_levels=8, shade_dist=12.0), seeds, "shaded"))
        # the 16x16 ASCII map (Table 2 symbols: keys, locked and unlocked doors,
        # candidates), same env count and frame size
        ascii_maps = dict(workload=W.ASCII["name"],
                          **variant_rate(W.ASCII["cfg"], W.seeds(W.ASCII["number"], n), "ascii"))
        # frames written straight into a learner's rollout buffer (with the
        # previous actions): NCHW float32 and u8, NHWC bfloat16
        buffers = [buffer_rate(1, 2), buffer_rate(0, 1), buffer_rate(1, 0)]
        keydoor = keydoor_rate()
    line = {
        "metric": "rendered env-steps/s @4096 envs 64x64 RGB; served p50/p99 step latency vs plain",
        "value": rate,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wu,
        "ms_per_step": ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u8",
        "data": "synthetic: seeded DFS mazes, uniform random actions",
        "config": {"workload": wl["name"], "n_envs": n, "map_side": cfg["side"],
                   "obs": f"{cfg['obs_h']}x{cfg['obs_w']}x3 uint8", "episode_cap": cfg["episode_cap"],
                   "form": args.form, "launch": launch,
                   "obs_ring_slots": slots, "global_batch": n},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_roll" if args.form == "fused" else
                               {"persistent": "k_persist", "pipeline": "k_pipe"}.get(args.form, "k_plain"),
                     "launches": launches, "steps_per_launch": K / launches,
                     "bytes_per_launch": per_launch,
                     "bytes_per_env_step": bytes_per_env_step, "obs_bytes_per_env_step": ab["obs"],
                     "kernel_avg_us": kern_s * 1e6,
                     "kernel_source_sha256_16": _kernel_source_digest(),
                     "write_only_ceiling_gbs": write_ceiling,
                     "frac_of_write_ceiling": achieved / write_ceiling,
                     "store_pattern_ceilings_gbs": pattern_ceilings,
                     "frac_of_frame_pattern_ceiling": (achieved / pattern_ceilings["env_frames_12B"]
                                                       if pattern_ceilings else None)},
        "single_slot": single,
        "distance_shading": shaded,
        "ascii_maps": ascii_maps,
        "training_buffer": buffers,
        "keydoor_workload": keydoor,
        "obs_write_gbs": ab["obs"] * n * K / sec / 1e9,
        "episodes_completed_in_timed_steps": episodes_timed,
        "episode_clocks": "staggered: env i starts at t = i mod cap",
        "wall_s": wall,
    }
    env.close()
    progress(f"headline {args.form}: {rate:.4g} env-steps/s")
    if not args.no_forms:
        line["batching_form"] = batch_form(jx, torch, [
            {"form": 0, "waves_per_group": 4, "groups_per_cu": 1, "store_mode": 0, "fused": True},
            {"form": 1, "waves_per_group": 4, "groups_per_cu": 2, "store_mode": 0, "fused": True},
            {"form": 1, "waves_per_group": 8, "groups_per_cu": 1, "store_mode": 0, "fused": True},
            {"form": 0, "waves_per_group": 4, "groups_per_cu": 1, "store_mode": 0},
            {"form": 1, "waves_per_group": 2, "groups_per_cu": 4, "store_mode": 0},
            {"form": 2, "waves_per_group": 2, "groups_per_cu": 2, "store_mode": 0}])
        progress("batching form done")
        nr = args.serve_requests
        line["serving_form"] = {
            "workload": W.SERVE["name"],
            "runs": [serve_form(jx, nr, jx.JX_SERVE_COALESCE),
                     serve_form(jx, nr, jx.JX_SERVE_PLAIN),
                     serve_form(jx, nr, jx.JX_SERVE_COALESCE, rate=4 * W.SERVE["rate"]),
                     serve_form(jx, nr, jx.JX_SERVE_PLAIN, rate=4 * W.SERVE["rate"]),
                     serve_form(jx, nr, jx.JX_SERVE_COALESCE, rate=8 * W.SERVE["rate"]),
                     serve_form(jx, nr, jx.JX_SERVE_PLAIN, rate=8 * W.SERVE["rate"]),
                     serve_form(jx, nr, jx.JX_SERVE_COALESCE, rate=16 * W.SERVE["rate"]),
                     serve_form(jx, nr, jx.JX_SERVE_PLAIN, rate=16 * W.SERVE["rate"]),
                     serve_form(jx, nr, jx.JX_SERVE_COALESCE, budget=24 << 20),
                     # results left in device rings (no copy to the host)
                     serve_form(jx, nr, jx.JX_SERVE_COALESCE, device_results=True),
                     serve_form(jx, nr, jx.JX_SERVE_COALESCE, rate=16 * W.SERVE["rate"], device_results=True),
                     serve_form(jx, nr, jx.JX_SERVE_COALESCE, rate=32 * W.SERVE["rate"], device_results=True)]}
        # the metric's second half: served step latency vs the plain per-request
        # launch at the serving workload's own arrival rate
        runs = line["serving_form"]["runs"]
        line["served_latency"] = {"offered_req_per_s": runs[0]["offered_req_per_s"],
                                  "coalesced_p50_ms": runs[0]["p50_ms"], "coalesced_p99_ms": runs[0]["p99_ms"],
                                  "plain_p50_ms": runs[1]["p50_ms"], "plain_p99_ms": runs[1]["p99_ms"],
                                  "coalesced_env_steps_per_s": runs[0]["env_steps_per_s"],
                                  "plain_env_steps_per_s": runs[1]["env_steps_per_s"],
                                  "coalesced_device_rings_p50_ms": runs[9]["p50_ms"],
                                  "coalesced_device_rings_p99_ms": runs[9]["p99_ms"]}
    if not args.no_cpu_baseline:
        progress("cpu baseline (oracle on the host cores)")
        line["cpu_baseline"] = cpu_baseline(wl, W.TINY)
        line["flagged_columns"] = line["cpu_baseline"]["flags"]
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
