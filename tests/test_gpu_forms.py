"""GPU: the batching and serving forms, checkpoint/resume and edge cases.

Every mapping of envs to waves computes each env with the same per-env code,
so the forms must agree with the plain launch on every output byte.  The
mixed-shape batch is also checked against the oracle."""
import threading

import numpy as np
import pytest

import oracle as orc
import workloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _run(env, acts_d, T, mode, torch):
    """T steps in the given launch mode; returns (obs[T], rew[T], done[T], state image)."""
    n, ob = env.n, env.obs_bytes
    obs = torch.zeros(T * ob, dtype=torch.uint8, device=env.dev)
    rew = torch.zeros(T * n, dtype=torch.float32, device=env.dev)
    done = torch.zeros(T * n, dtype=torch.uint8, device=env.dev)
    if mode == "eager":
        for t in range(T):
            env.step(acts_d[t], obs[t * ob:(t + 1) * ob], rew[t * n:(t + 1) * n], done[t * n:(t + 1) * n])
    elif mode == "rollout_eager":
        env.rollout(acts_d, obs, rew, done, T, obs_stride=ob, graph=False)
    elif mode == "fused":
        env.rollout(acts_d, obs, rew, done, T, obs_stride=ob, graph=False, fused=True)
    else:
        env.rollout(acts_d, obs, rew, done, T, obs_stride=ob, graph=True)
    torch.cuda.synchronize()
    return obs.cpu().numpy(), rew.cpu().numpy(), done.cpu().numpy(), env.get_state_bytes()


def _forms_equal(cfgs, seeds, cfg_index, T, launches):
    import torch
    env = U.env_of(cfgs, seeds, cfg_index, obs=False)
    n_act = max(c["n_actions"] for c in (cfgs if isinstance(cfgs, list) else [cfgs]))
    acts = W.actions(9, T, len(seeds), n_act)
    acts_d = torch.from_numpy(acts).to(env.dev)
    snap = env.get_state_bytes()
    ref = None
    for mode, launch in launches:
        env.set_state_bytes(snap)
        env.set_launch(**launch)
        out = _run(env, acts_d, T, mode, torch)
        if ref is None:
            ref = out
            continue
        for k, name in enumerate(("obs", "reward", "done", "state")):
            assert np.array_equal(out[k], ref[k]), f"{mode} {launch}: {name} differs"
    env.close()
    return ref


PLAIN1 = dict(form=0, waves_per_group=1, groups_per_cu=1, store_mode=0)


def test_graph_eager_persistent_identical():
    cfg = W.SCALE["cfg"]
    seeds = W.seeds(W.SCALE["number"], 1024)
    launches = [("eager", PLAIN1),
                ("rollout_eager", dict(form=0, waves_per_group=4, groups_per_cu=1, store_mode=1)),
                ("graph", dict(form=0, waves_per_group=8, groups_per_cu=1, store_mode=0)),
                ("graph", dict(form=1, waves_per_group=2, groups_per_cu=2, store_mode=0)),
                ("graph", dict(form=1, waves_per_group=4, groups_per_cu=8, store_mode=1)),
                ("eager", dict(form=1, waves_per_group=1, groups_per_cu=1, store_mode=0)),
                ("graph", dict(form=2, waves_per_group=1, groups_per_cu=1, store_mode=0)),
                ("eager", dict(form=2, waves_per_group=2, groups_per_cu=2, store_mode=1)),
                ("graph", dict(form=2, waves_per_group=4, groups_per_cu=4, store_mode=0)),
                ("fused", dict(form=0, waves_per_group=4, groups_per_cu=1, store_mode=0)),
                ("fused", dict(form=0, waves_per_group=1, groups_per_cu=1, store_mode=1)),
                # persistent fused rollouts: envs claimed one at a time
                ("fused", dict(form=1, waves_per_group=4, groups_per_cu=2, store_mode=0)),
                ("fused", dict(form=1, waves_per_group=1, groups_per_cu=1, store_mode=1)),
                ("fused", dict(form=1, waves_per_group=8, groups_per_cu=1, store_mode=0)),
                # several waves per env, each writing its share of the frame's rows
                ("eager", dict(form=0, waves_per_group=4, groups_per_cu=1, store_mode=0, waves_per_env=2)),
                ("graph", dict(form=0, waves_per_group=8, groups_per_cu=1, store_mode=1, waves_per_env=4)),
                ("fused", dict(form=0, waves_per_group=4, groups_per_cu=1, store_mode=0, waves_per_env=4)),
                ("fused", dict(form=0, waves_per_group=2, groups_per_cu=1, store_mode=0, waves_per_env=2))]
    _forms_equal(cfg, seeds, None, 40, launches)


def test_ascii_maps_every_form_identical():
    """ASCII maps (doors opened by bumps and keys across episodes) mixed with a
    generated maze in one batch: every launch form gives the same outputs."""
    cfgs = [W.ASCII["cfg"], W.ASCII_TINY["cfg"], dict(W.ASCII_TINY["cfg"], n_actions=6),
            W.env_cfg(side=16, loop_frac=0.1, goal_sprite=1, episode_cap=60)]
    n = 768
    idx = (np.arange(n) * 7 % 4).astype(np.int32)
    seeds = W.seeds(61, n)
    launches = [("eager", PLAIN1),
                ("graph", dict(form=0, waves_per_group=4, groups_per_cu=1, store_mode=0)),
                ("graph", dict(form=1, waves_per_group=2, groups_per_cu=4, store_mode=0)),
                ("graph", dict(form=2, waves_per_group=2, groups_per_cu=2, store_mode=1)),
                ("fused", dict(form=0, waves_per_group=8, groups_per_cu=1, store_mode=0)),
                ("fused", dict(form=1, waves_per_group=2, groups_per_cu=3, store_mode=0))]
    ref = _forms_equal(cfgs, seeds, idx, 150, launches)
    # doors were opened and keys taken along the way
    assert ref[1].max() >= 0.5


def test_fused_rollout_long_and_resets():
    """More than 128 steps (two action windows) across episode ends."""
    cfg = W.env_cfg(side=12, loop_frac=0.1, goal_sprite=1, key_door=1, max_decor=2,
                    episode_cap=37, obs_h=32, obs_w=32)
    seeds = W.seeds(12, 300)
    _forms_equal(cfg, seeds, None, 200, [("eager", PLAIN1),
                                         ("fused", dict(form=0, waves_per_group=8, groups_per_cu=1,
                                                        store_mode=0)),
                                         ("fused", dict(form=1, waves_per_group=4, groups_per_cu=1,
                                                        store_mode=0)),
                                         ("fused", dict(form=0, waves_per_group=4, groups_per_cu=1,
                                                        store_mode=0, waves_per_env=2))])


def test_shaded_fused_rollout_equals_graph_and_differs_from_unshaded():
    """Distance shading through the fused and the graph rollout: bit-identical
    to each other; walls darker than without shading, nothing else changed."""
    import torch
    base = W.env_cfg(side=16, loop_frac=0.1, goal_sprite=1, obs_h=64, obs_w=64, episode_cap=40)
    shaded = dict(base, shade_levels=6, shade_dist=9.0)
    seeds = W.seeds(31, 96)
    acts = W.actions(31, 70, 96, 6)
    out = {}
    for name, cfg, form in (("fused", shaded, "fused"), ("graph", shaded, "graph"),
                            ("plain", base, "fused")):
        env = U.env_of(cfg, seeds, obs=False)
        out[name] = _run(env, torch.from_numpy(acts).to(env.dev), 70, form, torch)
        env.close()
    for k in range(4):
        assert np.array_equal(out["fused"][k], out["graph"][k])
    assert np.array_equal(out["fused"][1], out["plain"][1])      # rewards unchanged
    assert np.array_equal(out["fused"][2], out["plain"][2])      # dones unchanged
    a = out["fused"][0].astype(np.int32)
    b = out["plain"][0].astype(np.int32)
    assert (a <= b).all() and (a < b).any()                      # only darker


def test_graph_replays_agree_with_eager():
    """A captured rollout replayed several times (with eager work and syncs in
    between) equals the same steps launched one by one."""
    import torch
    cfg = W.TINY["cfg"]
    seeds = W.seeds(1, 64)
    T, R = 16, 4
    acts = W.actions(3, T * R, 64, 4)
    env = U.env_of(cfg, seeds, obs=False)
    snap = env.get_state_bytes()
    acts_d = torch.from_numpy(acts).to(env.dev)
    e = [_run(env, acts_d[r * T:(r + 1) * T], T, "eager", torch) for r in range(R)]
    env.set_state_bytes(snap)
    for r in range(R):
        g = _run(env, acts_d[r * T:(r + 1) * T], T, "graph", torch)
        for k in range(4):
            assert np.array_equal(g[k], e[r][k]), f"replay {r} field {k}"
        env.render(torch.zeros(env.obs_bytes, dtype=torch.uint8, device=env.dev))
        torch.cuda.synchronize()
    env.close()


def test_mixed_shapes_batch_identical_and_oracle():
    import torch
    n = 2048
    cfgs, idx = W.batch_cfgs(n)
    seeds = W.seeds(W.BATCH["number"], n)
    launches = [("eager", PLAIN1),
                ("graph", dict(form=1, waves_per_group=2, groups_per_cu=4, store_mode=0)),
                ("graph", dict(form=1, waves_per_group=1, groups_per_cu=8, store_mode=1)),
                ("graph", dict(form=2, waves_per_group=2, groups_per_cu=1, store_mode=0)),
                ("eager", dict(form=2, waves_per_group=4, groups_per_cu=2, store_mode=1)),
                ("fused", dict(form=0, waves_per_group=2, groups_per_cu=1, store_mode=0)),
                ("fused", dict(form=1, waves_per_group=4, groups_per_cu=2, store_mode=0)),
                ("fused", dict(form=1, waves_per_group=2, groups_per_cu=16, store_mode=1)),
                ("fused", dict(form=0, waves_per_group=8, groups_per_cu=1, store_mode=0, waves_per_env=4)),
                ("eager", dict(form=0, waves_per_group=4, groups_per_cu=1, store_mode=0, waves_per_env=2))]
    _forms_equal(cfgs, seeds, idx, 12, launches)
    # oracle parity of the mixed batch from shared states (render + one step)
    env = U.env_of(cfgs, seeds, idx, obs=False)
    env.set_launch(form=1, waves_per_group=2, groups_per_cu=4, store_mode=0)
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(n, 96, replace=False))
    S0 = env.get_state()
    states = [U.gpu_state_dict(S0, i) for i in range(n)]
    grids = {}
    for i in pick:
        c = cfgs[idx[i]]
        grids[int(i)] = U.oracle_maze(c, seeds[i])
        states[int(i)] = U.synth_state(rng, c, seeds[i], grids[int(i)])
    env.set_state(U.gpu_fields(states))
    obs = torch.empty(env.obs_bytes, dtype=torch.uint8, device=env.dev)
    env.render(obs)
    acts = rng.integers(0, 6, size=n).astype(np.uint8)
    obs2 = torch.empty(env.obs_bytes, dtype=torch.uint8, device=env.dev)
    env.step(torch.from_numpy(acts).to(env.dev), obs2)
    torch.cuda.synchronize()
    o1, o2 = obs.cpu().numpy(), obs2.cpu().numpy()
    S = env.get_state()
    rew, done = env.reward.cpu().numpy(), env.done.cpu().numpy()
    stats = U.FrameStats()
    for i in pick:
        i = int(i)
        c = cfgs[idx[i]]
        oc = orc.make_cfg(c)
        U.check_frame(stats, U.frame_of(o1, env.obs_offsets, i, c["obs_h"], c["obs_w"]), grids[i], oc,
                      orc.state_from(states[i]), tag=f"render env {i}")
        g_after = U.gpu_state_dict(S, i)
        skip, errs, o = U.compare_step(states[i], c, seeds[i], grids[i], acts[i],
                                       g_after, rew[i], done[i], S["events"][i])
        assert skip or not errs, (i, errs)
        # the step's frame is the render of the post-step state the GPU stored
        U.check_frame(stats, U.frame_of(o2, env.obs_offsets, i, c["obs_h"], c["obs_w"]), grids[i], oc,
                      orc.state_from(g_after), tag=f"step env {i}")
    stats.report(f"render+one-step/{W.BATCH['name']}-2048")
    assert not stats.mismatch, stats.mismatch[:10]
    assert stats.frac_flagged() < U.FLAG_LIMIT, stats.summary()
    env.close()


def test_autotuned_mapping_is_bit_identical(tmp_path):
    import torch
    cfg = W.SCALE["cfg"]
    seeds = W.seeds(2, 2048)
    env = U.env_of(cfg, seeds, obs=False)
    acts = torch.from_numpy(W.actions(2, 8, 2048, 6)).to(env.dev)
    scratch = torch.empty(env.obs_bytes, dtype=torch.uint8, device=env.dev)
    cache = str(tmp_path / "tune.txt")
    snap = env.get_state_bytes()
    chosen = env.autotune(acts, 8, scratch, cache)
    assert np.array_equal(env.get_state_bytes(), snap)          # state restored
    again = env.autotune(acts, 8, scratch, cache)               # cache hit
    assert again == chosen
    env.close()
    _forms_equal(cfg, seeds, None, 8, [("eager", PLAIN1), ("graph", chosen)])


def test_checkpoint_resume_bit_identical():
    import torch
    cfg = W.KEYDOOR["cfg"]
    seeds = W.seeds(3, 256)
    acts = torch.from_numpy(W.actions(3, 150, 256, 6))
    a = U.env_of(cfg, seeds, obs=False)
    acts_d = acts.to(a.dev)
    _run(a, acts_d[:100], 100, "graph", torch)
    image = a.get_state_bytes()
    ra = _run(a, acts_d[100:], 50, "eager", torch)
    b = U.env_of(cfg, seeds, obs=False)           # fresh context
    b.set_state_bytes(image)
    rb = _run(b, acts_d[100:], 50, "graph", torch)
    for k in range(4):
        assert np.array_equal(ra[k], rb[k])
    a.close()
    b.close()


def test_edge_cases():
    import torch
    from paper_2605_19926_amd import jx
    cfg = W.TINY["cfg"]
    # step before reset
    e = jx.Env(W.seeds(1, 4), cfg)
    with pytest.raises(jx.JxError) as err:
        e.step(torch.zeros(4, dtype=torch.uint8, device="cuda"),
               torch.zeros(4 * 64 * 64 * 3, dtype=torch.uint8, device="cuda"),
               torch.zeros(4, device="cuda"), torch.zeros(4, dtype=torch.uint8, device="cuda"))
    assert err.value.code == jx.JX_ESTATE
    e.reset()
    # misaligned frame buffer
    buf = torch.zeros(4 * 64 * 64 * 3 + 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(jx.JxError):
        e.step(torch.zeros(4, dtype=torch.uint8, device="cuda"), buf[1:])
    # buffers too small for the launch are refused before anything is enqueued
    a8 = torch.zeros(8 * 4, dtype=torch.uint8, device="cuda")
    r8 = torch.zeros(8 * 4, device="cuda")
    d8 = torch.zeros(8 * 4, dtype=torch.uint8, device="cuda")
    frames = torch.zeros(8 * e.obs_bytes, dtype=torch.uint8, device="cuda")
    with pytest.raises(jx.JxError):
        e.rollout(a8[:-1], frames, r8, d8, 8, obs_stride=e.obs_bytes)
    with pytest.raises(jx.JxError):
        e.rollout(a8, frames[:-1], r8, d8, 8, obs_stride=e.obs_bytes)
    with pytest.raises(jx.JxError):
        e.rollout(a8, frames, r8[:-1], d8, 8, obs_stride=e.obs_bytes, fused=True, graph=False)
    with pytest.raises(jx.JxError):
        e.step(a8[:3], frames)
    with pytest.raises(jx.JxError):
        e.step(a8[:4], frames[:e.obs_bytes - 1])
    # out-of-range state values are refused on the host
    S = e.get_state()
    bad = {"goal": np.array([64, 0, 0, 0], np.int32)}
    with pytest.raises(jx.JxError):
        e.set_state(bad)
    with pytest.raises(jx.JxError):
        e.set_state({"x": np.array([np.nan, 1.5, 1.5, 1.5], np.float32)})
    # a map whose border does not block is refused (the walks rely on it)
    lay = e.state_layout()
    img = e.get_state_bytes()
    off = lay["maps"][0] + int(S["map_offset"][2])
    img[off + 3] = 0                                        # row 0 of env 2's map
    with pytest.raises(jx.JxError):
        e.set_state_bytes(img)
    e.close()
    # zero envs: every call is a no-op
    z = jx.Env(np.zeros(0, np.uint64), cfg)
    z.reset()
    assert z.obs_bytes == 0
    z.step(torch.zeros(1, dtype=torch.uint8, device="cuda"), torch.zeros(4, dtype=torch.uint8, device="cuda"))
    z.sync()
    z.close()


def _serve_run(srv, cid, acts, want_obs=True):
    out = []
    for t in range(acts.shape[0]):
        tk = srv.submit(cid, acts[t])
        out.append(srv.wait(cid, tk, want_obs=want_obs))
    return out


def test_serving_alone_equals_mix_equals_plain():
    import torch
    from paper_2605_19926_amd import jx
    cfg = W.env_cfg(side=24, loop_frac=0.1, goal_sprite=1, obs_h=64, obs_w=64, episode_cap=20)
    seeds = W.seeds(5, 37)
    T = 30
    acts = W.actions(5, T, 37, 6)
    # plain path
    env = U.env_of(cfg, seeds, obs=False)
    plain = _run(env, torch.from_numpy(acts).to(env.dev), T, "eager", torch)
    env.close()
    # an ASCII-map client (keys, doors, candidates) in the same mix
    acfg = W.ASCII_TINY["cfg"]
    aseeds = W.seeds(7, 16)
    aacts = W.actions(7, T, 16, acfg["n_actions"])
    env = U.env_of(acfg, aseeds, obs=False)
    aplain = _run(env, torch.from_numpy(aacts).to(env.dev), T, "eager", torch)
    env.close()
    # served alone
    srv = jx.Server(hbm_budget=1 << 30, n_streams=4)
    cid, ok = srv.open(seeds, cfg)
    assert ok
    alone = _serve_run(srv, cid, acts)
    srv.close()
    # served in a mix of concurrent clients of other shapes
    srv = jx.Server(hbm_budget=1 << 30, n_streams=4)
    cid, ok = srv.open(seeds, cfg)
    others = []
    for k in range(6):
        c2 = W.env_cfg(side=8 + 9 * k, loop_frac=0.1, key_door=k % 2, goal_sprite=1,
                       max_decor=2 * (k % 2), obs_h=84 if k % 2 else 64, obs_w=84 if k % 2 else 64)
        s2 = W.seeds(50 + k, 1 + 40 * k)
        o, _ = srv.open(s2, c2)
        others.append((o, W.actions(60 + k, T, len(s2), 6)))
    results = {}
    acid, _ = srv.open(aseeds, acfg)

    def client(o, a):
        results[o] = _serve_run(srv, o, a, want_obs=False)

    def ascii_client():
        results["ascii"] = _serve_run(srv, acid, aacts)

    th = [threading.Thread(target=client, args=oa) for oa in others] + [threading.Thread(target=ascii_client)]
    for t_ in th:
        t_.start()
    mix = _serve_run(srv, cid, acts)
    for t_ in th:
        t_.join()
    st = srv.stats()
    srv.close()
    n, ob1 = 37, 64 * 64 * 3
    for t in range(T):
        p_obs = plain[0][t * n * ob1:(t + 1) * n * ob1].reshape(n, ob1)
        for res in (alone[t], mix[t]):
            assert np.array_equal(res[0], p_obs), f"step {t}: frames differ"
            assert np.array_equal(res[1], plain[1][t * n:(t + 1) * n])
            assert np.array_equal(res[2], plain[2][t * n:(t + 1) * n])
    ob2 = acfg["obs_h"] * acfg["obs_w"] * 3
    for t in range(T):
        res = results["ascii"][t]
        assert np.array_equal(res[0], aplain[0][t * 16 * ob2:(t + 1) * 16 * ob2].reshape(16, ob2)), f"ascii step {t}"
        assert np.array_equal(res[1], aplain[1][t * 16:(t + 1) * 16])
        assert np.array_equal(res[2], aplain[2][t * 16:(t + 1) * 16])
    assert st["requests"] >= T * 8
    assert st["launches"] < st["requests"]          # requests were coalesced
    assert all(len(v) == T for v in results.values())


def _alone_digests(cfg, seeds, acts, frames=True, check_envs=()):
    """A client stepped alone by plain per-step launches: per request its
    rewards, dones and (if frames) the sha256 of its frames.  For the envs in
    check_envs every step is also checked against the oracle from the shared
    state (the GPU's stored state before and after the step)."""
    import hashlib
    import torch
    env = U.env_of(cfg, seeds, obs=False)
    obs = torch.empty(env.obs_bytes, dtype=torch.uint8, device=env.dev)
    oc = orc.make_cfg(cfg)
    grids = {i: U.oracle_maze(cfg, seeds[i]) for i in check_envs}
    stats, errors, skipped = U.FrameStats(), [], 0
    out = []
    for k, a in enumerate(acts):
        before = env.get_state() if check_envs else None
        env.step(torch.from_numpy(a).to(env.dev), obs)
        torch.cuda.synchronize()
        rew, done = env.reward.cpu().numpy().copy(), env.done.cpu().numpy().copy()
        o = obs.cpu().numpy() if frames or check_envs else None
        out.append((hashlib.sha256(o.tobytes()).hexdigest() if frames else None, rew, done))
        if check_envs:
            S = env.get_state()
            for i in check_envs:
                g_after = U.gpu_state_dict(S, i)
                skip, errs, _ = U.compare_step(U.gpu_state_dict(before, i), cfg, seeds[i], grids[i], a[i],
                                               g_after, rew[i], done[i], S["events"][i])
                skipped += int(skip)
                errors += [f"step {k} env {i}: {e}" for e in errs]
                g = U.frame_of(o, env.obs_offsets, i, cfg["obs_h"], cfg["obs_w"])
                U.check_frame(stats, g, grids[i], oc, orc.state_from(g_after), tag=f"step {k} env {i}")
    env.close()
    return out, stats, errors, skipped


def _serve_trace_check(n_requests, clients, rate, mean_session, budget, variants, frame_every):
    """Serves a trace of the serving recipe and compares every request with
    the same client stepped alone.

    Poisson arrivals at `rate` over `clients` slots with session churn (mean
    `mean_session` requests), clients of 1-512 envs (log-uniform), map sides
    8-64 and 64² or 84² frames (the recipe's configuration: loops 0.1, goal
    billboard); with `variants` every fourth client also has the key, door and
    decor sprites and every third a 4-step episode cap.  Every third client
    leaves its results in device rings.  All clients are opened first (those
    beyond the HBM budget wait for admission), each request is submitted at
    its arrival time, each client is closed right after its last request, and
    a collector thread takes requests in completion order.  Rewards and dones
    of every request, and the frames of every request of every
    `frame_every`-th client, must equal those of the client stepped alone by
    plain per-step launches; on sampled envs of three clients every step of
    that reference is checked against the oracle."""
    import hashlib
    import time
    import torch
    from paper_2605_19926_amd import jx
    tr = W.serve_trace(n_requests, clients=clients, rate=rate, mean_session=mean_session)
    sids = list(dict.fromkeys(int(s) for s in tr["session"]))
    count = {s: int((tr["session"] == s).sum()) for s in sids}
    rng = np.random.default_rng(23)
    cfgs, seeds, acts = {}, {}, {s: [] for s in sids}
    for s in sids:
        ob = int(tr["obs"][s])
        kd = variants and s % 4 == 1
        cfgs[s] = W.env_cfg(side=int(tr["side"][s]), loop_frac=0.1, goal_sprite=1, key_door=int(kd),
                            max_decor=2 if kd else 0, obs_h=ob, obs_w=ob,
                            episode_cap=4 if variants and s % 3 == 2 else 512)
        seeds[s] = tr["seed_base"][s] + np.arange(int(tr["n_envs"][s]), dtype=np.uint64)
    for s in tr["session"]:
        s = int(s)
        acts[s].append(rng.integers(0, 6, size=len(seeds[s]), dtype=np.uint8))
    dev = {s for s in sids if s % 3 == 0}
    framed = {s for k, s in enumerate(sids) if k % frame_every == 0}
    # served
    srv = jx.Server(hbm_budget=budget, n_streams=4)
    cid, rings, queued = {}, {}, 0
    for s in sids:
        n, fb = len(seeds[s]), cfgs[s]["obs_h"] * cfgs[s]["obs_w"] * 3
        if s in dev:
            rings[s] = (torch.zeros(count[s] * n * fb, dtype=torch.uint8, device="cuda"),
                        torch.zeros(count[s] * n, dtype=torch.float32, device="cuda"),
                        torch.zeros(count[s] * n, dtype=torch.uint8, device="cuda"))
            cid[s], ok = srv.open_dev(seeds[s], cfgs[s], *rings[s], slots=count[s])
        else:
            cid[s], ok = srv.open(seeds[s], cfgs[s])
        queued += int(not ok)
    sid_of = {c: s for s, c in cid.items()}
    got, failures = {}, []

    def collect():
        try:
            for _ in range(len(tr["session"])):
                r = srv.wait_any(timeout=120.0)
                if r is None:
                    failures.append("a request did not complete")
                    return
                c, tk = r
                want = sid_of[c] in framed
                res = srv.wait(c, tk, want_obs=want)
                got[tk] = None if res[1] is None else \
                    (hashlib.sha256(res[0].tobytes()).hexdigest() if want else None, res[1], res[2])
        except jx.JxError as e:
            failures.append(str(e))

    col = threading.Thread(target=collect)
    col.start()
    ticket, seen = [], {s: 0 for s in sids}
    t0 = time.perf_counter()
    for k, s in enumerate(tr["session"]):
        s = int(s)
        while time.perf_counter() - t0 < tr["t"][k]:
            pass
        ticket.append(srv.submit(cid[s], acts[s][seen[s]]))
        seen[s] += 1
        if seen[s] == count[s]:
            srv.close_client(cid[s])
    col.join()
    st = srv.stats()
    srv.close()
    assert not failures, failures
    assert st["requests"] == len(tr["session"]) and st["failed_launches"] == 0
    # every client alone, in the order of its requests
    checked = {sids[0], max(sids, key=lambda s: cfgs[s]["side"]),
               next(s for s in sids if cfgs[s]["key_door"]) if variants else sids[1]}
    stats = U.FrameStats()
    ref = {}
    for s in sids:
        pick = tuple(range(min(len(seeds[s]), 6))) if s in checked else ()
        ref[s], st_s, errs, skipped = _alone_digests(cfgs[s], seeds[s], acts[s], s in framed, pick)
        assert not errs, errs[:10]
        assert skipped <= 2, f"client {s}: {skipped} flagged steps"
        stats.cols += st_s.cols
        stats.flagged += st_s.flagged
        stats.mismatch += st_s.mismatch
    assert not stats.mismatch, stats.mismatch[:10]
    assert stats.cols > 0 and stats.frac_flagged() < 10 * U.FLAG_LIMIT, stats.summary()
    k_of = {s: 0 for s in sids}
    n_resets = n_frames = 0
    for k, s in enumerate(tr["session"]):
        s = int(s)
        j = k_of[s]
        k_of[s] += 1
        h, rew, done = ref[s][j]
        n_resets += int(done.sum())
        if s in dev:
            n, fb = len(seeds[s]), cfgs[s]["obs_h"] * cfgs[s]["obs_w"] * 3
            o, r_, d_ = rings[s]
            if h is not None:
                assert hashlib.sha256(o[j * n * fb:(j + 1) * n * fb].cpu().numpy().tobytes()).hexdigest() == h, \
                    f"client {s} request {j}: device-ring frames differ"
            g = (h, r_[j * n:(j + 1) * n].cpu().numpy(), d_[j * n:(j + 1) * n].cpu().numpy())
        else:
            g = got[ticket[k]]
            assert g[0] == h, f"client {s} request {j}: frames differ"
        assert np.array_equal(g[1], rew) and np.array_equal(g[2], done), f"client {s} request {j}"
        n_frames += int(h is not None)
    return st, queued, n_resets, n_frames


def test_serving_trace_equals_each_client_alone():
    """A test-size trace (360 requests at 20,000 req/s over 32 slots, mean
    session 4, with the key-door and short-episode variants) under a 12 MiB
    budget that holds fewer than all clients: every request's frames, rewards
    and dones equal those of its client stepped alone."""
    st, queued, n_resets, n_frames = _serve_trace_check(360, 32, 20000.0, 4, 12 << 20, True, 1)
    assert queued > 0 and st["admission_waits"] > 0
    assert st["launches"] < st["requests"]           # requests were coalesced
    assert n_resets > 0 and n_frames == 360


@pytest.mark.parametrize("rate", [W.SERVE["rate"], 64_000.0], ids=["2000rps", "64000rps"])
def test_serving_workload_full_size(rate):
    """The serving workload at its full size in the configuration the
    benchmark times: 20,000 requests at 2000 req/s (and at 64,000 req/s, the
    benchmark's highest offered load, where launches overlap on every stream)
    over 256 client slots (mean session 64), a 64 GB budget, coalesced
    launches on 4 streams.  Rewards and dones of every request, and every
    request's frames for every eighth client, equal those of the client
    stepped alone."""
    st, queued, n_resets, n_frames = _serve_trace_check(20_000, 256, rate, W.SERVE["mean_session"],
                                                        64 * 10 ** 9, False, 8)
    assert queued == 0 and st["requests"] == 20_000
    assert n_frames > 20_000 // 16


def test_serving_completion_queue():
    """wait_any hands out every completed request once, in completion order,
    and the results collected through it equal those of a plain wait."""
    from paper_2605_19926_amd import jx
    cfg = W.env_cfg(side=16, obs_h=64, obs_w=64)
    got_any, got_plain = {}, {}
    for use_any in (True, False):
        srv = jx.Server(hbm_budget=1 << 30, n_streams=2)
        cids = [srv.open(W.seeds(90 + k, 5 + 7 * k), cfg)[0] for k in range(3)]
        tickets = {}
        for t in range(4):
            for k, cid in enumerate(cids):
                acts = W.actions(95 + k, 4, 5 + 7 * k, 6)[t]
                tickets[srv.submit(cid, acts)] = (k, t)
        out = got_any if use_any else got_plain
        if use_any:
            seen = set()
            for _ in range(len(tickets)):
                cid, tk = srv.wait_any(timeout=30.0)
                assert tk in tickets and tk not in seen
                seen.add(tk)
                out[tickets[tk]] = srv.wait(cid, tk)
            assert srv.wait_any(timeout=0.0) is None
        else:
            for tk, (k, t) in tickets.items():
                out[(k, t)] = srv.wait(cids[k], tk)
        srv.close()
    assert got_any.keys() == got_plain.keys()
    for key in got_any:
        for a, b in zip(got_any[key][:3], got_plain[key][:3]):
            assert np.array_equal(a, b)


def test_serving_native_replay():
    """The native load generator: a dense trace (240 requests over 12 clients at
    20,000 req/s) completes with every latency recorded, and every client's
    requests ran in order: one more request per client afterwards returns the
    same results as a server fed the same requests one by one."""
    from paper_2605_19926_amd import jx
    cfgs = [W.env_cfg(side=8 + 4 * (k % 3), obs_h=32 + 32 * (k % 2), obs_w=32 + 32 * (k % 2))
            for k in range(12)]
    sizes = [1 + 37 * k for k in range(12)]
    rng = np.random.default_rng(3)
    order = rng.integers(0, 12, size=240)
    acts = [rng.integers(0, 6, size=sizes[c], dtype=np.uint8) for c in order]
    finals = [rng.integers(0, 6, size=sizes[c], dtype=np.uint8) for c in range(12)]
    results = []
    for native in (True, False):
        srv = jx.Server(hbm_budget=1 << 30, n_streams=4)
        cids = [srv.open(W.seeds(200 + k, sizes[k]), cfgs[k])[0] for k in range(12)]
        if native:
            lat, sub, wall = srv.replay(np.arange(240) / 20000.0, [cids[c] for c in order], acts,
                                        n_collectors=3, timeout=120.0)
            assert (lat > 0).all() and wall > 0 and sub > 0
            assert srv.stats()["requests"] == 240
        else:
            for c, a in zip(order, acts):
                srv.wait(cids[c], srv.submit(cids[c], a))
        results.append([srv.wait(cids[k], srv.submit(cids[k], finals[k]))[:3] for k in range(12)])
        srv.close()
    for k in range(12):
        for a, b in zip(results[0][k], results[1][k]):
            assert np.array_equal(a, b), f"client {k}"


def test_serving_admission_by_budget():
    """The HBM budget covers the admitted clients' state and maps: a client that
    does not fit next to the resident ones waits for admission in FIFO order."""
    from paper_2605_19926_amd import jx
    cfg = W.env_cfg(side=32, obs_h=84, obs_w=84)
    big_cfg = W.env_cfg(side=32, obs_h=16, obs_w=16)
    small_n, big_n = 200, 6000
    resident = 6 * jx.workspace_bytes(small_n, [cfg])
    big_bytes = jx.workspace_bytes(big_n, [big_cfg])
    srv = jx.Server(hbm_budget=resident + big_bytes - 4096, n_streams=2)
    ids = []
    admitted = []
    for k in range(6):
        cid, ok = srv.open(W.seeds(70 + k, small_n), cfg)
        ids.append(cid)
        admitted.append(ok)
    assert all(admitted)
    cid, ok = srv.open(W.seeds(80, big_n), big_cfg)      # fits the budget alone, not beside them
    assert not ok
    tk = srv.submit(cid, np.zeros(big_n, np.uint8))
    assert srv.wait(cid, tk, timeout=0.2) is None        # still queued for admission
    # closing a queued client keeps its queued request: it is admitted, runs it,
    # and the result stays collectable after the close
    srv.close_client(cid)
    # a queued client with nothing to run leaves the admission queue at once
    idle, ok = srv.open(W.seeds(81, big_n), big_cfg)
    assert not ok
    srv.close_client(idle)
    for c in ids:
        srv.close_client(c)
    res = srv.wait(cid, tk, timeout=60.0)
    assert res is not None and res[1].shape == (big_n,)
    assert res[0].shape == (big_n, 16 * 16 * 3)
    st = srv.stats()
    assert st["admission_waits"] >= 2
    assert st["clients_pending"] == 0
    srv.close()


def test_serving_device_results_equal_host_results():
    """A client opened with device result rings gets, in its ring slot k mod
    slots, exactly the frames, rewards and dones a host-result client of the
    same envs and actions gets copied to the host; in a coalesced mix with
    other clients and in the plain per-request mode.  Nothing is copied to the
    host for it."""
    import torch
    from paper_2605_19926_amd import jx
    cfg = W.env_cfg(side=20, loop_frac=0.1, goal_sprite=1, key_door=1, obs_h=84, obs_w=84, episode_cap=9)
    n, T, slots = 29, 7, 3
    seeds = W.seeds(17, n)
    acts = W.actions(17, T, n, 6)
    fb = 84 * 84 * 3
    for mode in (jx.JX_SERVE_COALESCE, jx.JX_SERVE_PLAIN):
        srv = jx.Server(hbm_budget=1 << 30, n_streams=3, mode=mode)
        hcid, _ = srv.open(seeds, cfg)
        ring_o = torch.zeros(slots * n * fb, dtype=torch.uint8, device="cuda")
        ring_r = torch.zeros(slots * n, dtype=torch.float32, device="cuda")
        ring_d = torch.zeros(slots * n, dtype=torch.uint8, device="cuda")
        dcid, _ = srv.open_dev(seeds, cfg, ring_o, ring_r, ring_d, slots)
        other, _ = srv.open(W.seeds(18, 5), W.env_cfg(side=9, obs_h=64, obs_w=64))
        for t in range(T):
            tk_o = srv.submit(other, W.actions(18, 1, 5, 6, stream=t)[0])
            tk_h = srv.submit(hcid, acts[t])
            tk_d = srv.submit(dcid, acts[t])
            host = srv.wait(hcid, tk_h)
            got = srv.wait(dcid, tk_d)
            assert got[0] is None and got[3] >= 0.0
            srv.wait(other, tk_o, want_obs=False)
            k = t % slots
            o = ring_o[k * n * fb:(k + 1) * n * fb].cpu().numpy().reshape(n, fb)
            assert np.array_equal(o, host[0]), f"mode {mode} step {t}: frames differ"
            assert np.array_equal(ring_r[k * n:(k + 1) * n].cpu().numpy(), host[1])
            assert np.array_equal(ring_d[k * n:(k + 1) * n].cpu().numpy(), host[2])
        # host buffers are refused for a device-result client
        tk = srv.submit(dcid, acts[0])
        with pytest.raises(jx.JxError) as e:
            lib = jx.lib()
            buf = np.zeros(n, np.float32)
            jx.check(lib.jx_server_wait(srv.h, tk, -1.0, None, buf.ctypes.data, None, None))
        assert e.value.code == jx.JX_EINVAL
        assert srv.wait(dcid, tk) is not None   # still collectable without buffers
        srv.close()


def test_serving_injected_launch_failure_fails_only_its_clients(monkeypatch):
    """JX_SERVER_FAIL_LAUNCH=1 makes the server's second launch fail on the
    host (no HIP call is made for it).  Only that launch's request and client
    fail; the other clients are served on and their results equal an
    unfailed server's."""
    from paper_2605_19926_amd import jx
    cfg = W.env_cfg(side=12, goal_sprite=1, obs_h=32, obs_w=32, episode_cap=50)
    sa, sb, sc = W.seeds(81, 6), W.seeds(82, 4), W.seeds(83, 9)
    T = 4
    acts = {k: W.actions(80 + k, T, n, 6) for k, n in ((0, 6), (1, 4), (2, 9))}

    def run(fail: bool, mode):
        if fail:
            monkeypatch.setenv("JX_SERVER_FAIL_LAUNCH", "1")
        else:
            monkeypatch.delenv("JX_SERVER_FAIL_LAUNCH", raising=False)
        srv = jx.Server(hbm_budget=1 << 28, n_streams=2, mode=mode)
        monkeypatch.delenv("JX_SERVER_FAIL_LAUNCH", raising=False)
        a, _ = srv.open(sa, cfg)
        b, _ = srv.open(sb, cfg)
        c, _ = srv.open(sc, cfg)
        out = {a: [], c: []}
        # one request in flight at a time: launch i holds request i alone
        for t in range(T):
            for cid, k in ((a, 0), (b, 1), (c, 2)):
                if fail and cid == b and t > 0:
                    with pytest.raises(jx.JxError) as e:   # the failed client takes no more steps
                        srv.submit(cid, acts[k][t])
                    assert e.value.code == jx.JX_EDEVICE
                    continue
                tk = srv.submit(cid, acts[k][t])
                if fail and cid == b and t == 0:
                    with pytest.raises(jx.JxError) as e:
                        srv.wait(cid, tk)
                    assert e.value.code == jx.JX_EDEVICE
                    continue
                res = srv.wait(cid, tk)
                if cid in out:
                    out[cid].append(res[:3])
        st = srv.stats()
        srv.close()
        return out, st

    for mode in (jx.JX_SERVE_PLAIN, jx.JX_SERVE_COALESCE):
        ref, st_ref = run(False, mode)
        got, st = run(True, mode)
        assert st_ref["failed_launches"] == 0 and st["failed_launches"] == 1
        for cid in ref:
            for t in range(T):
                for k in range(3):
                    assert np.array_equal(got[cid][t][k], ref[cid][t][k]), (mode, cid, t, k)


def test_persistent_step_captured_by_the_caller_replays_correctly():
    """A caller captures one jx_step under the persistent mapping (work queues)
    into its own graph and replays it several times, with eager launches and
    synchronisations between the replays.  Each replay must equal an eager plain
    step from the same state: the queue counters a launch used are back at zero
    when it ends, so a replay finds them clean."""
    import torch
    from paper_2605_19926_amd import jx
    n = 1536
    cfgs, idx = W.batch_cfgs(n, number=41)
    s = torch.cuda.Stream()
    env = jx.Env(W.seeds(41, n), cfgs, idx, stream=s)
    with torch.cuda.stream(s):
        env.reset()
        ob = env.obs_bytes
        acts = torch.zeros(n, dtype=torch.uint8, device=env.dev)
        obs = torch.zeros(ob, dtype=torch.uint8, device=env.dev)
        rew = torch.zeros(n, dtype=torch.float32, device=env.dev)
        done = torch.zeros(n, dtype=torch.uint8, device=env.dev)
    s.synchronize()
    persist = dict(form=1, waves_per_group=2, groups_per_cu=1, store_mode=0)
    env.set_launch(**persist)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        env.step(acts, obs, rew, done)
    s.synchronize()
    ref_obs = torch.zeros_like(obs)
    ref_rew = torch.zeros_like(rew)
    ref_done = torch.zeros_like(done)
    for r in range(4):
        a = torch.from_numpy(W.actions(41, 1, n, 6, stream=r)[0]).to(env.dev)
        with torch.cuda.stream(s):
            acts.copy_(a)
        s.synchronize()
        before = env.get_state_bytes()
        g.replay()
        s.synchronize()
        got = (obs.clone(), rew.clone(), done.clone(), env.get_state_bytes())
        # the same step eagerly, plain mapping, from the same state
        env.set_state_bytes(before)
        env.set_launch(form=0, waves_per_group=4, groups_per_cu=1, store_mode=0)
        with torch.cuda.stream(s):
            env.step(a, ref_obs, ref_rew, ref_done)
        s.synchronize()
        env.set_launch(**persist)
        assert torch.equal(got[0], ref_obs), f"replay {r}: frames differ"
        assert torch.equal(got[1], ref_rew) and torch.equal(got[2], ref_done), f"replay {r}: rewards/dones"
        assert np.array_equal(got[3], env.get_state_bytes()), f"replay {r}: state differs"
        # leave the env in the replayed state for the next round
        env.set_state_bytes(got[3])
    env.close()


def test_waves_per_env_limits():
    """waves_per_env: 1, 2 or 4, plain form only, at most waves_per_group."""
    from paper_2605_19926_amd import jx
    env = U.env_of(W.TINY["cfg"], W.seeds(1, 4), obs=False)
    for bad in (dict(form=0, waves_per_group=4, waves_per_env=3),
                dict(form=1, waves_per_group=4, waves_per_env=2),
                dict(form=0, waves_per_group=2, waves_per_env=4)):
        with pytest.raises(jx.JxError) as e:
            env.set_launch(**bad)
        assert e.value.code == jx.JX_EINVAL
    env.set_launch(form=0, waves_per_group=8, waves_per_env=4)
    assert env.get_launch()["waves_per_env"] == 4
    env.close()

