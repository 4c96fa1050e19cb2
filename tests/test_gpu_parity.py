"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Bars (stated per check): episode-start states bit-exact; one-step outcomes
(reward, done, events, pickups, resets) exact from shared states, positions
within 2 float32 ulp, heading within 1e-6 mod 2pi; frames bit-exact on every
unflagged column with hit and side exact and t* within 1e-4 relative; flagged
columns under 0.1 %.
"""
import math

import numpy as np
import pytest

import oracle as orc
import workloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _dbg_array(env, torch):
    return torch.zeros(env.n * max(c["obs_w"] for c in env.cfgs) * 16, dtype=torch.uint8,
                       device=env.dev)


def _dbg_np(buf, env):
    mw = max(c["obs_w"] for c in env.cfgs)
    return buf.cpu().numpy().view(np.dtype([("hit", "<i4"), ("side", "<i4"), ("t", "<f4"),
                                            ("cell", "<i4")])).reshape(env.n, mw)


@pytest.mark.parametrize("wl,n_check", [(W.TINY, 16), (W.SCALE, 96), (W.KEYDOOR, 64),
                                        (W.ASCII, 96), (W.ASCII_TINY, 16)])
def test_reset_state_and_first_frame(wl, n_check):
    import torch
    cfg = wl["cfg"]
    n = wl["n_envs"] if wl is not W.KEYDOOR else 2048
    seeds = W.seeds(wl["number"], n)
    env = U.env_of(cfg, seeds)
    S = env.get_state()
    lay = env.state_layout()
    dbg = _dbg_array(env, torch)
    env.render(None, dbg)
    torch.cuda.synchronize()
    D = _dbg_np(dbg, env)
    obs = env.obs0.cpu().numpy()
    rng = np.random.default_rng(1)
    pick = np.arange(n) if n <= n_check else np.sort(rng.choice(n, n_check, replace=False))
    stats = U.FrameStats()
    maps_off = lay["maps"][0]
    raw = env.get_state_bytes()
    for i in pick:
        grid = U.oracle_maze(cfg, seeds[i])
        mo = int(S["map_offset"][i])
        N = cfg["side"]
        gm = raw[maps_off + mo: maps_off + mo + N * N].reshape(N, N)
        assert (gm == grid).all(), f"env {i}: map differs"
        o = orc.reset(grid, orc.make_cfg(cfg), int(seeds[i]), 0).as_dict()
        errs = U.compare_reset_state(U.gpu_state_dict(S, i), o)
        assert not errs, f"env {i}: {errs}"
        g = U.frame_of(obs, env.obs_offsets, i, cfg["obs_h"], cfg["obs_w"])
        U.check_frame(stats, g, grid, orc.make_cfg(cfg), orc.state_from(o), D[i], tag=f"env {i}")
    stats.report(f"reset/{wl['name']}")
    assert not stats.mismatch, stats.mismatch[:10]
    assert stats.frac_flagged() < U.FLAG_LIMIT, stats.summary()
    env.close()


def _one_step_case(cfg, n, number, n_check, launch=None, seed_rng=7, invalid_frac=0.03, name=None):
    import torch
    seeds = W.seeds(number, n)
    env = U.env_of(cfg, seeds, obs=False)
    if launch:
        env.set_launch(**launch)
    rng = np.random.default_rng(seed_rng)
    pick = np.arange(n) if n <= n_check else np.sort(rng.choice(n, n_check, replace=False))
    grids = {int(i): U.oracle_maze(cfg, seeds[i]) for i in pick}
    states = []
    for i in range(n):
        if int(i) in grids:
            states.append(U.synth_state(rng, cfg, seeds[i], grids[int(i)]))
        else:
            states.append(None)
    # envs outside the sample get a sample state (cheap) so every env steps from a valid state
    filler = next(s for s in states if s is not None)
    states = [s if s is not None else filler for s in states]
    # the filler states live on other mazes: give those envs their own maze's reset state
    S0 = env.get_state()
    for i in range(n):
        if int(i) not in grids:
            states[i] = U.gpu_state_dict(S0, i)   # (not compared: only keeps the batch valid)
    env.set_state(U.gpu_fields(states))
    acts = rng.integers(0, cfg["n_actions"], size=n).astype(np.uint8)
    bad = rng.random(n) < invalid_frac
    acts[bad] = 250
    act_t = torch.from_numpy(acts).to(env.dev)
    obs = torch.empty(env.obs_bytes, dtype=torch.uint8, device=env.dev)
    env.step(act_t, obs)
    dbg = _dbg_array(env, torch)
    env.render(None, dbg)
    torch.cuda.synchronize()
    S = env.get_state()
    rew = env.reward.cpu().numpy()
    done = env.done.cpu().numpy()
    D = _dbg_np(dbg, env)
    obs_np = obs.cpu().numpy()
    stats = U.FrameStats()
    skipped = 0
    errors = []
    n_done = 0
    oc = orc.make_cfg(cfg)
    for i in pick:
        i = int(i)
        g_after = U.gpu_state_dict(S, i)
        skip, errs, o = U.compare_step(states[i], cfg, seeds[i], grids[i], acts[i],
                                       g_after, rew[i], done[i], S["events"][i])
        if skip:
            skipped += 1
        else:
            errors += [f"env {i}: {e}" for e in errs]
            n_done += int(done[i])
        # The frame the step returned is the render of the post-step state the
        # GPU stored (float32); the oracle renders that same state (shared-state
        # check), so every sampled frame is compared, flagged steps included.
        g = U.frame_of(obs_np, env.obs_offsets, i, cfg["obs_h"], cfg["obs_w"])
        U.check_frame(stats, g, grids[i], oc, orc.state_from(g_after), D[i], tag=f"env {i}")
    stats.report(f"one-step/{name or cfg.get('obs_w')}")
    assert skipped <= max(2, len(pick) // 50), f"too many flagged steps: {skipped}"
    assert not errors, errors[:10]
    assert not stats.mismatch, stats.mismatch[:10]
    assert stats.frac_flagged() < U.FLAG_LIMIT, stats.summary()
    inv = S["invalid"]
    assert int(inv.sum()) == int(bad.sum())
    env.close()
    return n_done, stats


def _render_case(cfg, n, number, n_check, seed_rng=3, launch=None, name=None):
    """Shared input state set into the GPU, rendered by both sides."""
    import torch
    seeds = W.seeds(number, n)
    env = U.env_of(cfg, seeds, obs=False)
    if launch:
        env.set_launch(**launch)
    rng = np.random.default_rng(seed_rng)
    pick = np.arange(n) if n <= n_check else np.sort(rng.choice(n, n_check, replace=False))
    S0 = env.get_state()
    states = [U.gpu_state_dict(S0, i) for i in range(n)]
    grids = {}
    for i in pick:
        grids[int(i)] = U.oracle_maze(cfg, seeds[i])
        states[int(i)] = U.synth_state(rng, cfg, seeds[i], grids[int(i)])
    env.set_state(U.gpu_fields(states))
    obs = torch.empty(env.obs_bytes, dtype=torch.uint8, device=env.dev)
    dbg = _dbg_array(env, torch)
    env.render(obs, dbg)
    torch.cuda.synchronize()
    D = _dbg_np(dbg, env)
    obs_np = obs.cpu().numpy()
    stats = U.FrameStats()
    oc = orc.make_cfg(cfg)
    for i in pick:
        i = int(i)
        g = U.frame_of(obs_np, env.obs_offsets, i, cfg["obs_h"], cfg["obs_w"])
        U.check_frame(stats, g, grids[i], oc, orc.state_from(states[i]), D[i], tag=f"env {i}")
    if name:
        stats.report(f"render/{name}")
    assert not stats.mismatch, stats.mismatch[:10]
    assert stats.frac_flagged() < U.FLAG_LIMIT, stats.summary()
    env.close()
    return stats


@pytest.mark.parametrize("wl,n,n_check", [(W.TINY, 16, 16), (W.SCALE, 4096, 256),
                                          (W.KEYDOOR, 8192, 160), (W.ASCII, 4096, 256),
                                          (W.ASCII_TINY, 16, 16)])
def test_render_shared_state(wl, n, n_check):
    _render_case(wl["cfg"], n, wl["number"], n_check, name=wl["name"])


@pytest.mark.parametrize("wl,n,n_check,levels,dist", [(W.SCALE, 4096, 256, 8, 12.0),
                                                        (W.KEYDOOR, 8192, 160, 4, 20.0),
                                                        (W.TINY, 16, 16, 16, 3.0)])
def test_render_shared_state_distance_shading(wl, n, n_check, levels, dist):
    cfg = dict(wl["cfg"], shade_levels=levels, shade_dist=dist)
    stats = _render_case(cfg, n, wl["number"], n_check, seed_rng=41, name=f"{wl['name']}-shaded{levels}")
    assert stats.cols >= n_check * cfg["obs_w"]


@pytest.mark.parametrize("wl", [W.OPEN64, W.PILLARS64])
def test_long_rays_render_and_one_step(wl):
    # 64-side maps where rays cross up to ~90 tiles (128 columns each): the
    # longest walks the kernel makes, where each crossing parameter comes from
    # the most line counts
    stats = _render_case(wl["cfg"], wl["n_envs"], wl["number"], wl["n_envs"], seed_rng=17,
                         name=wl["name"])
    assert stats.cols == wl["n_envs"] * 128
    for k in range(3):
        _one_step_case(wl["cfg"], wl["n_envs"], wl["number"], wl["n_envs"], seed_rng=90 + k,
                       name=wl["name"])


def test_one_step_tiny_all_envs():
    for k in range(8):
        _one_step_case(W.TINY["cfg"], 16, W.TINY["number"], 16, seed_rng=100 + k, name=W.TINY["name"])


def test_one_step_scale_full_size_sampled():
    # the headline workload's full batch, plain per-step mapping (the timed
    # fused launch is checked by test_headline_fused_rollout_full_size)
    _one_step_case(W.SCALE["cfg"], 4096, W.SCALE["number"], 160,
                   launch=dict(form=0, waves_per_group=1, groups_per_cu=4, store_mode=0),
                   name=W.SCALE["name"])


def test_one_step_ascii_maps():
    # every Table 2 symbol: keys by colour, locked and unlocked doors (random
    # open/taken states), candidates, coloured walls
    _one_step_case(W.ASCII["cfg"], 4096, W.ASCII["number"], 200, seed_rng=61, name=W.ASCII["name"])
    for k in range(4):
        _one_step_case(W.ASCII_TINY["cfg"], 16, W.ASCII_TINY["number"], 16, seed_rng=70 + k)


def test_one_step_keydoor_sampled():
    _one_step_case(W.KEYDOOR["cfg"], 8192, W.KEYDOOR["number"], 96, name=W.KEYDOOR["name"])


@pytest.mark.parametrize("side,hw", [(5, (2, 4)), (64, (128, 128)), (9, (84, 84)), (33, (32, 32)),
                                     (64, (32, 128)), (16, (128, 4)),
                                     # widths whose column-group count does not divide
                                     # the wave: 55 of 64 lanes at W = 44, 62 at W = 124
                                     (12, (30, 44)), (24, (64, 124))])
def test_one_step_shape_extremes(side, hw):
    cfg = W.env_cfg(side=side, loop_frac=0.1, key_door=1 if side >= 9 else 0, goal_sprite=1,
                    max_decor=2, obs_h=hw[0], obs_w=hw[1], episode_cap=64)
    _one_step_case(cfg, 48, 11, 48, seed_rng=side, name=f"side{side}-{hw[0]}x{hw[1]}")


def test_persistent_form_matches_plain_one_step():
    a, _ = _one_step_case(W.SCALE["cfg"], 1024, 2, 64,
                          launch=dict(form=1, waves_per_group=2, groups_per_cu=2, store_mode=1))
    assert a >= 0


def _fused_vs_single_full_size(wl, T, launch, n_pick, tag, stagger=False):
    """One fused T-step launch of workload `wl` at full size under `launch`,
    against T single-step launches from the same start (every frame compared on
    the device, rewards, dones, final state) and, along those steps, n_pick
    sampled envs against the oracle at every step from the shared state."""
    import torch
    cfg, n = wl["cfg"], wl["n_envs"]
    H, W_ = cfg["obs_h"], cfg["obs_w"]
    seeds = W.seeds(wl["number"], n)
    acts = W.actions(wl["number"], T, n, cfg["n_actions"])
    env = U.env_of(cfg, seeds, obs=False)
    if stagger:   # every env reaches its cap inside the rollout
        env.set_state({"t": (cfg["episode_cap"] - 1 - (np.arange(n) % T)).astype(np.uint32)})
    env.set_launch(**launch)
    snap = env.get_state_bytes()
    ob = env.obs_bytes
    act_d = torch.from_numpy(acts).to(env.dev)
    ring = torch.empty(T * ob, dtype=torch.uint8, device=env.dev)
    rew = torch.empty(T * n, dtype=torch.float32, device=env.dev)
    done = torch.empty(T * n, dtype=torch.uint8, device=env.dev)
    env.rollout(act_d, ring, rew, done, T, obs_stride=ob, graph=False, fused=True)
    torch.cuda.synchronize()
    fused_state = env.get_state_bytes()
    f_rew, f_done = rew.cpu().numpy(), done.cpu().numpy()
    env.set_state_bytes(snap)
    env.set_launch(form=0, waves_per_group=1, groups_per_cu=1, store_mode=0)
    one = torch.empty(ob, dtype=torch.uint8, device=env.dev)
    r1 = torch.empty(n, dtype=torch.float32, device=env.dev)
    d1 = torch.empty(n, dtype=torch.uint8, device=env.dev)
    rng = np.random.default_rng(11)
    pick = [int(i) for i in np.sort(rng.choice(n, n_pick, replace=False))]
    grids = {i: U.oracle_maze(cfg, seeds[i]) for i in pick}
    oc = orc.make_cfg(cfg)
    S_prev = env.get_state()
    stats = U.FrameStats()
    skipped = checked = 0
    errors = []
    for t in range(T):
        env.step(act_d[t], one, r1, d1)
        torch.cuda.synchronize()
        assert torch.equal(one, ring[t * ob:(t + 1) * ob]), f"step {t}: fused frames differ"
        r_np, d_np = r1.cpu().numpy(), d1.cpu().numpy()
        assert np.array_equal(r_np, f_rew[t * n:(t + 1) * n]), f"step {t}: rewards differ"
        assert np.array_equal(d_np, f_done[t * n:(t + 1) * n]), f"step {t}: dones differ"
        S = env.get_state()
        one_np = one.cpu().numpy()
        for i in pick:
            checked += 1
            g_after = U.gpu_state_dict(S, i)
            skip, errs, _ = U.compare_step(U.gpu_state_dict(S_prev, i), cfg, seeds[i], grids[i], acts[t, i],
                                           g_after, r_np[i], d_np[i], S["events"][i])
            skipped += int(skip)
            errors += [f"step {t} env {i}: {e}" for e in errs]
            U.check_frame(stats, U.frame_of(one_np, env.obs_offsets, i, H, W_), grids[i], oc,
                          orc.state_from(g_after), tag=f"step {t} env {i}")
        S_prev = S
    assert np.array_equal(env.get_state_bytes(), fused_state), "final state differs"
    assert not errors, errors[:10]
    assert skipped <= max(2, checked // 50), f"too many flagged steps: {skipped}"
    stats.report(tag)
    assert not stats.mismatch, stats.mismatch[:10]
    assert stats.frac_flagged() < U.FLAG_LIMIT, stats.summary()
    env.close()
    return f_done


def test_keydoor_fused_rollout_full_size():
    """The key-door workload as bench.py times it: 8192 envs of 32x32 mazes
    (door, key, goal and decor billboards, 84x84 frames) in one fused launch
    with 8 waves per workgroup, every env reaching its cap inside the rollout."""
    f_done = _fused_vs_single_full_size(W.KEYDOOR, 32, dict(form=0, waves_per_group=8, groups_per_cu=4,
                                                            store_mode=0), 24,
                                        f"fused-rollout/{W.KEYDOOR['name']}", stagger=True)
    assert f_done.reshape(32, -1).any(axis=0).all(), "every env resets inside the rollout"


def test_headline_fused_rollout_full_size():
    """The benchmark's timed configuration itself: the 4096 envs of the headline
    workload in one fused 128-step launch with 8 waves per workgroup, frames into
    a 128-slot ring.  (a) Every output equals 128 single-step launches from the
    same start bit for bit (each ring slot compared on the device, every reward
    and done, the final state); (b) along those single steps a sample of 32 envs
    is checked against the oracle at every step from the shared state (outcomes
    exact, positions within 2 ulp, frames bit-exact on unflagged columns)."""
    import torch
    wl = W.SCALE
    cfg, n, T = wl["cfg"], wl["n_envs"], 128
    H, W_ = cfg["obs_h"], cfg["obs_w"]
    seeds = W.seeds(wl["number"], n)
    acts = W.actions(wl["number"], T, n, cfg["n_actions"])
    env = U.env_of(cfg, seeds, obs=False)
    env.set_launch(form=0, waves_per_group=8, groups_per_cu=4, store_mode=0)
    snap = env.get_state_bytes()
    ob = env.obs_bytes
    act_d = torch.from_numpy(acts).to(env.dev)
    ring = torch.empty(T * ob, dtype=torch.uint8, device=env.dev)
    rew = torch.empty(T * n, dtype=torch.float32, device=env.dev)
    done = torch.empty(T * n, dtype=torch.uint8, device=env.dev)
    env.rollout(act_d, ring, rew, done, T, obs_stride=ob, graph=False, fused=True)
    torch.cuda.synchronize()
    fused_state = env.get_state_bytes()
    f_rew, f_done = rew.cpu().numpy(), done.cpu().numpy()
    # the same steps one launch at a time, from the same start
    env.set_state_bytes(snap)
    one = torch.empty(ob, dtype=torch.uint8, device=env.dev)
    r1 = torch.empty(n, dtype=torch.float32, device=env.dev)
    d1 = torch.empty(n, dtype=torch.uint8, device=env.dev)
    rng = np.random.default_rng(5)
    pick = [int(i) for i in np.sort(rng.choice(n, 32, replace=False))]
    grids = {i: U.oracle_maze(cfg, seeds[i]) for i in pick}
    oc = orc.make_cfg(cfg)
    S_prev = env.get_state()
    stats = U.FrameStats()
    skipped = checked = n_done = 0
    errors = []
    for t in range(T):
        env.step(act_d[t], one, r1, d1)
        torch.cuda.synchronize()
        assert torch.equal(one, ring[t * ob:(t + 1) * ob]), f"step {t}: fused frames differ"
        r_np, d_np = r1.cpu().numpy(), d1.cpu().numpy()
        assert np.array_equal(r_np, f_rew[t * n:(t + 1) * n]), f"step {t}: rewards differ"
        assert np.array_equal(d_np, f_done[t * n:(t + 1) * n]), f"step {t}: dones differ"
        S = env.get_state()
        one_np = one.cpu().numpy()
        for i in pick:
            checked += 1
            g_after = U.gpu_state_dict(S, i)
            skip, errs, o = U.compare_step(U.gpu_state_dict(S_prev, i), cfg, seeds[i], grids[i],
                                           acts[t, i], g_after, r_np[i], d_np[i], S["events"][i])
            if skip:
                skipped += 1
            errors += [f"step {t} env {i}: {e}" for e in errs]
            n_done += int(d_np[i])
            # the frame of the post-step state the GPU stored, rendered by both
            U.check_frame(stats, U.frame_of(one_np, env.obs_offsets, i, H, W_), grids[i], oc,
                          orc.state_from(g_after), tag=f"step {t} env {i}")
        S_prev = S
    assert np.array_equal(env.get_state_bytes(), fused_state), "final state differs"
    assert not errors, errors[:10]
    assert skipped <= max(2, checked // 50), f"too many flagged steps: {skipped}"
    stats.report(f"fused-rollout/{wl['name']}")
    assert not stats.mismatch, stats.mismatch[:10]
    assert stats.frac_flagged() < U.FLAG_LIMIT, stats.summary()
    assert stats.cols == checked * W_
    env.close()


@pytest.mark.parametrize("wl", [W.TINY, W.ASCII_TINY])
def test_trajectory_tiny_full(wl):
    """A small workload end to end (16 envs, every env every step, 1000 steps on
    a maze or 400 on the ASCII map), GPU and oracle each running its own
    trajectory from the same seeds and actions.  Outcomes (reward, done, events,
    keys taken, doors open) must agree at every step; a step whose outcome
    differs must be one the oracle flags, with its window widened by the
    measured FP32/FP64 drift (after which that env is no longer compared)."""
    import torch
    cfg, n, T = wl["cfg"], wl["n_envs"], wl["steps"]
    seeds = W.seeds(wl["number"], n)
    acts = W.actions(wl["number"], T, n, cfg["n_actions"])
    env = U.env_of(cfg, seeds)
    oc = orc.make_cfg(cfg)
    grids = [U.oracle_maze(cfg, s) for s in seeds]
    ost = [orc.reset(grids[i], oc, int(seeds[i]), 0) for i in range(n)]
    act_d = torch.from_numpy(acts).to(env.dev)
    obs = torch.empty(T * env.obs_bytes, dtype=torch.uint8, device=env.dev)
    rew = torch.empty(T * n, dtype=torch.float32, device=env.dev)
    done = torch.empty(T * n, dtype=torch.uint8, device=env.dev)
    # record per-step state via one step at a time (positions are compared each step)
    xs = np.zeros((T, n), np.float32)
    ys = np.zeros((T, n), np.float32)
    evs = np.zeros((T, n), np.uint8)
    eps = np.zeros((T, n), np.uint32)
    fls = np.zeros((T, n), np.uint8)
    drs = np.zeros((T, n), np.uint32)
    for t in range(T):
        env.step(act_d[t], obs[t * env.obs_bytes:(t + 1) * env.obs_bytes], rew[t * n:(t + 1) * n],
                 done[t * n:(t + 1) * n])
        S = env.get_state()
        xs[t], ys[t], evs[t], eps[t] = S["x"], S["y"], S["events"], S["episode"]
        fls[t], drs[t] = S["flags"], S["doors"]
    obs_np = obs.cpu().numpy().reshape(T, -1)
    rew_np = rew.cpu().numpy().reshape(T, n)
    done_np = done.cpu().numpy().reshape(T, n)
    diverged = {}
    stats = U.FrameStats()
    exact_frames = 0
    for t in range(T):
        for i in range(n):
            if i in diverged:
                continue
            nxt, r, d, ev, sf = orc.step(grids[i], oc, int(seeds[i]), ost[i], int(acts[t, i]))
            drift = max(abs(float(xs[t, i]) - nxt.x), abs(float(ys[t, i]) - nxt.y))
            same = (r == rew_np[t, i] and d == done_np[t, i] and ev == evs[t, i] and
                    nxt.akey_taken == (fls[t, i] >> 2) & 7 and nxt.doors_open == drs[t, i])
            if not same:
                prev = 0.0 if t == 0 else max(abs(float(xs[t - 1, i]) - ost[i].x),
                                              abs(float(ys[t - 1, i]) - ost[i].y))
                sfw = orc.step(grids[i], oc, int(seeds[i]), ost[i], int(acts[t, i]),
                               window=1e-5 + 4 * prev)[4]
                near = sfw != 0
                assert near, (f"step {t} env {i}: unexplained divergence: gpu ev {evs[t, i]:#x} "
                              f"oracle ev {ev:#x} (drift {drift:.2e})")
                diverged[i] = t
                continue
            assert drift < 1e-3, f"step {t} env {i}: drift {drift}"
            ost[i] = nxt
            g = obs_np[t].reshape(n, cfg["obs_h"], cfg["obs_w"], 3)[i]
            if d:
                # episode starts are exact states: the frame must match outright
                U.check_frame(stats, g, grids[i], oc, nxt, tag=f"t{t} e{i}")
                exact_frames += 1
            else:
                loose = U.FrameStats()
                U.check_frame(loose, g, grids[i], oc, nxt, tag=f"t{t} e{i}")
                # states differ by the drift here: allow a column within the drift of a tie
                loose.mismatch = [m + " (drift)" for m in loose.mismatch]
                stats.add(loose)
    n_cols = stats.cols
    drift_mismatch = [m for m in stats.mismatch if m.endswith("(drift)")]
    hard = [m for m in stats.mismatch if not m.endswith("(drift)")]
    assert not hard, hard[:10]
    assert len(drift_mismatch) <= n_cols * 1e-3, drift_mismatch[:10]
    assert len(diverged) <= 2, diverged
    assert stats.frac_flagged() < U.FLAG_LIMIT, stats.summary()
    assert exact_frames >= 16 * 3                       # several resets per env were checked
    env.close()


def test_batching_form_full_size_persistent_fused():
    """The batching workload at full size in the launch configuration bench.py
    times for it: 16,384 envs of mixed shapes (map side 8-64, frames 32^2-128^2,
    key-door on half) in one persistent fused launch (4 waves x 2 workgroups per
    compute unit, envs claimed one at a time), with episode clocks set so that
    every env reaches its cap inside the rollout (a device reset in every env).
    (a) Every output equals single-step launches from the same start bit for bit
    (each step's frames compared on the device, rewards, dones, final state);
    (b) along those single steps 32 sampled envs are checked against the oracle
    at every step from the shared state."""
    import torch
    n, T = W.BATCH["n_envs"], 40
    cfgs, idx = W.batch_cfgs(n)
    seeds = W.seeds(W.BATCH["number"], n)
    acts = W.actions(W.BATCH["number"], T, n, 6)
    env = U.env_of(cfgs, seeds, idx, obs=False)
    caps = np.array([c["episode_cap"] for c in cfgs], np.int64)[idx]
    env.set_state({"t": (caps - 1 - (np.arange(n) % T)).astype(np.uint32)})
    env.set_launch(form=1, waves_per_group=4, groups_per_cu=2, store_mode=0)
    snap = env.get_state_bytes()
    ob = env.obs_bytes
    act_d = torch.from_numpy(acts).to(env.dev)
    ring = torch.empty(T * ob, dtype=torch.uint8, device=env.dev)
    rew = torch.empty(T * n, dtype=torch.float32, device=env.dev)
    done = torch.empty(T * n, dtype=torch.uint8, device=env.dev)
    env.rollout(act_d, ring, rew, done, T, obs_stride=ob, graph=False, fused=True)
    torch.cuda.synchronize()
    fused_state = env.get_state_bytes()
    f_rew, f_done = rew.cpu().numpy(), done.cpu().numpy()
    assert f_done.reshape(T, n).any(axis=0).all(), "every env resets inside the rollout"
    env.set_state_bytes(snap)
    env.set_launch(form=0, waves_per_group=1, groups_per_cu=1, store_mode=0)
    one = torch.empty(ob, dtype=torch.uint8, device=env.dev)
    r1 = torch.empty(n, dtype=torch.float32, device=env.dev)
    d1 = torch.empty(n, dtype=torch.uint8, device=env.dev)
    rng = np.random.default_rng(9)
    pick = [int(i) for i in np.sort(rng.choice(n, 32, replace=False))]
    grids = {i: U.oracle_maze(cfgs[idx[i]], seeds[i]) for i in pick}
    ocs = {i: orc.make_cfg(cfgs[idx[i]]) for i in pick}
    S_prev = env.get_state()
    stats = U.FrameStats()
    skipped = checked = 0
    errors = []
    for t in range(T):
        env.step(act_d[t], one, r1, d1)
        torch.cuda.synchronize()
        assert torch.equal(one, ring[t * ob:(t + 1) * ob]), f"step {t}: fused frames differ"
        r_np, d_np = r1.cpu().numpy(), d1.cpu().numpy()
        assert np.array_equal(r_np, f_rew[t * n:(t + 1) * n]), f"step {t}: rewards differ"
        assert np.array_equal(d_np, f_done[t * n:(t + 1) * n]), f"step {t}: dones differ"
        S = env.get_state()
        one_np = one.cpu().numpy()
        for i in pick:
            c = cfgs[idx[i]]
            checked += 1
            g_after = U.gpu_state_dict(S, i)
            skip, errs, _ = U.compare_step(U.gpu_state_dict(S_prev, i), c, seeds[i], grids[i], acts[t, i],
                                           g_after, r_np[i], d_np[i], S["events"][i])
            skipped += int(skip)
            errors += [f"step {t} env {i}: {e}" for e in errs]
            U.check_frame(stats, U.frame_of(one_np, env.obs_offsets, i, c["obs_h"], c["obs_w"]), grids[i],
                          ocs[i], orc.state_from(g_after), tag=f"step {t} env {i}")
        S_prev = S
    assert np.array_equal(env.get_state_bytes(), fused_state), "final state differs"
    assert not errors, errors[:10]
    assert skipped <= max(2, checked // 50), f"too many flagged steps: {skipped}"
    stats.report(f"persistent-fused/{W.BATCH['name']}")
    assert not stats.mismatch, stats.mismatch[:10]
    assert stats.frac_flagged() < U.FLAG_LIMIT, stats.summary()
    env.close()
