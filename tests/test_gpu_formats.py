"""GPU: frames written in the training-buffer formats (NHWC or NCHW; the byte,
or byte / 255 as bfloat16 or float32) and the previous action beside them.

Bars: every unflagged column of every format bit-exact against the oracle's
render converted by the oracle's format function (float elements compared as
bit patterns); the previous action equal to the oracle's rule on every env and
step; a format's frames equal to the byte frames of the same trajectory
converted element by element (all pixels, flagged columns included, since both
come from the same cast); every launch form of one format identical."""
import numpy as np
import pytest

import oracle as orc
import workloads as W
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

FORMATS = [(lay, dt) for lay in (0, 1) for dt in (0, 1, 2)]
ELEM = {0: 1, 1: 2, 2: 4}
VIEW = {0: np.uint8, 1: np.uint16, 2: np.uint32}   # floats compared as bit patterns


def typed_hwc(raw: np.ndarray, H: int, W_: int, layout: int, dtype: int) -> np.ndarray:
    """A frame's bytes as elements in [H, W, 3] order."""
    a = np.ascontiguousarray(raw).view(VIEW[dtype])
    return a.reshape(H, W_, 3) if layout == 0 else a.reshape(3, H, W_).transpose(1, 2, 0)


def oracle_hwc(frame_u8: np.ndarray, layout: int, dtype: int) -> np.ndarray:
    f = orc.format_frame(frame_u8, layout, dtype)
    f = f.view(VIEW[dtype]) if dtype else f
    return f if layout == 0 else f.transpose(1, 2, 0)


def gpu_frame(obs_np, env, i, cfg):
    H, W_ = cfg["obs_h"], cfg["obs_w"]
    nb = H * W_ * 3 * ELEM[cfg["obs_dtype"]]
    o = int(env.obs_offsets[i])
    return typed_hwc(obs_np[o:o + nb], H, W_, cfg["obs_layout"], cfg["obs_dtype"])


def fmt_cfg(base: dict, layout: int, dtype: int) -> dict:
    c = dict(base)
    c["obs_layout"], c["obs_dtype"] = layout, dtype
    return c


CASES = [
    ("tiny-64px", W.TINY["cfg"], 16),
    ("keydoor-84px", W.env_cfg(side=16, n_colors=8, key_door=1, goal_sprite=1, max_decor=2,
                               obs_h=84, obs_w=84, episode_cap=64), 48),
    ("ascii-32x48", W.env_cfg(side=10, ascii_map=W.MAP10, goal_sprite=1, n_actions=4,
                              episode_cap=128, obs_h=32, obs_w=48), 16),
    # the largest map and frame, and the smallest frame
    ("max-64side-128px", W.env_cfg(side=64, loop_frac=0.1, key_door=1, goal_sprite=1, max_decor=2,
                                   obs_h=128, obs_w=128, episode_cap=64), 8),
    ("min-2x4px", W.env_cfg(side=5, goal_sprite=1, obs_h=2, obs_w=4, episode_cap=16), 8),
]


@pytest.mark.parametrize("layout,dtype", FORMATS)
@pytest.mark.parametrize("name,base,n", CASES, ids=[c[0] for c in CASES])
def test_reset_and_step_frames_against_oracle(name, base, n, layout, dtype):
    import torch
    cfg = fmt_cfg(base, layout, dtype)
    seeds = W.seeds(31, n)
    env = U.env_of(cfg, seeds)
    assert env.obs_bytes == n * cfg["obs_h"] * cfg["obs_w"] * 3 * ELEM[dtype]
    oc = orc.make_cfg(cfg)
    grids = [U.oracle_maze(cfg, s) for s in seeds]
    stats = U.FrameStats()
    obs0 = env.obs0.cpu().numpy()
    conv = lambda f: oracle_hwc(f, layout, dtype)   # noqa: E731
    for i in range(n):
        o = orc.reset(grids[i], oc, int(seeds[i]), 0)
        U.check_frame(stats, gpu_frame(obs0, env, i, cfg), grids[i], oc, o, tag=f"reset env {i}",
                      convert=conv)
    # steps: the frame is the render of the stored post-step state
    rng = np.random.default_rng(7)
    obs = torch.empty(env.obs_bytes, dtype=torch.uint8, device=env.dev)
    prev = torch.full((n,), 99, dtype=torch.uint8, device=env.dev)
    for t in range(6):
        acts = rng.integers(0, cfg["n_actions"] + 1, size=n).astype(np.uint8)   # some out of range
        env.step(torch.from_numpy(acts).to(env.dev), obs, prev=prev)
        torch.cuda.synchronize()
        S = env.get_state()
        done = env.done.cpu().numpy()
        pv = prev.cpu().numpy()
        on = obs.cpu().numpy()
        for i in range(n):
            assert pv[i] == orc.prev_action(oc, int(acts[i]), int(done[i])), f"step {t} env {i}"
            st = orc.state_from(U.gpu_state_dict(S, i))
            U.check_frame(stats, gpu_frame(on, env, i, cfg), grids[i], oc, st, tag=f"step {t} env {i}",
                          convert=conv)
    # render without stepping: the frame of the current state, as the last step returned it
    again = torch.zeros_like(obs)
    env.render(again)
    torch.cuda.synchronize()
    assert torch.equal(again, obs)
    assert not stats.mismatch, stats.mismatch[:10]
    # (a small sample: the flag-rate bar of the main parity tests, loosened tenfold)
    assert stats.frac_flagged() < 10 * U.FLAG_LIMIT, stats.summary()
    env.close()


def _trajectory(cfg, seeds, acts, mode):
    import torch
    env = U.env_of(cfg, seeds, obs=False)
    if mode == "persistent":   # a training format maps every launch form to the plain kernel
        env.set_launch(form=1, waves_per_group=2, groups_per_cu=4, store_mode=0)
    if mode.endswith("-wpe"):   # several waves per env, each writing its share of the rows
        env.set_launch(form=0, waves_per_group=4, groups_per_cu=1, store_mode=0, waves_per_env=4 if
                       mode.startswith("fused") else 2)
        mode = mode[:-4]
    n, T, ob = len(seeds), acts.shape[0], env.obs_bytes
    acts_d = torch.from_numpy(acts).to(env.dev)
    obs = torch.zeros(T * ob, dtype=torch.uint8, device=env.dev)
    rew = torch.zeros(T * n, dtype=torch.float32, device=env.dev)
    done = torch.zeros(T * n, dtype=torch.uint8, device=env.dev)
    prev = torch.zeros(T * n, dtype=torch.uint8, device=env.dev)
    if mode in ("eager", "persistent"):
        for t in range(T):
            env.step(acts_d[t], obs[t * ob:(t + 1) * ob], rew[t * n:(t + 1) * n], done[t * n:(t + 1) * n],
                     prev=prev[t * n:(t + 1) * n])
    else:
        env.rollout(acts_d, obs, rew, done, T, obs_stride=ob, graph=mode == "graph",
                    fused=mode == "fused", prev=prev)
    torch.cuda.synchronize()
    out = (obs.cpu().numpy(), rew.cpu().numpy(), done.cpu().numpy(), prev.cpu().numpy(),
           env.get_state_bytes())
    offs = env.obs_offsets.copy()
    env.close()
    return out, offs, ob


MAZE_KD = W.env_cfg(side=16, n_colors=8, loop_frac=0.1, goal_sprite=1, key_door=1, max_decor=1,
                    n_actions=6, episode_cap=24, obs_h=64, obs_w=64)
ASCII_64 = W.env_cfg(side=10, ascii_map=W.MAP10, goal_sprite=1, n_actions=4, episode_cap=24,
                     obs_h=64, obs_w=64)


@pytest.mark.parametrize("base,layout,dtype", [(MAZE_KD, 1, 2), (MAZE_KD, 0, 1), (MAZE_KD, 1, 0),
                                               (ASCII_64, 1, 2), (ASCII_64, 0, 1)],
                         ids=["maze-nchw-f32", "maze-nhwc-bf16", "maze-nchw-u8", "ascii-nchw-f32",
                              "ascii-nhwc-bf16"])
def test_format_is_the_byte_frame_converted_in_every_form(base, layout, dtype):
    cfg = fmt_cfg(base, layout, dtype)
    n, T = 96, 40
    seeds = W.seeds(33, n)
    acts = W.actions(34, T, n, base["n_actions"] + 1)   # the last code is out of range
    (ref_obs, ref_rew, ref_done, ref_prev, _), offs, ob = _trajectory(base, seeds, acts, "eager")
    tab32 = np.array([orc.norm_f32(b) for b in range(256)], np.float32).view(np.uint32)
    tab16 = np.array([orc.norm_bf16(b) for b in range(256)], np.uint16)
    first = None
    for mode in ("eager", "graph", "fused", "persistent", "eager-wpe", "fused-wpe"):
        out, offs_f, obf = _trajectory(cfg, seeds, acts, mode)
        if first is None:
            first = out
            assert np.array_equal(out[1], ref_rew) and np.array_equal(out[2], ref_done)
            assert np.array_equal(out[3], ref_prev)
            # every pixel of every step: the byte frame converted
            for t in range(T):
                for i in range(0, n, 7):
                    g8 = ref_obs[t * ob + offs[i]: t * ob + offs[i] + 64 * 64 * 3].reshape(64, 64, 3)
                    want = g8 if dtype == 0 else (tab16[g8] if dtype == 1 else tab32[g8])
                    raw = out[0][t * obf + offs_f[i]: t * obf + offs_f[i + 1]]
                    got = typed_hwc(raw, 64, 64, layout, dtype)
                    assert np.array_equal(got, want), f"step {t} env {i}"
            # previous actions follow the rule
            oc = orc.make_cfg(cfg)
            for t in range(T):
                for i in range(n):
                    assert out[3][t * n + i] == orc.prev_action(oc, int(acts[t, i]), int(out[2][t * n + i]))
            assert (out[2] == 1).sum() >= n               # episodes ended (cap 24) inside the window
        else:
            for k, name in enumerate(("obs", "reward", "done", "prev", "state")):
                assert np.array_equal(out[k], first[k]), f"{mode}: {name} differs"


def test_format_errors():
    import torch
    from paper_2605_19926_amd import jx
    base = W.TINY["cfg"]
    seeds = W.seeds(35, 4)
    # every configuration of one context must share the format
    e = jx.Env(seeds, [base, fmt_cfg(base, 1, 2)], cfg_index=[0, 1, 0, 1])
    with pytest.raises(jx.JxError):
        e.reset()
    e.close()
    e = U.env_of(fmt_cfg(base, 0, 2), seeds)
    ob = e.obs_bytes
    buf = torch.zeros(ob + 64, dtype=torch.uint8, device=e.dev)
    acts = torch.zeros(4, dtype=torch.uint8, device=e.dev)
    with pytest.raises(jx.JxError):
        e.step(acts, buf[4:4 + ob])                       # floating formats need 16-byte alignment
    e.step(acts, buf[16:16 + ob])
    frames = torch.zeros(2 * ob + 64, dtype=torch.uint8, device=e.dev)
    a2 = torch.zeros(8, dtype=torch.uint8, device=e.dev)
    r2 = torch.zeros(8, dtype=torch.float32, device=e.dev)
    d2 = torch.zeros(8, dtype=torch.uint8, device=e.dev)
    with pytest.raises(jx.JxError):
        e.rollout(a2, frames, r2, d2, 2, obs_stride=ob + 8, graph=False)
    with pytest.raises(jx.JxError):
        e.rollout(a2, frames, r2, d2, 2, obs_stride=ob, graph=False, prev=torch.zeros(7, dtype=torch.uint8,
                                                                                    device=e.dev))
    e.rollout(a2, frames, r2, d2, 2, obs_stride=ob, graph=False)
    torch.cuda.synchronize()
    e.close()
    # the serving API takes the default format only
    srv = jx.Server(device=0, hbm_budget=1 << 28, n_streams=1)
    try:
        with pytest.raises(jx.JxError):
            srv.open(seeds, fmt_cfg(base, 1, 0))
    finally:
        srv.close()
