"""GPU: the C-ABI from a C++ caller with no Python (paper_2605_19926_amd/jx_demo):
its figures (reward sum, done count, FNV-1a of the last step's frames after a
fused rollout) equal those of the same workload driven through the Python
binding."""
import os
import subprocess

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEMO = os.path.join(ROOT, "paper_2605_19926_amd", "jx_demo")


def splitmix64(x: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        x = x + np.uint64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return x ^ (x >> np.uint64(31))


def fnv1a(b: bytes) -> int:
    h = 0xCBF29CE484222325
    for v in b:
        h = ((h ^ v) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def test_cpp_caller_matches_binding():
    import torch
    from paper_2605_19926_amd import jx
    assert os.path.exists(DEMO), "jx_demo is built with the library"
    n, T = 256, 600          # past the episode cap (512): every env resets once
    out = subprocess.run([DEMO, str(n), str(T)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    f = out.stdout.split()
    got = dict(zip(f[0::2], f[1::2]))
    cfg = W.env_cfg(side=16, n_colors=8, loop_frac=0.1, goal_sprite=1, n_actions=6, episode_cap=512,
                    obs_h=64, obs_w=64)
    seeds = (np.uint64(7) << np.uint64(32)) | np.arange(n, dtype=np.uint64)
    idx = (np.arange(T, dtype=np.uint64)[:, None] * np.uint64(n) + np.arange(n, dtype=np.uint64)[None, :]
           + np.uint64(1))
    acts = (splitmix64(idx) % np.uint64(6)).astype(np.uint8)
    env = jx.Env(seeds, cfg)
    env.reset()
    ob = env.obs_bytes
    obs = torch.empty(T * ob, dtype=torch.uint8, device=env.dev)
    rew = torch.empty(T * n, dtype=torch.float32, device=env.dev)
    done = torch.empty(T * n, dtype=torch.uint8, device=env.dev)
    env.rollout(torch.from_numpy(acts).to(env.dev), obs, rew, done, T, obs_stride=ob, graph=False, fused=True)
    torch.cuda.synchronize()
    r = rew.cpu().numpy().astype(np.float64)
    d = done.cpu().numpy()
    last = obs[(T - 1) * ob:].cpu().numpy().tobytes()
    env.close()
    assert int(got["envs"]) == n and int(got["steps"]) == T
    assert f"{r.sum():.1f}" == got["reward_sum"]
    assert int(d.sum()) == int(got["dones"])
    assert f"{fnv1a(last):016x}" == got["last_frames_fnv1a"]
    assert float(got["env_steps_per_s"]) > 0
    assert int(d.sum()) >= n
