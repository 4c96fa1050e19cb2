"""Seeded synthetic workloads: the inputs both the HIP path and the oracle consume.

This module holds no arithmetic of the method (no stepping, casting, maze
generation or episode logic).  It defines the workload configurations,
per-environment seeds, uniform-random action streams, per-environment shape
draws for the mixed-shape batch, and the arrival trace of the serving workload.
All draws use numpy's PCG64 from fixed seeds.

The paper times a uniform random policy on a fixed maze (Appendix A.1); its
maps are not available, so seeded mazes generated from these seeds stand in.
"""
from __future__ import annotations

import math

import numpy as np

PI = math.pi

# Per-environment configuration fields, in the C-ABI struct's order.
CFG_FIELDS = ("side", "n_colors", "loop_frac", "key_door", "goal_sprite", "max_decor",
              "obs_h", "obs_w", "fov_deg", "n_actions", "episode_cap", "move", "turn",
              "pickup_radius", "r_goal", "r_key", "shade_levels", "shade_dist", "ascii_map",
              "obs_layout", "obs_dtype")


def env_cfg(**kw) -> dict:
    base = dict(side=16, n_colors=8, loop_frac=0.0, key_door=0, goal_sprite=0, max_decor=0,
                obs_h=64, obs_w=64, fov_deg=60.0, n_actions=6, episode_cap=512, move=0.1,
                turn=PI / 16, pickup_radius=0.3, r_goal=1.0, r_key=0.5, shade_levels=0,
                shade_dist=8.0, ascii_map=None, obs_layout=0, obs_dtype=0)
    for k in kw:
        if k not in base:
            raise KeyError(k)
    base.update(kw)
    return base


# The workloads: (number used to derive seeds, env count, steps, cfg).
TINY = dict(number=1, name="tiny-16env-8x8-64px", n_envs=16, steps=1000,
            cfg=env_cfg(side=8, n_colors=4, loop_frac=0.0, n_actions=4, episode_cap=256))
SCALE = dict(number=2, name="scale-4096env-16x16-64px", n_envs=4096, steps=10_240, warmup=128,
             cfg=env_cfg(side=16, n_colors=8, loop_frac=0.1, goal_sprite=1, n_actions=6,
                         episode_cap=512))
KEYDOOR = dict(number=3, name="keydoor-8192env-32x32-84px", n_envs=8192, steps=2048,
               cfg=env_cfg(side=32, n_colors=8, loop_frac=0.0, key_door=1, goal_sprite=1,
                           max_decor=2, obs_h=84, obs_w=84, n_actions=6, episode_cap=1024,
                           r_goal=1.0, r_key=0.5))
BATCH = dict(number=4, name="batch-16384env-mixed", n_envs=16384, rollout=128)
# A 16x16 map in the paper's ASCII format (Table 2), written for this
# repository: five rooms joined by a red-locked, a blue-locked and a yellow-locked
# door and two unlocked doors, the three keys, spawn and goal candidates and
# coloured walls.
MAP16 = "\n".join([
    "################",
    "#S....1..#....G#",
    "#.....1..#.....#",
    "#..r.....R..y..#",
    "#.....1..#.....#",
    '##"#######\\#####',
    "#......#.......#",
    "#.2222.#..S....#",
    "#.2..2.B.......#",
    "#.2222.#...b...#",
    "#......#.......#",
    "####Y#######.###",
    "#..............#",
    "#.S.....33...G.#",
    "#..............#",
    "################",
])

# A 10x10 map with every symbol, for oracle-scale trajectories.
MAP10 = "\n".join([
    "##########",
    "#S..1...G#",
    "#.##1#.#.#",
    '#..r"..R.#',
    "####.###.#",
    "#b..B..\\.#",
    "#.######.#",
    "#y...2...#",
    "#S...9.GY#",
    "##########",
])

SERVE = dict(number=5, name="serve-256clients-poisson2000", clients=256, rate=2000.0,
             min_envs=1, max_envs=512, min_side=8, max_side=64, obs=(64, 84),
             mean_session=64)

WORKLOADS = {w["name"]: w for w in (TINY, SCALE, KEYDOOR, BATCH, SERVE)}


ASCII = dict(number=6, name="ascii-4096env-16x16-64px", n_envs=4096, steps=2560, warmup=128,
             cfg=env_cfg(side=16, ascii_map=MAP16, goal_sprite=1, n_actions=6, episode_cap=512,
                         obs_h=64, obs_w=64))
ASCII_TINY = dict(number=7, name="ascii-16env-10x10-64px", n_envs=16, steps=400,
                  cfg=env_cfg(side=10, ascii_map=MAP10, goal_sprite=1, n_actions=4, episode_cap=128,
                              obs_h=64, obs_w=64))


# Long rays: a 64x64 room walled only at its border (rays cross up to ~90
# tiles), and the 64-side maze with every separator wall removed (a hall of
# pillars, long rays between them).
ROOM64 = "\n".join(["#" * 64] + ["#" + "." * 62 + "#"] * 62 + ["#" * 64])
OPEN64 = dict(number=8, name="open-32env-64x64room-128px", n_envs=32,
              cfg=env_cfg(side=64, ascii_map=ROOM64, goal_sprite=1, n_actions=6, episode_cap=256,
                          obs_h=128, obs_w=128))
PILLARS64 = dict(number=9, name="pillars-32env-64side-128px", n_envs=32,
                 cfg=env_cfg(side=64, loop_frac=1.0, goal_sprite=1, n_actions=6, episode_cap=256,
                             obs_h=128, obs_w=128))


def seeds(number: int, n: int, offset: int = 0) -> np.ndarray:
    """seeds[i] = (number << 32) | (offset + i), as uint64."""
    i = np.arange(offset, offset + n, dtype=np.uint64)
    return (np.uint64(number) << np.uint64(32)) | i


def actions(number: int, steps: int, n: int, n_actions: int, stream: int = 0) -> np.ndarray:
    """Uniform random actions [steps, n] uint8 (the paper's uniform random policy)."""
    rng = np.random.Generator(np.random.PCG64([number, 0xAC710, stream]))
    return rng.integers(0, n_actions, size=(steps, n), dtype=np.uint8)


def batch_cfgs(n: int, number: int = BATCH["number"]):
    """Mixed shapes for the batched form: map side from {8,16,32,64}, frame from
    {32,64,128} square, key-door on a random half.  Returns (cfg list, index[n])."""
    rng = np.random.Generator(np.random.PCG64([number, 0xC0F16]))
    sides = rng.choice(np.array([8, 16, 32, 64]), size=n)
    obs = rng.choice(np.array([32, 64, 128]), size=n)
    kd = rng.integers(0, 2, size=n)
    table: dict[tuple, int] = {}
    cfgs: list[dict] = []
    idx = np.zeros(n, np.int32)
    for i in range(n):
        key = (int(sides[i]), int(obs[i]), int(kd[i]))
        if key not in table:
            table[key] = len(cfgs)
            if key[2]:
                c = env_cfg(side=key[0], n_colors=8, loop_frac=0.0, key_door=1, goal_sprite=1,
                            max_decor=2, obs_h=key[1], obs_w=key[1], n_actions=6,
                            episode_cap=1024)
            else:
                c = env_cfg(side=key[0], n_colors=8, loop_frac=0.1, goal_sprite=1,
                            obs_h=key[1], obs_w=key[1], n_actions=6, episode_cap=512)
            cfgs.append(c)
        idx[i] = table[key]
    return cfgs, idx


def serve_trace(n_requests: int, number: int = SERVE["number"], clients: int = SERVE["clients"],
                rate: float = SERVE["rate"], max_envs: int = SERVE["max_envs"],
                mean_session: float = SERVE["mean_session"]):
    """Open-loop arrival trace for the serving workload.

    Requests arrive as a Poisson process of `rate` per second over `clients`
    slots (slot chosen uniformly).  Each slot hosts a session of geometric length
    (mean `mean_session` requests); when it ends a new client takes the slot with
    a fresh env count (log-uniform in [1, max_envs]), map side (uniform integer in
    [8, 64]) and frame (64 or 84 square, equally likely).

    Returns a dict of arrays: t (arrival seconds), slot, session (global session
    id), and per-session n_envs, side, obs, seed_base.
    """
    rng = np.random.Generator(np.random.PCG64([number, 0x5E77E]))
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    t = np.cumsum(gaps)
    slot = rng.integers(0, clients, size=n_requests)
    sess_of_slot = -np.ones(clients, np.int64)
    left = np.zeros(clients, np.int64)
    session = np.zeros(n_requests, np.int64)
    s_n, s_side, s_obs = [], [], []

    def new_session():
        n = int(np.clip(math.floor(math.exp(rng.uniform() * math.log(max_envs + 1))), 1, max_envs))
        s_n.append(n)
        s_side.append(int(rng.integers(SERVE["min_side"], SERVE["max_side"] + 1)))
        s_obs.append(int(SERVE["obs"][int(rng.integers(0, 2))]))
        return len(s_n) - 1

    for k in range(n_requests):
        c = slot[k]
        if left[c] <= 0:
            sess_of_slot[c] = new_session()
            left[c] = int(rng.geometric(1.0 / mean_session))
        session[k] = sess_of_slot[c]
        left[c] -= 1
    n_sess = len(s_n)
    return {"t": t, "slot": slot, "session": session,
            "n_envs": np.array(s_n, np.int32), "side": np.array(s_side, np.int32),
            "obs": np.array(s_obs, np.int32),
            "seed_base": seeds(number, n_sess) << np.uint64(12)}


def random_poses(rng: np.random.Generator, free_tiles: np.ndarray, n: int):
    """n random float32 poses: a uniformly chosen free tile, a uniform point
    inside it, a uniform heading in [0, 2pi).  Returns (x, y, theta) float32."""
    pick = free_tiles[rng.integers(0, len(free_tiles), size=n)]
    fx = pick[:, 0].astype(np.float64) + rng.uniform(0.0, 1.0, size=n)
    fy = pick[:, 1].astype(np.float64) + rng.uniform(0.0, 1.0, size=n)
    x = np.float32(fx)
    y = np.float32(fy)
    # keep float32 rounding inside the chosen tile
    x = np.minimum(np.maximum(x, pick[:, 0].astype(np.float32)),
                   np.nextafter(pick[:, 0].astype(np.float32) + 1, np.float32(0)))
    y = np.minimum(np.maximum(y, pick[:, 1].astype(np.float32)),
                   np.nextafter(pick[:, 1].astype(np.float32) + 1, np.float32(0)))
    th = np.float32(rng.uniform(0.0, 2 * math.pi, size=n))
    th = np.where(th >= np.float32(2 * math.pi), np.float32(0), th).astype(np.float32)
    return x.astype(np.float32), y.astype(np.float32), th
