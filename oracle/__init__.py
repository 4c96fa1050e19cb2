"""FP64 CPU oracle for the batched first-person step and raycast render.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2605_19926_amd``) never imports it and shares no code with it.

The C source (``jx_oracle.c``) holds the rules; this module is argument
marshalling over ctypes plus :func:`build`.  What the paper (JAXenstein) fixes:
one ray per image column to the first wall, found by DDA marching over tile
boundaries (Sec. 2.1); tile-map worlds (Sec. 2.2, Sec. 3.2, Table 2); fixed
billboard sprites (Fig. 1).  Everything else is a stated reading, written next
to each C function.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "jx_oracle.c")
_LIB = os.path.join(_HERE, "libjxoracle.so")

EV_BLOCKED_X, EV_BLOCKED_Y, EV_KEY, EV_GOAL = 0x01, 0x02, 0x04, 0x08
EV_TRUNC, EV_INVALID, EV_RESET = 0x10, 0x20, 0x40
EV_DOOR = 0x80
TILE_DOOR, TILE_SPAWN, TILE_GOAL = 0x80, 0x20, 0x40
SF_MOVE, SF_KEY, SF_GOAL = 0x01, 0x02, 0x04
CF_DDA, CF_SPAN, CF_SPRITE, CF_MULTI, CF_SHADE = 0x01, 0x02, 0x04, 0x08, 0x10
MAX_DECOR = 2


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (IEEE arithmetic, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcCfg(ctypes.Structure):
    _fields_ = [("side", ctypes.c_int32), ("n_colors", ctypes.c_int32),
                ("loop_frac", ctypes.c_double), ("key_door", ctypes.c_int32),
                ("goal_sprite", ctypes.c_int32), ("max_decor", ctypes.c_int32),
                ("obs_h", ctypes.c_int32), ("obs_w", ctypes.c_int32),
                ("fov_deg", ctypes.c_double), ("n_actions", ctypes.c_int32),
                ("episode_cap", ctypes.c_int32), ("move", ctypes.c_double),
                ("turn", ctypes.c_double), ("pickup_radius", ctypes.c_double),
                ("r_goal", ctypes.c_double), ("r_key", ctypes.c_double),
                ("shade_levels", ctypes.c_int32), ("shade_dist", ctypes.c_double),
                ("ascii_map", ctypes.c_char_p)]


class OrcState(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("y", ctypes.c_double), ("theta", ctypes.c_double),
                ("t", ctypes.c_int32), ("episode", ctypes.c_int32),
                ("goal", ctypes.c_int32), ("door", ctypes.c_int32), ("key", ctypes.c_int32),
                ("key_taken", ctypes.c_int32), ("door_open", ctypes.c_int32),
                ("n_decor", ctypes.c_int32), ("decor", ctypes.c_int32 * MAX_DECOR),
                ("akey", ctypes.c_int32 * 3), ("akey_taken", ctypes.c_int32),
                ("doors_open", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"x": self.x, "y": self.y, "theta": self.theta, "t": self.t,
                "episode": self.episode, "goal": self.goal, "door": self.door,
                "key": self.key, "key_taken": self.key_taken, "door_open": self.door_open,
                "n_decor": self.n_decor, "decor": list(self.decor),
                "akey": list(self.akey), "akey_taken": self.akey_taken,
                "doors_open": self.doors_open}


_FLOAT_FIELDS = ("loop_frac", "fov_deg", "move", "turn", "pickup_radius", "r_goal", "r_key",
                 "shade_dist")


def make_cfg(d: dict) -> OrcCfg:
    """Configuration struct; float fields take the float32 value, widened exactly."""
    c = OrcCfg()
    for name, _ in OrcCfg._fields_:
        if name == "ascii_map":
            m = d.get("ascii_map")
            c.ascii_map = None if m is None else m.encode("ascii")
            continue
        v = d[name]
        if name in _FLOAT_FIELDS:
            setattr(c, name, float(np.float32(v)))
        else:
            setattr(c, name, int(v))
    return c


def state_from(d: dict) -> OrcState:
    s = OrcState()
    for k in ("x", "y", "theta"):
        setattr(s, k, float(d[k]))
    for k in ("t", "episode", "goal", "door", "key", "key_taken", "door_open", "n_decor"):
        setattr(s, k, int(d[k]))
    dec = list(d.get("decor", [-1] * MAX_DECOR)) + [-1] * MAX_DECOR
    for j in range(MAX_DECOR):
        s.decor[j] = int(dec[j])
    ak = list(d.get("akey", [-1, -1, -1]))
    for c in range(3):
        s.akey[c] = int(ak[c])
    s.akey_taken = int(d.get("akey_taken", 0))
    s.doors_open = int(d.get("doors_open", 0))
    return s


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.orc_rng_next.argtypes = [u64p]
        L.orc_rng_next.restype = ctypes.c_uint64
        L.orc_mix64.argtypes = [ctypes.c_uint64]
        L.orc_mix64.restype = ctypes.c_uint64
        L.orc_rng_range.argtypes = [u64p, ctypes.c_uint32]
        L.orc_rng_range.restype = ctypes.c_uint32
        L.orc_maze.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_double, u8p]
        L.orc_maze.restype = ctypes.c_int32
        L.orc_reset.argtypes = [u8p, ctypes.POINTER(OrcCfg), ctypes.c_uint64, ctypes.c_int32,
                                ctypes.POINTER(OrcState)]
        L.orc_reset.restype = ctypes.c_int32
        L.orc_step.argtypes = [u8p, ctypes.POINTER(OrcCfg), ctypes.c_uint64,
                               ctypes.POINTER(OrcState), ctypes.c_int32,
                               ctypes.POINTER(OrcState), f64p, i32p, i32p, i32p]
        L.orc_step.restype = ctypes.c_int32
        L.orc_step_w.argtypes = L.orc_step.argtypes + [ctypes.c_double]
        L.orc_step_w.restype = ctypes.c_int32
        L.orc_render.argtypes = [u8p, ctypes.POINTER(OrcCfg), ctypes.POINTER(OrcState), u8p,
                                 i32p, i32p, f64p, i32p, i32p, i32p, f64p]
        L.orc_render.restype = ctypes.c_int32
        L.orc_render_ex.argtypes = [u8p, ctypes.POINTER(OrcCfg), ctypes.POINTER(OrcState),
                                    ctypes.c_int32, u8p, i32p, i32p, f64p, i32p, i32p, i32p, f64p, u8p]
        L.orc_render_ex.restype = ctypes.c_int32
        L.orc_cast.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, i32p, f64p, i32p]
        L.orc_cast.restype = ctypes.c_int32
        L.orc_ascii.argtypes = [ctypes.c_char_p, ctypes.c_int32, u8p, ctypes.POINTER(ctypes.c_int32)]
        L.orc_ascii.restype = ctypes.c_int32
        L.orc_rollout.argtypes = [ctypes.POINTER(OrcCfg), ctypes.c_int32, u64p, ctypes.c_int32,
                                  u8p, u8p, ctypes.POINTER(ctypes.c_int64)]
        L.orc_rollout.restype = ctypes.c_int64
        L.orc_norm_f32.argtypes = [ctypes.c_int32]
        L.orc_norm_f32.restype = ctypes.c_float
        L.orc_norm_bf16.argtypes = [ctypes.c_int32]
        L.orc_norm_bf16.restype = ctypes.c_uint16
        L.orc_format_frame.argtypes = [u8p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_void_p]
        L.orc_format_frame.restype = ctypes.c_int64
        L.orc_prev_action.argtypes = [ctypes.POINTER(OrcCfg), ctypes.c_int32, ctypes.c_int32]
        L.orc_prev_action.restype = ctypes.c_int32
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ---- random numbers ---------------------------------------------------------
def rng_stream(seed: int, count: int) -> list[int]:
    s = ctypes.c_uint64(seed & (2**64 - 1))
    return [lib().orc_rng_next(ctypes.byref(s)) for _ in range(count)]


def mix64(v: int) -> int:
    return lib().orc_mix64(v & (2**64 - 1))


def rng_range(state: int, n: int) -> tuple[int, int]:
    """One draw in [0, n); returns (value, new_state)."""
    s = ctypes.c_uint64(state & (2**64 - 1))
    v = lib().orc_rng_range(ctypes.byref(s), n)
    return v, s.value


# ---- layout / episodes -------------------------------------------------------
def maze(seed: int, side: int, loop_frac: float) -> np.ndarray:
    g = np.zeros((side, side), np.uint8)
    k = lib().orc_maze(seed & (2**64 - 1), side, float(np.float32(loop_frac)), _p(g, ctypes.c_uint8))
    if k < 0:
        raise ValueError("bad maze arguments")
    return g


def ascii_layout(text: str, side: int):
    """(grid [side, side] tile bytes, keys (r, b, y tile ids, -1 absent), doors)
    of an ASCII map; raises ValueError with the parser's code on error."""
    g = np.zeros((side, side), np.uint8)
    k = (ctypes.c_int32 * 3)()
    n = lib().orc_ascii(text.encode("ascii"), side, _p(g, ctypes.c_uint8), k)
    if n < 0:
        raise ValueError(f"ascii map rejected ({n})")
    return g, list(k), n


def layout(cfg: dict, seed: int) -> np.ndarray:
    """The env's tile grid: its ASCII map when the configuration has one, else
    the seeded maze."""
    if cfg.get("ascii_map") is not None:
        return ascii_layout(cfg["ascii_map"], cfg["side"])[0]
    return maze(seed, cfg["side"], cfg["loop_frac"])


def maze_loops(seed: int, side: int, loop_frac: float) -> int:
    g = np.zeros((side, side), np.uint8)
    return lib().orc_maze(seed & (2**64 - 1), side, float(np.float32(loop_frac)), _p(g, ctypes.c_uint8))


def reset(grid: np.ndarray, cfg: OrcCfg, seed: int, episode: int) -> OrcState:
    g = np.ascontiguousarray(grid, np.uint8)
    out = OrcState()
    rc = lib().orc_reset(_p(g, ctypes.c_uint8), ctypes.byref(cfg), seed & (2**64 - 1), episode,
                         ctypes.byref(out))
    if rc != 0:
        raise ValueError("reset failed")
    return out


def step(grid: np.ndarray, cfg: OrcCfg, seed: int, state: OrcState, action: int,
         window: float = 1e-5):
    """Returns (next_state, reward, done, events, step_flags); the step flags
    mark decisions within `window` of their boundary."""
    g = np.ascontiguousarray(grid, np.uint8)
    out = OrcState()
    r = ctypes.c_double()
    d, ev, sf = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    rc = lib().orc_step_w(_p(g, ctypes.c_uint8), ctypes.byref(cfg), seed & (2**64 - 1),
                          ctypes.byref(state), int(action), ctypes.byref(out), ctypes.byref(r),
                          ctypes.byref(d), ctypes.byref(ev), ctypes.byref(sf), float(window))
    if rc != 0:
        raise ValueError("step failed")
    return out, r.value, d.value, ev.value, sf.value


def render(grid: np.ndarray, cfg: OrcCfg, state: OrcState, branch: int = 0):
    """Returns (obs[H,W,3] uint8, per-column dict: hit, side, t, flags, alt_hit,
    alt_side, alt_t, and tie[H,W]: 1 where the pixel is decided inside a
    window).  branch 1 renders every flagged DDA tie's other side."""
    g = np.ascontiguousarray(grid, np.uint8)
    H, W = cfg.obs_h, cfg.obs_w
    obs = np.zeros((H, W, 3), np.uint8)
    cols = {"hit": np.zeros(W, np.int32), "side": np.zeros(W, np.int32),
            "t": np.zeros(W, np.float64), "flags": np.zeros(W, np.int32),
            "alt_hit": np.zeros(W, np.int32), "alt_side": np.zeros(W, np.int32),
            "alt_t": np.zeros(W, np.float64), "tie": np.zeros((H, W), np.uint8)}
    rc = lib().orc_render_ex(_p(g, ctypes.c_uint8), ctypes.byref(cfg), ctypes.byref(state),
                             int(branch), _p(obs, ctypes.c_uint8), _p(cols["hit"], ctypes.c_int32),
                             _p(cols["side"], ctypes.c_int32), _p(cols["t"], ctypes.c_double),
                             _p(cols["flags"], ctypes.c_int32), _p(cols["alt_hit"], ctypes.c_int32),
                             _p(cols["alt_side"], ctypes.c_int32), _p(cols["alt_t"], ctypes.c_double),
                             _p(cols["tie"], ctypes.c_uint8))
    if rc != 0:
        raise ValueError("render failed")
    return obs, cols


def cast(grid: np.ndarray, door: int, door_open: int, x: float, y: float, rx: float, ry: float):
    """Single ray; returns (hit, side, t, flags)."""
    g = np.ascontiguousarray(grid, np.uint8)
    side = ctypes.c_int32()
    t = ctypes.c_double()
    fl = ctypes.c_int32()
    hit = lib().orc_cast(_p(g, ctypes.c_uint8), g.shape[0], door, door_open, x, y, rx, ry,
                         ctypes.byref(side), ctypes.byref(t), ctypes.byref(fl))
    return hit, side.value, t.value, fl.value


def rollout(cfg: OrcCfg, seeds: np.ndarray, actions: np.ndarray, want_obs: bool = False,
            counts: bool = False):
    """Steps len(seeds) envs through actions[T, n]; returns (env_steps, last_obs
    or None), and with counts=True a third item: {columns, flagged, f1,
    steps_flagged} over every rendered frame."""
    seeds = np.ascontiguousarray(seeds, np.uint64)
    actions = np.ascontiguousarray(actions, np.uint8)
    n = seeds.shape[0]
    T = actions.shape[0]
    assert actions.shape == (T, n)
    last = np.zeros((n, cfg.obs_h, cfg.obs_w, 3), np.uint8) if want_obs else None
    cnt = np.zeros(4, np.int64)
    done = lib().orc_rollout(ctypes.byref(cfg), n, _p(seeds, ctypes.c_uint64), T,
                             _p(actions, ctypes.c_uint8),
                             _p(last, ctypes.c_uint8) if want_obs else None,
                             _p(cnt, ctypes.c_int64) if counts else None)
    if counts:
        return done, last, {"columns": int(cnt[0]), "flagged": int(cnt[1]), "f1": int(cnt[2]),
                            "steps_flagged": int(cnt[3])}
    return done, last


# ---- training-buffer formats --------------------------------------------------
OBS_NHWC, OBS_NCHW = 0, 1
OBS_U8, OBS_BF16, OBS_F32 = 0, 1, 2
_FMT_NP = {OBS_U8: np.uint8, OBS_BF16: np.uint16, OBS_F32: np.float32}


def norm_f32(b: int) -> float:
    return float(lib().orc_norm_f32(int(b)))


def norm_bf16(b: int) -> int:
    """Bit pattern of b / 255 rounded to bfloat16."""
    return int(lib().orc_norm_bf16(int(b)))


def format_frame(hwc: np.ndarray, layout: int, dtype: int) -> np.ndarray:
    """The frame hwc[H, W, 3] in a training-buffer format: shape (H, W, 3) for
    NHWC or (3, H, W) for NCHW; uint8, bfloat16 bit patterns (uint16) or float32."""
    f = np.ascontiguousarray(hwc, np.uint8)
    H, W, _ = f.shape
    out = np.zeros((H, W, 3) if layout == OBS_NHWC else (3, H, W), _FMT_NP[dtype])
    n = lib().orc_format_frame(_p(f, ctypes.c_uint8), H, W, layout, dtype,
                               out.ctypes.data_as(ctypes.c_void_p))
    if n != out.nbytes:
        raise ValueError("bad format arguments")
    return out


def prev_action(cfg: OrcCfg, action: int, done: int) -> int:
    return int(lib().orc_prev_action(ctypes.byref(cfg), int(action), int(done)))


def tan_half_fov(cfg: OrcCfg) -> float:
    return math.tan(cfg.fov_deg * math.pi / 360.0)
