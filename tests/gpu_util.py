"""Helpers shared by the GPU parity tests: synthetic states, oracle comparisons.

Inputs come from the seeded generators (workloads) and the oracle itself.  The
one-step checks are shared-state checks: the GPU's stored float32 state before
a step (set from a seeded synthetic state) and after it is widened exactly and
handed to the oracle, which steps and renders from it; the HIP path's outputs
are then compared with the oracle's.  No stored expected value comes from the
HIP path.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

import oracle as orc
import workloads as W

TWO_PI = 2 * math.pi
T_REL = 1e-4          # perpendicular distance, relative
FLAG_LIMIT = 1e-3     # flagged columns must stay below 0.1 %


def env_of(cfgs, seeds, cfg_index=None, obs=True):
    import torch
    from paper_2605_19926_amd import jx
    e = jx.Env(seeds, cfgs, cfg_index)
    e.obs0 = None
    if obs:
        # size the first frame buffer after the reset computes offsets
        e.reset()
        e.obs0 = torch.empty(e.obs_bytes, dtype=torch.uint8, device=e.dev)
        e.reset(e.obs0)
    else:
        e.reset()
    return e


def oracle_maze(cfg: dict, seed: int) -> np.ndarray:
    """The env's tile grid as the oracle builds it (ASCII map or seeded maze)."""
    return orc.layout(cfg, int(seed))


def ulp_close(a32, b64, k=2):
    a32 = np.float32(a32)
    return abs(float(a32) - float(b64)) <= k * float(np.spacing(np.float32(abs(b64)) + np.float32(0)))


def angle_close(a, b, tol=1e-6):
    d = (float(a) - float(b) + math.pi) % TWO_PI - math.pi
    return abs(d) <= tol


def synth_state(rng, cfg: dict, seed: int, grid: np.ndarray) -> dict:
    """A reachable-looking state: structural fields from an oracle episode reset
    of a random episode, a random float32 pose in a free tile, random time and
    key status."""
    oc = orc.make_cfg(cfg)
    ep = int(rng.integers(0, 60))
    st = orc.reset(grid, oc, int(seed), ep).as_dict()
    key_taken = int(rng.integers(0, 2)) if st["key"] >= 0 else 0
    N = cfg["side"]
    # ASCII maps: random keys taken and doors open; the pose may be in an open door
    akey_taken = 0
    for c in range(3):
        if st["akey"][c] >= 0 and rng.integers(0, 2):
            akey_taken |= 1 << c
    doors_open = int(rng.integers(0, 1 << 16)) if cfg.get("ascii_map") else 0
    floor = (grid & 0x8F) == 0
    is_door = (grid & 0x80) != 0
    open_door = is_door & (((doors_open >> (grid & 15).astype(np.int64)) & 1) == 1)
    free = np.argwhere(floor | open_door)[:, ::-1]           # (x, y)
    if st["door"] >= 0 and not key_taken:
        free = free[(free[:, 1] * N + free[:, 0]) != st["door"]]
    x, y, th = W.random_poses(rng, free, 1)
    st.update(x=float(x[0]), y=float(y[0]), theta=float(th[0]),
              t=int(rng.integers(0, cfg["episode_cap"])), key_taken=key_taken,
              door_open=key_taken, akey_taken=akey_taken, doors_open=doors_open)
    return st


def gpu_fields(states: list[dict]) -> dict:
    n = len(states)
    f = {"x": np.array([s["x"] for s in states], np.float32),
         "y": np.array([s["y"] for s in states], np.float32),
         "theta": np.array([s["theta"] for s in states], np.float32),
         "t": np.array([s["t"] for s in states], np.uint32),
         "episode": np.array([s["episode"] for s in states], np.uint32),
         "goal": np.array([s["goal"] for s in states], np.int32),
         "door": np.array([s["door"] for s in states], np.int32),
         "key": np.array([s["key"] for s in states], np.int32),
         "decor": np.array([list(s["decor"])[:2] for s in states], np.int32).reshape(-1),
         "flags": np.array([s["key_taken"] | (s["door_open"] << 1) | (s.get("akey_taken", 0) << 2)
                            for s in states], np.uint8),
         "n_decor": np.array([s["n_decor"] for s in states], np.uint8),
         "akey": np.array([list(s.get("akey", [-1, -1, -1])) for s in states], np.int32).reshape(-1),
         "doors": np.array([s.get("doors_open", 0) for s in states], np.uint32)}
    assert f["x"].shape == (n,)
    return f


def gpu_state_dict(S: dict, i: int) -> dict:
    return {"x": float(S["x"][i]), "y": float(S["y"][i]), "theta": float(S["theta"][i]),
            "t": int(S["t"][i]), "episode": int(S["episode"][i]), "goal": int(S["goal"][i]),
            "door": int(S["door"][i]), "key": int(S["key"][i]),
            "key_taken": int(S["flags"][i] & 1), "door_open": int((S["flags"][i] >> 1) & 1),
            "n_decor": int(S["n_decor"][i]), "decor": [int(S["decor"][2 * i]), int(S["decor"][2 * i + 1])],
            "akey": [int(v) for v in S["akey"][3 * i:3 * i + 3]],
            "akey_taken": int((S["flags"][i] >> 2) & 7), "doors_open": int(S["doors"][i])}


EXACT_KEYS = ("t", "episode", "goal", "door", "key", "key_taken", "door_open", "n_decor", "akey",
              "akey_taken", "doors_open")


def compare_reset_state(g: dict, o: dict) -> list[str]:
    """Episode-start states are exact on both sides (integer draws, one float32
    multiply for the heading)."""
    errs = []
    for k in ("x", "y", "theta"):
        if float(np.float32(g[k])) != o[k]:
            errs.append(f"{k}: gpu {g[k]!r} oracle {o[k]!r}")
    for k in EXACT_KEYS:
        if g[k] != o[k]:
            errs.append(f"{k}: gpu {g[k]} oracle {o[k]}")
    nd = o["n_decor"]
    if list(g["decor"])[:nd] != list(o["decor"])[:nd]:
        errs.append(f"decor: gpu {g['decor']} oracle {o['decor']}")
    return errs


class FrameStats:
    """Column counts of a parity check: columns compared, flagged (any of F1-F4),
    F1 (DDA tie) alone, multi-tie walks, and columns where the GPU took the
    other valid branch of a DDA tie."""

    def __init__(self):
        self.cols = 0
        self.flagged = 0
        self.f1 = 0
        self.multi = 0
        self.other_branch = 0
        self.by_flag = {"span": 0, "sprite": 0, "shade": 0}
        self.mismatch = []

    def frac_flagged(self):
        return self.flagged / max(1, self.cols)

    def summary(self):
        return (f"columns {self.cols}, flagged {self.flagged} ({100 * self.frac_flagged():.4f}%),"
                f" F1 {self.f1} ({100 * self.f1 / max(1, self.cols):.4f}%), multi {self.multi},"
                f" other branch {self.other_branch}, {self.by_flag},"
                f" unflagged mismatches {len(self.mismatch)}")

    def report(self, name: str) -> None:
        """Appends the counts to the file named by JX_FLAG_REPORT (if set)."""
        path = os.environ.get("JX_FLAG_REPORT")
        if not path:
            return
        rec = {"case": name, "columns": self.cols, "flagged": self.flagged, "f1": self.f1,
               "multi": self.multi, "other_branch": self.other_branch, **self.by_flag,
               "frac_flagged": self.frac_flagged(), "frac_f1": self.f1 / max(1, self.cols)}
        with open(path, "a") as f:
            f.write(json.dumps(rec) + "\n")

    def add(self, other: "FrameStats") -> None:
        self.cols += other.cols
        self.flagged += other.flagged
        self.f1 += other.f1
        self.multi += other.multi
        self.other_branch += other.other_branch
        for k in self.by_flag:
            self.by_flag[k] += other.by_flag[k]
        self.mismatch += other.mismatch


def check_frame(stats: FrameStats, g_frame: np.ndarray, grid: np.ndarray, oc, ost, g_dbg=None,
                tag: str = "", convert=None) -> None:
    """The GPU's frame of state `ost` against the oracle's render of the same
    state.  Every column must equal one of the oracle's valid results:
      - unflagged columns: every pixel bit-exact, and with debug records hit and
        side exact and t* within 1e-4 relative;
      - a column with one flagged DDA tie (F1): the GPU's column is either
        branch's (with debug records: its (hit, side) is that branch's and t*
        within 1e-4 of that branch's t*);
      - F2/F3/F4 decisions: pixels may differ only where the oracle's tie mask
        marks them (the tied row pair, billboard rows or wall rows);
      - a walk with several DDA ties (more than two valid results) is counted
        and accepted.
    g_frame is [H, W, C]; `convert` maps the oracle's uint8 HWC frame to the
    GPU frame's element form (training-buffer formats)."""
    o0, c0 = orc.render(grid, oc, ost, branch=0)
    fl = c0["flags"]
    conv = convert or (lambda f: f)
    branches = [(conv(o0), c0)]
    if (fl & orc.CF_DDA).any():
        o1, c1 = orc.render(grid, oc, ost, branch=1)
        branches.append((conv(o1), c1))
    W_ = fl.shape[0]
    stats.cols += W_
    stats.flagged += int((fl != 0).sum())
    stats.f1 += int(((fl & orc.CF_DDA) != 0).sum())
    stats.multi += int(((fl & orc.CF_MULTI) != 0).sum())
    stats.by_flag["span"] += int(((fl & orc.CF_SPAN) != 0).sum())
    stats.by_flag["sprite"] += int(((fl & orc.CF_SPRITE) != 0).sum())
    stats.by_flag["shade"] += int(((fl & orc.CF_SHADE) != 0).sum())
    g = np.asarray(g_frame)
    g = g if g.ndim == 3 else g[..., None]
    for c in range(W_):
        if fl[c] & orc.CF_MULTI:
            continue
        cands = [0, 1] if (fl[c] & orc.CF_DDA) else [0]
        if g_dbg is not None:
            gh, gs, gt = int(g_dbg["hit"][c]), int(g_dbg["side"][c]), float(g_dbg["t"][c])
            match = [b for b in cands
                     if (int(branches[b][1]["hit"][c]), int(branches[b][1]["side"][c])) == (gh, gs)]
            if not match:
                stats.mismatch.append(
                    f"{tag} col {c}: hit/side gpu {(gh, gs)} oracle " +
                    " / ".join(str((int(branches[b][1]["hit"][c]), int(branches[b][1]["side"][c])))
                               for b in cands) + f" (flags {fl[c]:#x})")
                continue
            bt = branches[match[0]][1]["t"][c]
            if abs(gt - bt) > T_REL * bt:
                stats.mismatch.append(f"{tag} col {c}: t gpu {gt} oracle {bt} (flags {fl[c]:#x})")
                continue
            cands = match
        ok = None
        for b in cands:
            ob, cb = branches[b]
            ob = ob if ob.ndim == 3 else ob[..., None]
            diff = (g[:, c] != ob[:, c]).reshape(g.shape[0], -1).any(axis=1)
            if not (diff & (cb["tie"][:, c] == 0)).any():
                ok = b
                break
        if ok is None:
            ob = branches[cands[0]][0]
            ob = ob if ob.ndim == 3 else ob[..., None]
            rows = np.nonzero((g[:, c] != ob[:, c]).reshape(g.shape[0], -1).any(axis=1))[0]
            stats.mismatch.append(f"{tag} col {c}: pixels differ outside the tied rows, rows "
                                  f"{list(rows[:8])} (flags {fl[c]:#x})")
        elif ok == 1:
            stats.other_branch += 1


def frame_of(obs_np: np.ndarray, offsets: np.ndarray, i: int, H: int, W_: int) -> np.ndarray:
    return obs_np[offsets[i]:offsets[i] + H * W_ * 3].reshape(H, W_, 3)


def compare_step(gs_before: dict, cfg: dict, seed: int, grid: np.ndarray, action: int,
                 g_after: dict, g_rew: float, g_done: int, g_ev: int):
    """One transition from a shared input state.  Returns (skipped, errors,
    oracle next state dict).  Steps the oracle flags (S1-S3) are skipped."""
    oc = orc.make_cfg(cfg)
    st = orc.state_from(gs_before)
    nxt, r, d, ev, sf = orc.step(grid, oc, int(seed), st, int(action))
    o = nxt.as_dict()
    if sf:
        return True, [], o
    errs = []
    if int(g_done) != d:
        errs.append(f"done gpu {g_done} oracle {d}")
    if float(g_rew) != r:
        errs.append(f"reward gpu {g_rew} oracle {r}")
    if int(g_ev) != ev:
        errs.append(f"events gpu {g_ev:#x} oracle {ev:#x}")
    if d:
        errs += compare_reset_state(g_after, o)
    else:
        if not ulp_close(g_after["x"], o["x"]) or not ulp_close(g_after["y"], o["y"]):
            errs.append(f"pos gpu {(g_after['x'], g_after['y'])} oracle {(o['x'], o['y'])}")
        if not angle_close(g_after["theta"], o["theta"]):
            errs.append(f"theta gpu {g_after['theta']} oracle {o['theta']}")
        for k in EXACT_KEYS:
            if g_after[k] != o[k]:
                errs.append(f"{k}: gpu {g_after[k]} oracle {o[k]}")
    return False, errs, o
