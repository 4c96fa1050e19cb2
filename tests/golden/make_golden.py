"""Writes oracle_regression.json: oracle outputs for a few fixed inputs.

Calls only the oracle (and the seeded workload definitions).  The file guards
the oracle against unintended edits; it holds no value from the HIP path.
Run: python tests/golden/make_golden.py
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_regression.json")


def sha(b: bytes) -> str:
    return hashlib.sha256(b).hexdigest()[:32]


def build() -> dict:
    out = {"mazes": [], "resets": [], "frames": [], "rollouts": []}
    for seed, N, lf in ((0, 8, 0.0), (1, 16, 0.1), (7, 32, 0.0), (9, 64, 0.1), (2**63 + 3, 17, 0.1)):
        g = oracle.maze(seed, N, lf)
        out["mazes"].append({"seed": seed, "side": N, "loop_frac": lf, "sha": sha(g.tobytes())})
    for wl in (W.TINY, W.SCALE, W.KEYDOOR):
        cfg = oracle.make_cfg(wl["cfg"])
        seeds = W.seeds(wl["number"], 3)
        for s in seeds:
            s = int(s)
            g = oracle.maze(s, cfg.side, cfg.loop_frac)
            for ep in (0, 3):
                st = oracle.reset(g, cfg, s, ep)
                out["resets"].append({"workload": wl["name"], "seed": s, "episode": ep,
                                      "state": st.as_dict()})
                obs, cols = oracle.render(g, cfg, st)
                out["frames"].append({"workload": wl["name"], "seed": s, "episode": ep,
                                      "sha": sha(obs.tobytes()),
                                      "hit": cols["hit"].tolist()[:8]})
        n, T = 4, 300
        acts = W.actions(wl["number"], T, n, cfg.n_actions)
        steps, last = oracle.rollout(cfg, W.seeds(wl["number"], n), acts, want_obs=True)
        out["rollouts"].append({"workload": wl["name"], "n": n, "T": T, "steps": int(steps),
                                "sha": sha(last.tobytes())})
    return out


if __name__ == "__main__":
    with open(OUT, "w") as f:
        json.dump(build(), f, indent=1, sort_keys=True)
    print("wrote", OUT)
