"""Pins for the oracle's ASCII map front-end (Table 2 symbols): parsed tile
bytes and errors, spawn and goal candidates (uniform draws, BFS fallback
against scipy), unlocked doors that open when walked into, locked doors opened
by the key of their colour only, the colours of coloured walls and doors, and
a key billboard straight ahead.  The maps are written for these tests.  CPU
only."""
import math

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path
from scipy.stats import chisquare

import workloads as W

DOOR, SPAWN, GOAL = 0x80, 0x20, 0x40

# a 10x10 map with every symbol of Table 2
FULL = "\n".join([
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


def cfg_for(text, side, **kw):
    return W.env_cfg(side=side, ascii_map=text, n_colors=8, obs_h=64, obs_w=64, **kw)


def test_parse_tile_bytes(orc):
    g, keys, n_doors = orc.ascii_layout(FULL, 12)
    assert n_doors == 5
    assert g[0, 0] == 1 and g[1, 4] == 2 + 0                     # '#', '1'
    assert g[7, 5] == 2 + 1 and g[8, 5] == 2 + 8                  # '2', '9'
    assert g[1, 1] == SPAWN and g[8, 1] == SPAWN and g[1, 8] == GOAL and g[8, 7] == GOAL
    assert g[1, 2] == 0 and g[3, 3] == 0                          # floor, key tile is floor
    # doors in row-major order: '"' (3,4) blue unlocked, 'R' (3,7), 'B' (5,4), '\' (5,7), 'Y' (8,8)
    assert g[3, 4] == DOOR | (3 << 4) | 0
    assert g[3, 7] == DOOR | (0 << 4) | 1
    assert g[5, 4] == DOOR | (1 << 4) | 2
    assert g[5, 7] == DOOR | (4 << 4) | 3
    assert g[8, 8] == DOOR | (2 << 4) | 4
    assert keys == [3 * 12 + 3, 5 * 12 + 1, 7 * 12 + 1]          # r, b, y
    assert (g[10:, :] == 1).all() and (g[:, 10:] == 1).all()     # beyond the text: walls


@pytest.mark.parametrize("text,code", [
    ("#####\n#.x.#\n#####", -2),            # unknown symbol
    ("#" * 9, -3),                          # wider than N = 8
    ("#####\n#r.r#\n#####", -5),            # two red keys
    ("#####\n#####\n#####", -6),            # no floor
    ("#" + '"' * 17 + "#\n#.#", -4),        # 17 doors
])
def test_parse_errors(orc, text, code):
    N = 8 if code == -3 else 20
    with pytest.raises(ValueError, match=f"\\({code}\\)"):
        orc.ascii_layout(text, N)


def test_spawn_and_goal_candidates_uniform(orc):
    cfg = orc.make_cfg(cfg_for(FULL, 10))
    g, _, _ = orc.ascii_layout(FULL, 10)
    spawns, goals = [], []
    for ep in range(1200):
        s = orc.reset(g, cfg, 99, ep)
        spawns.append((int(s.y), int(s.x)))
        goals.append(s.goal)
        assert s.akey_taken == 0 and s.doors_open == 0 and list(s.akey) == [33, 51, 71]
    assert set(spawns) == {(1, 1), (8, 1)}
    assert set(goals) == {1 * 10 + 8, 8 * 10 + 7}
    assert chisquare([spawns.count((1, 1)), spawns.count((8, 1))]).pvalue > 1e-3
    assert chisquare([goals.count(18), goals.count(87)]).pvalue > 1e-3


def test_goal_without_candidates_is_bfs_farthest_through_doors(orc):
    text = "\n".join(["#########",
                      "#S..R...#",
                      "#.#######",
                      "#...\"...#",
                      "#########"])
    N = 9
    cfg = orc.make_cfg(cfg_for(text, N))
    g, _, _ = orc.ascii_layout(text, N)
    passable = ((g & 0x8F) == 0) | ((g & DOOR) != 0)
    idx = np.arange(N * N).reshape(N, N)
    rows, cols = [], []
    for y in range(N):
        for x in range(N):
            if not passable[y, x]:
                continue
            for dy, dx in ((0, 1), (1, 0)):
                if y + dy < N and x + dx < N and passable[y + dy, x + dx]:
                    rows += [idx[y, x], idx[y + dy, x + dx]]
                    cols += [idx[y + dy, x + dx], idx[y, x]]
    A = csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(N * N, N * N))
    for ep in range(20):
        s = orc.reset(g, cfg, 5, ep)
        spawn = int(s.y) * N + int(s.x)
        assert spawn == 1 * N + 1                              # the only S
        d = shortest_path(A, unweighted=True, indices=spawn)
        d[~np.isfinite(d)] = -1
        far = d.max()
        assert d[s.goal] == far and s.goal == int(np.nonzero(d == far)[0].min())


def state_at(orc, x, y, th, akey=(-1, -1, -1), taken=0, doors=0, goal=-1):
    return orc.state_from(dict(x=x, y=y, theta=th, t=0, episode=0, goal=goal, door=-1, key=-1,
                               key_taken=0, door_open=0, n_decor=0, decor=[-1, -1],
                               akey=list(akey), akey_taken=taken, doors_open=doors))


CORRIDOR = "\n".join(["##########",
                      '#..."..R.#',
                      "##########"])


def test_unlocked_door_opens_when_walked_into(orc):
    cfg = orc.make_cfg(cfg_for(CORRIDOR, 10, n_actions=4, move=0.25))
    g, _, _ = orc.ascii_layout(CORRIDOR, 10)
    s = state_at(orc, 3.8, 1.5, 0.0)                           # facing east, door at x = 4
    nx, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)               # forward: bumps the door
    assert nx.x == 3.8 and (ev & 0x01) and (ev & 0x80) and nx.doors_open == 1
    nx2, _, _, ev2, _ = orc.step(g, cfg, 1, nx, 0)              # forward again: passes
    assert abs(nx2.x - 4.05) < 1e-12 and not (ev2 & 0x01) and nx2.doors_open == 1
    # the red-locked door (index 1) is not opened by walking into it
    s = state_at(orc, 6.8, 1.5, 0.0, doors=1)
    nx, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)
    assert nx.x == 6.8 and (ev & 0x01) and not (ev & 0x80) and nx.doors_open == 1


def test_key_opens_only_doors_of_its_colour(orc):
    text = "\n".join(["###########",
                      "#.b.B.R.Y.#",
                      "###########"])
    cfg = orc.make_cfg(cfg_for(text, 11, n_actions=4, move=0.1))
    g, keys, nd = orc.ascii_layout(text, 11)
    assert nd == 3 and keys == [-1, 11 + 2, -1]
    s = state_at(orc, 2.15, 1.5, 0.0, akey=keys)               # 0.35 from the key centre
    nx, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)               # to 2.25: within 0.3
    assert (ev & 0x04) and (ev & 0x80) and r == np.float32(0.5)
    assert nx.akey_taken == 0b010 and nx.doors_open == 0b001   # blue door (index 0) only
    nx2, r2, _, ev2, _ = orc.step(g, cfg, 1, nx, 0)
    assert r2 == 0 and not (ev2 & 0x04)                        # taken once


def test_wall_and_door_colours(orc):
    text = "\n".join(["#######",
                      "#.....3",
                      '#.....\\',
                      '#....."',
                      "#######"])
    N = 8
    cfg = orc.make_cfg(cfg_for(text, N))
    g, _, _ = orc.ascii_layout(text, N)
    # facing east from x = 2.5: rows 1, 2, 3 end at column 6 with '3', yellow
    # unlocked door, blue unlocked door (x-faces, no side darkening)
    for y, rgb in ((1.5, (40, 60, 180)), (2.5, (230, 200, 60)), (3.5, (70, 110, 230))):
        obs, cols = orc.render(g, cfg, state_at(orc, 2.5, y, 0.0))
        c = 31
        assert cols["hit"][c] == int(y) * N + 6 and cols["side"][c] == 0 and cols["flags"][c] == 0
        assert tuple(obs[32, c]) == rgb
    # an open door is floor: the ray passes to the wall behind it (column 7)
    obs, cols = orc.render(g, cfg, state_at(orc, 2.5, 3.5, 0.0, doors=0b10))
    assert cols["hit"][31] == 3 * N + 7


def test_key_billboard_straight_ahead(orc):
    text = "\n".join(["##########",
                      "#.....y..#",
                      "##########"])
    N = 10
    cfg = orc.make_cfg(cfg_for(text, N))
    g, keys, _ = orc.ascii_layout(text, N)
    s = state_at(orc, 2.5, 1.5, 0.0, akey=keys)                # yellow key 4 tiles ahead
    obs, cols = orc.render(g, cfg, s)
    W_, H = 64, 64
    tanH = math.tan(math.radians(30))
    hw = (W_ / 2) * 0.25 / (tanH * 4.0)                        # 3.46 columns
    hs = H * 0.25 / 4.0                                        # 4 rows
    assert tuple(obs[32, 32]) == (255, 200, 40) and tuple(obs[32, 31]) == (255, 200, 40)
    assert tuple(obs[32, 32 + int(hw) + 1]) != (255, 200, 40)
    assert tuple(obs[32 - int(hs) - 1, 32]) != (255, 200, 40)
    taken = state_at(orc, 2.5, 1.5, 0.0, akey=keys, taken=0b100)
    obs2, _ = orc.render(g, cfg, taken)
    assert tuple(obs2[32, 32]) != (255, 200, 40)
