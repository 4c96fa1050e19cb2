"""Pins for the oracle's distance shading (the render option that scales a wall
column's colour by its hit distance): hand-derived colours at known distances,
the floor rounding, the level cap, identity for S = 0 and S = 1, monotonic
darkening with distance, the side darkening applied first, and the F4 flag on
a level boundary.  CPU only."""
import math

import numpy as np
import pytest

import workloads as W


def room(N):
    g = np.ones((N, N), np.uint8)
    g[1:N - 1, 1:N - 1] = 0
    return g


def st(orc, x, y, th):
    return orc.state_from(dict(x=x, y=y, theta=th, t=0, episode=0, goal=-1, door=-1, key=-1,
                               key_taken=0, door_open=0, n_decor=0, decor=[-1, -1]))


def centre_row(orc, N, x, y, th, **kw):
    cfg = orc.make_cfg(W.env_cfg(side=N, n_colors=1, obs_h=64, obs_w=64, **kw))
    obs, cols = orc.render(room(N), cfg, st(orc, x, y, th))
    return obs[32], cols


# Facing east (theta = 0) in an empty 16x16 room every column hits the east wall
# (x = 15, an x-face, palette colour 0 = (180, 40, 40) with one colour) at
# t* = 15 - x exactly.
@pytest.mark.parametrize("x,levels,dist,rgb", [
    (10.0, 4, 8.0, (90, 20, 20)),     # t* 5: q = 2.5, level 2, 2/4 of each channel
    (13.5, 4, 8.0, (180, 40, 40)),    # t* 1.5: level 0, unchanged
    (1.5, 4, 8.0, (45, 10, 10)),      # t* 13.5: past D, capped at level 3, 1/4
    (11.5, 3, 6.0, (120, 26, 26)),    # t* 3.5: q = 1.75, level 1, 2/3 rounded down (40*2/3 = 26.67)
    (6.0, 5, 10.0, (36, 8, 8)),       # t* 9: q = 4.5, the last level, 1/5
])
def test_wall_colour_at_known_distance(orc, x, levels, dist, rgb):
    row, cols = centre_row(orc, 16, x, 8.5, 0.0, shade_levels=levels, shade_dist=dist)
    ok = (cols["flags"] == 0) & (cols["side"] == 0)   # far away the FOV edges reach other walls
    assert ok.sum() > 40
    assert (cols["t"][ok] == 15 - x).all()
    assert (row[ok] == np.array(rgb, np.uint8)).all()


@pytest.mark.parametrize("levels", [0, 1])
def test_zero_and_one_level_are_the_unshaded_frame(orc, levels):
    rng = np.random.default_rng(3 + levels)
    N = 16
    base_cfg = orc.make_cfg(W.env_cfg(side=N, obs_h=64, obs_w=64))
    cfg = orc.make_cfg(W.env_cfg(side=N, obs_h=64, obs_w=64, shade_levels=levels, shade_dist=2.0))
    g = orc.maze(77, N, 0.1)
    free = np.argwhere(g == 0)
    for _ in range(10):
        ty, tx = free[rng.integers(len(free))]
        s = st(orc, tx + rng.uniform(0.1, 0.9), ty + rng.uniform(0.1, 0.9), rng.uniform(0, 2 * math.pi))
        a, _ = orc.render(g, base_cfg, s)
        b, _ = orc.render(g, cfg, s)
        assert np.array_equal(a, b)


def test_darkening_is_monotonic_in_distance(orc):
    last = None
    for x in np.arange(14.75, 1.0, -0.25):        # t* = 15 - x grows
        row, cols = centre_row(orc, 16, float(x), 8.5, 0.0, shade_levels=8, shade_dist=12.0)
        v = int(row[32].astype(int).sum())
        if last is not None:
            assert v <= last
        last = v
    assert last == (180 // 8) + (40 // 8) * 2      # capped at the last level


def test_side_darkening_comes_first(orc):
    # facing north (theta = 3 pi / 2): the middle columns hit the north wall (a
    # y-face) at t* = y - 1 = 5.5; side darkening halves (180, 40, 40) to
    # (90, 20, 20), then level floor(5.5 * 4 / 8) = 2 keeps 2/4 of it
    row, cols = centre_row(orc, 16, 8.5, 6.5, 1.5 * math.pi, shade_levels=4, shade_dist=8.0)
    for c in (31, 32):
        assert cols["side"][c] == 1 and cols["flags"][c] == 0
        assert tuple(row[c]) == (45, 10, 10)


def test_level_boundary_is_flagged(orc):
    # t* = 15 - 11 = 4 and S / D = 3 / 6: q = 2 exactly, a level boundary
    _, cols = centre_row(orc, 16, 11.0, 8.5, 0.0, shade_levels=3, shade_dist=6.0)
    assert (cols["flags"] & 0x10).all()
    _, cols = centre_row(orc, 16, 11.5, 8.5, 0.0, shade_levels=3, shade_dist=6.0)
    assert not (cols["flags"] & 0x10).any()
