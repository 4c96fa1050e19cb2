"""Pins for the oracle's decision-window flags and its acceptance data: each
flag is set by a state built exactly on its boundary and clear just outside
the window, and the tie mask and the second branch mark exactly the pixels and
the walk a tied decision can change.  The windows are this implementation's
reading of the DDA's exact ties (Sec. 2.1 marches along tile boundaries, so a
ray through a tile corner crosses both grid lines at one parameter).  CPU only."""
import math

import numpy as np

import workloads as W

CEIL = (50, 50, 60)
FLOOR = (90, 80, 70)
GOAL = (255, 230, 0)
DECOR = (0, 200, 120)
TAN_H = math.tan(math.pi / 6)
R32 = float(np.float32(0.3))          # pickup radius as the configuration holds it


def room(N):
    g = np.ones((N, N), np.uint8)
    g[1:N - 1, 1:N - 1] = 0
    return g


def cfg_of(orc, **kw):
    return orc.make_cfg(W.env_cfg(**kw))


def st(orc, x, y, th, **kw):
    d = dict(x=x, y=y, theta=th, t=0, episode=0, goal=-1, door=-1, key=-1, key_taken=0,
             door_open=0, n_decor=0, decor=[-1, -1])
    d.update(kw)
    return orc.state_from(d)


# ---- F1: DDA ties ------------------------------------------------------------

# The ray from (2.5, 2.75) along (2, 1) passes exactly through the tile
# corners (3, 3) at t = 0.25 and (5, 4) at t = 1.25, then enters the wall tile
# (6, 4) through its x-face at t = 1.75, away from any corner.
X0, Y0, RX, RY = 2.5, 2.75, 2.0, 1.0


def corner_room():
    g = room(8)
    g[4, 6] = 1                                   # tile (6, 4)
    return g


def test_f1_corner_between_free_tiles_not_flagged(orc):
    # Around both corners every tile is free: the two orders of crossing reach
    # the same diagonal tile at the same parameter, so either gives one result.
    g = corner_room()
    hit, side, t, fl = orc.cast(g, -1, 1, X0, Y0, RX, RY)
    assert fl == 0
    assert hit == 4 * 8 + 6 and side == 0 and t == 1.75


def test_f1_blocker_beside_corner_flagged(orc):
    g = corner_room()
    g[2, 3] = 1                                   # tile (3, 2): the x-first side of corner (3, 3)
    hit, side, t, fl = orc.cast(g, -1, 1, X0, Y0, RX, RY)
    assert fl & orc.CF_DDA and not fl & orc.CF_MULTI
    # ties cross y first: into (2, 3), then x into (3, 3): the walk goes on
    assert hit == 4 * 8 + 6 and t == 1.75


def test_f1_window_edges(orc):
    # Tilting the ray moves the crossing parameters at corner (3, 3) apart by
    # a relative eps: inside the 1e-5 window for 5e-6, outside for 5e-5.
    g = corner_room()
    g[2, 3] = 1
    for eps, flagged in ((5e-6, True), (-5e-6, True), (5e-5, False), (-5e-5, False)):
        hit, side, t, fl = orc.cast(g, -1, 1, X0, Y0, RX, RY * (1.0 + eps))
        assert bool(fl & orc.CF_DDA) == flagged, (eps, fl)


def test_f1_two_ties_marked_multi(orc):
    g = corner_room()
    g[2, 3] = 1                                   # beside corner (3, 3)
    g[3, 5] = 1                                   # tile (5, 3): beside corner (5, 4)
    hit, side, t, fl = orc.cast(g, -1, 1, X0, Y0, RX, RY)
    assert fl & orc.CF_DDA and fl & orc.CF_MULTI
    g[2, 3] = 0
    hit, side, t, fl = orc.cast(g, -1, 1, X0, Y0, RX, RY)
    assert fl & orc.CF_DDA and not fl & orc.CF_MULTI


def test_f1_multi_in_a_rendered_column(orc):
    # the same two corners seen by a camera looking along (2, 1) with a field
    # of view so small that every column's ray is within rounding of that line
    g = corner_room()
    g[2, 3] = 1
    g[3, 5] = 1
    cfg = cfg_of(orc, side=8, obs_w=4, obs_h=8, fov_deg=1e-6)
    obs, c = orc.render(g, cfg, st(orc, X0, Y0, math.atan2(RY, RX)))
    # (rounding decides on which side of the first corner each ray passes: the
    # walks that go on past it meet the second tie)
    assert ((c["flags"] & orc.CF_DDA) != 0).all()
    assert (((c["flags"] & orc.CF_MULTI) != 0) == (c["t"] > 1.0)).all() and (c["t"] > 1.0).any()
    g[3, 5] = 0
    obs, c = orc.render(g, cfg, st(orc, X0, Y0, math.atan2(RY, RX)))
    assert not (c["flags"] & orc.CF_MULTI).any() and ((c["flags"] & orc.CF_DDA) != 0).all()


def test_branch_one_renders_the_other_side_of_the_tie(orc):
    # One column looking exactly through a corner next to a blocker: branch 0
    # crosses y first (enters (2, 3), then the free (3, 3), ...); branch 1 crosses
    # x first into the blocker (3, 2) at t = 0.5 through its x-face.
    N = 8
    g = room(N)
    g[2, 3] = 1
    cfg = cfg_of(orc, side=N, obs_w=4, obs_h=8, fov_deg=1e-6)
    s = st(orc, 2.5, 2.5, math.pi / 4)
    o0, c0 = orc.render(g, cfg, s, branch=0)
    o1, c1 = orc.render(g, cfg, s, branch=1)
    for c in range(4):
        assert c0["flags"][c] & orc.CF_DDA
        assert (c1["hit"][c], c1["side"][c]) == (c0["alt_hit"][c], c0["alt_side"][c])
        assert c1["t"][c] == c0["alt_t"][c]
    # heading pi/4 and the tiny field of view put every ray within rounding of
    # the corner, so which walk is branch 0 is a rounding matter: one of the two
    # enters the blocker (3, 2) through its x-face at t = 0.5 sqrt(2), the other
    # goes on past the corner
    for c in range(4):
        walks = {(int(c0["hit"][c]), int(c0["side"][c])): (c0["t"][c], o0[:, c]),
                 (int(c1["hit"][c]), int(c1["side"][c])): (c1["t"][c], o1[:, c])}
        assert len(walks) == 2
        t_near, col_near = walks.pop((2 * N + 3, 0))
        (t_far, col_far), = walks.values()
        assert abs(t_near - 0.5 * math.sqrt(2)) < 1e-6 and t_far > 1.0
        # the blocker at perpendicular distance 0.707 fills the whole 8-row column
        assert not any(tuple(p) in (CEIL, FLOOR) for p in col_near)
        assert tuple(col_far[0]) == CEIL


def test_branches_equal_on_columns_without_f1(orc):
    rng = np.random.default_rng(4)
    N = 16
    cfg = cfg_of(orc, side=N, loop_frac=0.1, goal_sprite=1)
    n_f1 = 0
    for k in range(30):
        g = orc.maze(500 + k, N, 0.1)
        free = np.argwhere(g == 0)
        ty, tx = free[rng.integers(len(free))]
        gy, gx = free[rng.integers(len(free))]
        # half the states stand on a tile corner looking along a diagonal
        if k % 2:
            x, y, th = float(tx), float(ty), (math.pi / 4) * (1 + 2 * rng.integers(4))
        else:
            x, y, th = tx + rng.uniform(0.05, 0.95), ty + rng.uniform(0.05, 0.95), rng.uniform(0, 2 * math.pi)
        s = st(orc, x, y, th, goal=int(gy * N + gx))
        o0, c0 = orc.render(g, cfg, s, branch=0)
        o1, c1 = orc.render(g, cfg, s, branch=1)
        f1 = (c0["flags"] & orc.CF_DDA) != 0
        n_f1 += int(f1.sum())
        same = ~f1
        assert (o0[:, same] == o1[:, same]).all()
        assert (c0["hit"][same] == c1["hit"][same]).all()
    assert n_f1 > 0


# ---- F2: span edge on a pixel centre -----------------------------------------

def test_f2_span_edge_on_pixel_centre(orc):
    # Facing the flat east wall of a 16-room from x = 7: t* = 8 on every column,
    # so with H = 120 the half-height H/(2t*) = 7.5 lies on the centre of the
    # row pair at distance 7 (rows 52 and 67), which the strict rule leaves out.
    N, H, Wd = 16, 120, 64
    cfg = cfg_of(orc, side=N, obs_h=H, obs_w=Wd)
    obs, c = orc.render(room(N), cfg, st(orc, 7.0, 8.5, 0.0))
    assert (c["t"] == 8.0).all()
    assert (c["flags"] == orc.CF_SPAN).all()
    tie_rows = np.nonzero(c["tie"].any(axis=1))[0]
    assert list(tie_rows) == [52, 67]
    assert (c["tie"][[52, 67]] == 1).all()
    assert all(tuple(obs[52, k]) == CEIL and tuple(obs[67, k]) == FLOOR for k in range(Wd))
    assert all(tuple(obs[53, k]) not in (CEIL, FLOOR) for k in range(Wd))
    # t* scaled by 1 +- 2e-5 moves hh by 1.5e-4, twice the window: not flagged
    for s_ in (1 + 2e-5, 1 - 2e-5):
        obs2, c2 = orc.render(room(N), cfg, st(orc, 15.0 - 8.0 * s_, 8.5, 0.0))
        assert (c2["flags"] == 0).all() and not c2["tie"].any()
    # 1 +- 5e-6 is inside
    obs3, c3 = orc.render(room(N), cfg, st(orc, 15.0 - 8.0 * (1 + 5e-6), 8.5, 0.0))
    assert (c3["flags"] == orc.CF_SPAN).all()


# ---- F3: billboards ------------------------------------------------------------

def _ahead(orc, d, H=64, Wd=64, **kw):
    """Facing +x in a 16-room with the goal billboard straight ahead at depth d."""
    N = 16
    cfg = cfg_of(orc, side=N, goal_sprite=1, obs_h=H, obs_w=Wd, **kw)
    gx, gy = 12, 8
    return orc.render(room(N), cfg, st(orc, gx + 0.5 - d, gy + 0.5, 0.0, goal=gy * N + gx))


def test_f3_horizontal_edge_on_column_centre(orc):
    # half-width (W/2) 0.25 / (tanH d) = 4.5 puts the edges u -+ hw = 27.5, 36.5
    # on the centres of columns 27 and 36 (u = 32 straight ahead)
    d = 32 * 0.25 / (TAN_H * 4.5)
    obs, c = _ahead(orc, d)
    flagged = np.nonzero(c["flags"] & orc.CF_SPRITE)[0]
    assert list(flagged) == [27, 36]
    hs = 64 * 0.25 / d
    rows = [r for r in range(64) if abs(r + 0.5 - 32) < hs]
    for col in (27, 36):
        assert list(np.nonzero(c["tie"][:, col])[0]) == rows
    assert not c["tie"][:, 28:36].any() and not c["tie"][:, :27].any()
    goal_cols = np.nonzero((obs == np.array(GOAL, np.uint8)).all(-1).any(0))[0]
    assert list(goal_cols) == list(range(28, 36))
    # hw = 4.5 -+ 0.01: no column edge inside the window
    for hw in (4.49, 4.51):
        obs2, c2 = _ahead(orc, 32 * 0.25 / (TAN_H * hw))
        assert not (c2["flags"] & orc.CF_SPRITE).any()


def test_f3_vertical_edge_on_row_centre(orc):
    # half-height H 0.25 / d = 5.5 at d = 64 * 0.25 / 5.5: the row pair at
    # distance 5 (rows 26 and 37) is tied on every covered column
    d = 64 * 0.25 / 5.5
    obs, c = _ahead(orc, d)
    covered = np.nonzero((obs == np.array(GOAL, np.uint8)).all(-1).any(0))[0]
    assert len(covered) > 0
    for col in covered:
        assert c["flags"][col] & orc.CF_SPRITE
        assert list(np.nonzero(c["tie"][:, col])[0]) == [26, 37]
    rows = np.nonzero((obs[:, covered[0]] == np.array(GOAL, np.uint8)).all(-1))[0]
    assert list(rows) == list(range(27, 37))        # strict: rows 26 and 37 left out
    obs2, c2 = _ahead(orc, 64 * 0.25 / 5.52)
    assert not (c2["flags"] & orc.CF_SPRITE).any()


def test_f3_near_clip(orc):
    # A decor billboard 0.05 ahead (the clip depth) is tied on every column it
    # would cover; at 0.06 it is drawn and not tied.
    N = 16
    cfg = cfg_of(orc, side=N, key_door=1, max_decor=2, obs_h=64, obs_w=64)
    dx, dy = 9, 8
    for dist, tied in ((0.05, True), (0.05 + 5e-6, True), (0.05 - 5e-6, True),
                       (0.05 + 2e-5, False), (0.05 - 2e-5, False), (0.06, False), (0.04, False)):
        s = st(orc, dx + 0.5 - dist, dy + 0.5, 0.0, n_decor=1, decor=[dy * N + dx, -1])
        obs, c = orc.render(room(N), cfg, s)
        f3 = (c["flags"] & orc.CF_SPRITE) != 0
        assert f3.all() == tied and (f3.any() == tied), dist
        shown = (obs == np.array(DECOR, np.uint8)).all(-1).any()
        if not tied:
            assert shown == (dist > 0.05)
        else:
            assert c["tie"].all()                 # the billboard would cover every pixel


def test_f3_two_billboards_at_one_depth(orc):
    # Two sprite slots on the same tile (a constructed state): equal depth, the
    # painter shows the later slot (goal after key), and the covered pixels
    # are tied.
    N = 16
    cfg = cfg_of(orc, side=N, goal_sprite=1, key_door=1, obs_h=64, obs_w=64)
    tile = 8 * N + 11
    s = st(orc, 7.5, 8.5, 0.0, goal=tile, key=tile, door=1 * N + 14)
    obs, c = orc.render(room(N), cfg, s)
    goal_px = (obs == np.array(GOAL, np.uint8)).all(-1)
    assert goal_px.any()
    cols = np.nonzero(goal_px.any(0))[0]
    for col in cols:
        assert c["flags"][col] & orc.CF_SPRITE
        assert (c["tie"][goal_px[:, col], col] == 1).all()
    # key and goal on neighbouring tiles at the same depth never overlap
    # (their centres are 1 apart laterally, the billboards 0.5 wide)
    s2 = st(orc, 7.5, 8.5, 0.0, goal=8 * N + 11, key=9 * N + 11, door=1 * N + 14)
    obs2, c2 = orc.render(room(N), cfg, s2)
    assert not (c2["flags"] & orc.CF_SPRITE).any()


def test_zero_depth_gap_unreachable(orc):
    # A billboard at a tile centre is at least 0.5 from every grid line and
    # 0.25 wide, so on a column it covers the wall it is compared with lies at
    # least 0.25 cos(30 deg) deeper or nearer: the z-test never falls in its
    # window for the sprites this library draws.
    rng = np.random.default_rng(12)
    N = 16
    cfg = cfg_of(orc, side=N, goal_sprite=1, key_door=1, max_decor=2, loop_frac=0.1)
    tanH = TAN_H
    worst = math.inf
    for k in range(120):
        g = orc.maze(900 + k, N, 0.1)
        free = np.argwhere(g == 0)
        picks = free[rng.choice(len(free), 5, replace=False)]
        (ay, ax), *sp = picks
        x, y, th = ax + rng.uniform(0.02, 0.98), ay + rng.uniform(0.02, 0.98), rng.uniform(0, 2 * math.pi)
        tiles = [int(b * N + a) for b, a in sp]
        s = st(orc, x, y, th, key=tiles[0], goal=tiles[1], door=-1, n_decor=2, decor=tiles[2:])
        obs, c = orc.render(g, cfg, s)
        cs, sn = math.cos(th), math.sin(th)
        for tid in tiles:
            dx, dy = tid % N + 0.5 - x, tid // N + 0.5 - y
            tY, tX = dx * cs + dy * sn, -dx * sn + dy * cs
            if tY <= 0.05:
                continue
            u = 32 * (1 + tX / (tanH * tY))
            hw = 32 * 0.25 / (tanH * tY)
            for col in range(64):
                if abs(col + 0.5 - u) < hw:
                    worst = min(worst, abs(c["t"][col] - tY))
    assert worst >= 0.25 * math.cos(math.pi / 6) - 1e-12


def test_tie_mask_empty_on_unflagged_columns(orc):
    rng = np.random.default_rng(21)
    for wl in (W.SCALE, W.KEYDOOR):
        cfg = cfg_of(orc, **{k: v for k, v in wl["cfg"].items()})
        cfg_d = wl["cfg"]
        for k in range(12):
            g = orc.layout(cfg_d, 77 + k)
            o = orc.reset(g, cfg, 77 + k, int(rng.integers(0, 9)))
            free = np.argwhere(g == 0)
            ty, tx = free[rng.integers(len(free))]
            o.x, o.y = tx + rng.uniform(0.01, 0.99), ty + rng.uniform(0.01, 0.99)
            o.theta = rng.uniform(0, 2 * math.pi)
            obs, c = orc.render(g, cfg, o)
            clear = c["flags"] == 0
            assert not c["tie"][:, clear].any()
            # columns flagged only for a DDA tie have no tied pixel: the other
            # branch accounts for them
            f1_only = c["flags"] == orc.CF_DDA
            assert not c["tie"][:, f1_only].any()


# ---- step flags ------------------------------------------------------------------

def test_s2_pickup_radius_window(orc):
    N = 8
    g = room(N)
    cfg = cfg_of(orc, side=N, n_actions=4, key_door=1)
    key = 4 * N + 3                                  # centre (3.5, 4.5)
    r2 = R32 * R32
    for delta, flagged, picked in ((5e-6, True, False), (-5e-6, True, True),
                                   (2e-5, False, False), (-2e-5, False, True)):
        x = 3.5 + math.sqrt(r2 + delta)
        s = st(orc, x, 4.5, 0.0, key=key, door=1 * N + 6)
        s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 2)          # a turn: the pose stays
        assert bool(sf & orc.SF_KEY) == flagged, delta
        assert bool(ev & orc.EV_KEY) == picked, delta


def test_s3_goal_edge_window(orc):
    N = 8
    g = room(N)
    cfg = cfg_of(orc, side=N, n_actions=4)
    gx, gy = 5, 3
    goal = gy * N + gx
    for x, flagged, reached in ((gx - 5e-6, True, False), (gx + 5e-6, True, True),
                                (gx - 2e-5, False, False), (gx + 2e-5, False, True),
                                (gx + 1 - 5e-6, True, True), (gx + 1 + 5e-6, True, False)):
        s = st(orc, x, gy + 0.5, 0.0, goal=goal)
        s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 2)
        assert bool(sf & orc.SF_GOAL) == flagged, x
        assert bool(ev & orc.EV_GOAL) == reached, x
    # y edges
    for y, flagged, reached in ((gy - 5e-6, True, False), (gy + 5e-6, True, True),
                                (gy + 2e-5, False, True)):
        s = st(orc, gx + 0.5, y, 0.0, goal=goal)
        s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 2)
        assert bool(sf & orc.SF_GOAL) == flagged, y
        assert bool(ev & orc.EV_GOAL) == reached, y
    # an edge point away from the cell (outside its other extent) is not flagged
    s = st(orc, gx - 5e-6, gy + 2.5, 0.0, goal=goal)
    assert orc.step(g, cfg, 1, s, 2)[4] == 0


def test_s1_collision_window_only_where_passability_changes(orc):
    N = 8
    g = room(N)
    cfg = cfg_of(orc, side=N, n_actions=4)
    m = float(np.float32(0.1))
    # landing 3e-6 short of the wall face: flagged; 3e-5 short: not
    assert orc.step(g, cfg, 1, st(orc, 7.0 - m - 3e-6, 3.5, 0.0), 0)[4] & orc.SF_MOVE
    assert not orc.step(g, cfg, 1, st(orc, 7.0 - m - 3e-5, 3.5, 0.0), 0)[4] & orc.SF_MOVE
    # landing on a grid line between two free tiles: the outcome does not change
    assert orc.step(g, cfg, 1, st(orc, 4.0 - m - 3e-6, 3.5, 0.0), 0)[4] == 0
