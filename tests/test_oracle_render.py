"""Pins for the oracle's raycast and frame: closed forms in an empty room, a flat
wall, column heights, mirror and rotation invariants, a brute-force marcher, and
sprite closed forms plus a per-pixel nearest-sprite renderer.  CPU only."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.march import march

CEIL = (50, 50, 60)
FLOOR = (90, 80, 70)
GOAL = (255, 230, 0)


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


def rays(cfg, th):
    W_, tanH = cfg.obs_w, math.tan(cfg.fov_deg * math.pi / 360)
    c, s = math.cos(th), math.sin(th)
    out = []
    for col in range(W_):
        cam = (2 * col + 1 - W_) / W_
        out.append((c + cam * tanH * (-s), s + cam * tanH * c))
    return out


@pytest.mark.parametrize("N", [8, 13, 16])
def test_empty_room_closed_form(orc, N):
    rng = np.random.default_rng(N)
    cfg = cfg_of(orc, side=N, obs_w=64, obs_h=64)
    g = room(N)
    checked = 0
    for _ in range(60):
        x, y = rng.uniform(1.01, N - 1.01, size=2)
        th = rng.uniform(0, 2 * math.pi)
        obs, cols = orc.render(g, cfg, st(orc, x, y, th))
        for col, (rx, ry) in enumerate(rays(cfg, th)):
            if cols["flags"][col]:
                continue
            tx = ((N - 1 if rx > 0 else 1) - x) / rx if rx != 0 else math.inf
            ty = ((N - 1 if ry > 0 else 1) - y) / ry if ry != 0 else math.inf
            t = min(tx, ty)
            side = 0 if tx < ty else 1
            if side == 0:
                hit = (int(math.floor(y + t * ry)), N - 1 if rx > 0 else 0)
            else:
                hit = (N - 1 if ry > 0 else 0, int(math.floor(x + t * rx)))
            assert cols["side"][col] == side
            assert cols["hit"][col] == hit[0] * N + hit[1]
            assert abs(cols["t"][col] - t) <= 1e-12 * max(1.0, t)
            checked += 1
    assert checked > 60 * 60


@pytest.mark.parametrize("x", [13.25, 12.0625, 14.5])
def test_flat_wall_constant_distance(orc, x):
    N = 16
    cfg = cfg_of(orc, side=N)
    obs, cols = orc.render(room(N), cfg, st(orc, x, 8.5, 0.0))
    assert (cols["side"] == 0).all()
    assert (cols["t"] == (N - 1) - x).all()                 # bitwise identical, all columns
    assert (cols["hit"] % N == N - 1).all()


def wall_rows(obs_col):
    return sum(1 for px in obs_col if tuple(px) not in (CEIL, FLOOR))


@pytest.mark.parametrize("H,Wd", [(64, 64), (84, 84), (32, 32), (128, 128), (64, 32)])
def test_column_height_closed_form(orc, H, Wd):
    rng = np.random.default_rng(H + Wd)
    N = 16
    cfg = cfg_of(orc, side=N, obs_h=H, obs_w=Wd, loop_frac=0.1)
    g = orc.maze(H * 7 + Wd, N, 0.1)
    free = np.argwhere(g == 0)
    for _ in range(25):
        ty, tx = free[rng.integers(len(free))]
        x, y = tx + rng.uniform(0.02, 0.98), ty + rng.uniform(0.02, 0.98)
        obs, cols = orc.render(g, cfg, st(orc, x, y, rng.uniform(0, 2 * math.pi)))
        for col in range(Wd):
            if cols["flags"][col]:
                continue
            hh = H / (2 * cols["t"][col])
            expect = 2 * min(max(math.ceil(hh - 0.5), 0), H // 2)
            assert wall_rows(obs[:, col]) == expect
            col_px = [tuple(p) for p in obs[:, col]]
            # wall band is centred on the horizon
            rows = [r for r in range(H) if col_px[r] not in (CEIL, FLOOR)]
            if rows:
                assert rows[0] + rows[-1] == H - 1


def mirrored_cases(orc, N, seed):
    g = orc.maze(seed, N, 0.1)
    rng = np.random.default_rng(seed)
    free = np.argwhere(g == 0)
    ty, tx = free[rng.integers(len(free))]
    return g, tx + rng.uniform(0.05, 0.95), ty + rng.uniform(0.05, 0.95), rng.uniform(0, 2 * math.pi)


@pytest.mark.parametrize("seed", range(12))
def test_mirror_and_rotation_invariants(orc, seed):
    N = 16
    cfg = cfg_of(orc, side=N, n_colors=1, loop_frac=0.1)
    Wd = cfg.obs_w
    g, x, y, th = mirrored_cases(orc, N, seed)
    obs, c0 = orc.render(g, cfg, st(orc, x, y, th))

    def tid(t):
        return t % N, t // N

    # reflect x
    gx = g[:, ::-1].copy()
    obsx, cx = orc.render(gx, cfg, st(orc, N - x, y, (math.pi - th) % (2 * math.pi)))
    # reflect y
    gy = g[::-1, :].copy()
    obsy, cy = orc.render(gy, cfg, st(orc, x, N - y, (-th) % (2 * math.pi)))
    # rotate by +90 degrees: tile (a, b) -> (N-1-b, a), point (x, y) -> (N-y, x)
    gr = np.zeros_like(g)
    for b in range(N):
        for a in range(N):
            gr[a, N - 1 - b] = g[b, a]
    obsr, cr = orc.render(gr, cfg, st(orc, N - y, x, (th + math.pi / 2) % (2 * math.pi)))
    n_ok = 0
    for col in range(Wd):
        m = Wd - 1 - col
        a, b = tid(c0["hit"][col])
        if not (c0["flags"][col] or cx["flags"][m]):
            assert tid(cx["hit"][m]) == (N - 1 - a, b)
            assert cx["side"][m] == c0["side"][col]
            assert abs(cx["t"][m] - c0["t"][col]) <= 1e-9 * c0["t"][col]
            assert (obsx[:, m] == obs[:, col]).all()
            n_ok += 1
        if not (c0["flags"][col] or cy["flags"][m]):
            assert tid(cy["hit"][m]) == (a, N - 1 - b)
            assert cy["side"][m] == c0["side"][col]
            assert abs(cy["t"][m] - c0["t"][col]) <= 1e-9 * c0["t"][col]
            assert (obsy[:, m] == obs[:, col]).all()
        if not (c0["flags"][col] or cr["flags"][col]):
            assert tid(cr["hit"][col]) == (N - 1 - b, a)
            assert cr["side"][col] == 1 - c0["side"][col]
            assert abs(cr["t"][col] - c0["t"][col]) <= 1e-9 * c0["t"][col]
    assert n_ok > Wd // 2


def corner_distance(x, y):
    return math.hypot(x - round(x), y - round(y))


@pytest.mark.parametrize("N", [8, 16])
def test_brute_force_marcher_agrees(orc, N):
    rng = np.random.default_rng(100 + N)
    checked = 0
    for seed in range(6):
        g = orc.maze(seed + 50 * N, N, 0.1)
        free = np.argwhere(g == 0)
        for _ in range(30):
            ty, tx = free[rng.integers(len(free))]
            x, y = tx + rng.uniform(0.01, 0.99), ty + rng.uniform(0.01, 0.99)
            ang = rng.uniform(0, 2 * math.pi)
            rx, ry = math.cos(ang) * rng.uniform(1, 1.2), math.sin(ang) * rng.uniform(1, 1.2)
            hit, side, t, fl = orc.cast(g, -1, 1, x, y, rx, ry)
            mh, mt = march(g, x, y, rx, ry, h=1e-4)
            px, py = x + t * rx, y + t * ry
            assert abs(mt - t) <= 2e-4
            if corner_distance(px, py) > 3e-4:
                assert mh == hit
            checked += 1
    assert checked == 180


def test_door_blocks_rays_until_open(orc):
    N = 8
    g = room(N)
    door = 3 * N + 5
    hit, side, t, fl = orc.cast(g, door, 0, 2.5, 3.5, 1.0, 0.0)
    assert hit == door and t == 2.5 and side == 0
    hit, side, t, fl = orc.cast(g, door, 1, 2.5, 3.5, 1.0, 0.0)
    assert hit == 3 * N + 7 and t == 4.5


def test_sprite_straight_ahead_closed_form(orc):
    N, H, Wd = 16, 64, 64
    cfg = cfg_of(orc, side=N, goal_sprite=1)
    g = room(N)
    tanH = math.tan(math.pi / 6)
    for gx, x in ((12, 3.5), (6, 3.5), (4, 3.5), (9, 8.25)):
        gy = 7
        d = gx + 0.5 - x
        obs, cols = orc.render(g, cfg, st(orc, x, gy + 0.5, 0.0, goal=gy * N + gx))
        hw = (Wd / 2) * 0.25 / (tanH * d)
        hs = H * 0.25 / d
        ncol = 2 * min(max(math.ceil(hw - 0.5), 0), Wd // 2)
        nrow = 2 * min(max(math.ceil(hs - 0.5), 0), H // 2)
        mask = (obs == np.array(GOAL, np.uint8)).all(-1)
        assert int(mask.sum()) == ncol * nrow
        colsum = mask.any(0)
        assert int(colsum.sum()) == ncol
        assert colsum[Wd // 2 - 1] and colsum[Wd // 2]      # centred on u = W/2
    # behind a wall: never drawn
    g2 = room(N)
    g2[7, 8] = 1
    obs, _ = orc.render(g2, cfg, st(orc, 3.5, 7.5, 0.0, goal=7 * N + 12))
    assert not (obs == np.array(GOAL, np.uint8)).all(-1).any()


def test_painter_equals_nearest_sprite(orc):
    N, H, Wd = 16, 64, 64
    cfg = cfg_of(orc, side=N, goal_sprite=1, key_door=1, max_decor=2)
    g = room(N)
    tanH = math.tan(math.pi / 6)
    cols_rgb = {0: (255, 40, 40), 1: GOAL, 2: (0, 200, 120), 3: (0, 200, 120)}
    rng = np.random.default_rng(9)
    n_pix = 0
    for _ in range(40):
        tiles = rng.choice(np.arange(N * N).reshape(N, N)[1:N - 1, 1:N - 1].reshape(-1), 5,
                           replace=False)
        a = tiles[0]
        x, y = a % N + rng.uniform(0.1, 0.9), a // N + rng.uniform(0.1, 0.9)
        th = rng.uniform(0, 2 * math.pi)
        s = st(orc, x, y, th, key=int(tiles[1]), goal=int(tiles[2]), n_decor=2,
               decor=[int(tiles[3]), int(tiles[4])], door=0)
        obs, cols = orc.render(g, cfg, s)
        c, sn = math.cos(th), math.sin(th)
        sp = []
        for j, tid in enumerate(tiles[1:]):
            dx, dy = tid % N + 0.5 - x, tid // N + 0.5 - y
            tY, tX = dx * c + dy * sn, -dx * sn + dy * c
            if tY > 0.05:
                sp.append((j, tY, (Wd / 2) * (1 + tX / (tanH * tY)),
                           (Wd / 2) * 0.25 / (tanH * tY), H * 0.25 / tY))
        for col in range(Wd):
            if cols["flags"][col]:
                continue
            for r in range(H):
                best = None
                for j, tY, u, hw, hs in sp:
                    if abs(col + 0.5 - u) < hw and tY < cols["t"][col] and abs(r + 0.5 - H / 2) < hs:
                        if best is None or tY < best[1] or (tY == best[1] and j > best[0]):
                            best = (j, tY)
                px = tuple(obs[r, col])
                if best is not None:
                    assert px == cols_rgb[best[0]]
                    n_pix += 1
                else:
                    assert px not in ((255, 40, 40), GOAL, (0, 200, 120))
    assert n_pix > 1000


def test_wall_colour_and_side_shade(orc):
    # Palette by tile id mod K; a y-face hit halves each channel of the same colour.
    N = 16
    cfg = cfg_of(orc, side=N, n_colors=8)
    g = room(N)
    obs0, c0 = orc.render(g, cfg, st(orc, 8.5, 8.5, 0.0))            # faces east wall
    obs1, c1 = orc.render(g, cfg, st(orc, 8.5, 8.5, math.pi / 2))    # faces south wall
    mid = cfg.obs_w // 2
    assert c0["side"][mid] == 0 and c1["side"][mid] == 1
    # both hit tiles with the same id mod 8 -> same base colour
    a, b = c0["hit"][mid], c1["hit"][mid]
    px0 = obs0[cfg.obs_h // 2, mid].astype(int)
    px1 = obs1[cfg.obs_h // 2, mid].astype(int)
    if a % 8 == b % 8:
        assert (px1 == px0 >> 1).all()
    # tile ids differing by 8 share the colour
    hits = c0["hit"][~c0["flags"].astype(bool)]
    for col in range(cfg.obs_w):
        for col2 in range(cfg.obs_w):
            if c0["flags"][col] or c0["flags"][col2]:
                continue
            if c0["hit"][col] % 8 == c0["hit"][col2] % 8 and c0["side"][col] == c0["side"][col2]:
                assert (obs0[cfg.obs_h // 2, col] == obs0[cfg.obs_h // 2, col2]).all()
    assert len(hits) > 0


def test_agent_against_wall_fills_column(orc):
    N = 8
    cfg = cfg_of(orc, side=N, n_actions=4)
    g = room(N)
    obs, cols = orc.render(g, cfg, st(orc, 6.999, 3.5, 0.0))
    mid = cfg.obs_w // 2
    assert cols["t"][mid] < 0.002
    assert wall_rows(obs[:, mid]) == cfg.obs_h


def test_exact_corner_tie_crosses_y_first(orc):
    # A ray through a tile corner crosses both grid lines at the same parameter;
    # the rule crosses y first, so a blocking diagonal tile is entered through
    # its x-face.  The tie is flagged and the other branch (y-face) reported.
    N = 8
    g = room(N)
    g[3, 3] = 1
    hit, side, t, fl = orc.cast(g, -1, 1, 2.5, 2.5, 1.0, 1.0)
    assert hit == 3 * N + 3 and side == 0 and t == 0.5 and fl & orc.CF_DDA
    cfg = cfg_of(orc, side=N, obs_w=2, obs_h=8, fov_deg=0.0)
    obs, cols = orc.render(g, cfg, st(orc, 2.5, 2.5, math.pi / 4))
    assert cols["flags"][0] & orc.CF_DDA
    assert {cols["side"][0], cols["alt_side"][0]} == {0, 1}


def test_side_shade_same_tile(orc):
    # One pillar tile seen through its x-face and through its y-face: the y-face
    # colour is the x-face colour with every channel halved.
    N = 16
    g = room(N)
    g[8, 8] = 1
    cfg = cfg_of(orc, side=N, n_colors=8)
    mid, hr = cfg.obs_w // 2, cfg.obs_h // 2
    o0, c0 = orc.render(g, cfg, st(orc, 5.5, 8.5, 0.0))
    o1, c1 = orc.render(g, cfg, st(orc, 8.5, 5.5, math.pi / 2))
    assert c0["hit"][mid] == c1["hit"][mid] == 8 * N + 8
    assert c0["side"][mid] == 0 and c1["side"][mid] == 1
    assert (o1[hr, mid].astype(int) == o0[hr, mid].astype(int) >> 1).all()
    assert (o0[hr, mid] != o1[hr, mid]).any()
