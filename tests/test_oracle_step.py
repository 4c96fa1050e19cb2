"""Pins for the oracle's transition: closed forms of movement, collision, turns,
pickups, goal, truncation and invalid actions.  CPU only."""
import math

import numpy as np

import workloads as W

M32 = float(np.float32(0.1))
TURN32 = float(np.float32(math.pi / 16))


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


def test_forward_count_to_wall(orc):
    # Facing +x from x0 in an empty room, accepted forward moves are the j with
    # x0 + j*move < N-1 (the east wall's face), then every move is refused.
    N = 8
    g, cfg = room(N), cfg_of(orc, side=N, n_actions=4)
    for x0 in (1.5, 1.25, 2.93):
        s = st(orc, x0, 3.5, 0.0)
        accepted = 0
        for k in range(80):
            s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)
            assert not d and r == 0.0
            if ev & orc.EV_BLOCKED_X:
                assert s2.x == s.x
            else:
                accepted += 1
            s = s2
        expect = sum(1 for j in range(1, 200) if x0 + j * M32 < N - 1)
        assert accepted == expect
        assert abs(s.x - (x0 + expect * M32)) < 1e-12


def test_backward_and_strafe_axes(orc):
    N = 8
    g = room(N)
    cfg6 = cfg_of(orc, side=N, n_actions=6)
    s = st(orc, 3.5, 3.5, 0.0)
    fwd = orc.step(g, cfg6, 1, s, 0)[0]
    back = orc.step(g, cfg6, 1, s, 1)[0]
    sl = orc.step(g, cfg6, 1, s, 2)[0]
    sr = orc.step(g, cfg6, 1, s, 3)[0]
    assert (fwd.x, fwd.y) == (3.5 + M32, 3.5)
    assert (back.x, back.y) == (3.5 - M32, 3.5)
    # facing +x with +y pointing south, the agent's right is +y
    assert sr.y == 3.5 + M32 and sr.x == 3.5
    assert sl.y == 3.5 - M32 and sl.x == 3.5
    # heading pi/2 (facing +y): right is -x
    s = st(orc, 3.5, 3.5, math.pi / 2)
    sr = orc.step(g, cfg6, 1, s, 3)[0]
    assert abs(sr.x - (3.5 - M32)) < 1e-15 and abs(sr.y - 3.5) < 1e-15


def test_diagonal_into_wall_slides(orc):
    N = 8
    g, cfg = room(N), cfg_of(orc, side=N, n_actions=4)
    s = st(orc, 6.95, 3.5, math.pi / 4)
    s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)
    assert ev & orc.EV_BLOCKED_X and not ev & orc.EV_BLOCKED_Y
    assert s2.x == 6.95
    assert abs(s2.y - (3.5 + M32 * math.sin(math.pi / 4))) < 1e-15
    # corner-cutting through a diagonal wall pair is refused on both axes
    g2 = room(N)
    g2[2, 3] = 1
    g2[3, 2] = 1
    s = st(orc, 3.03, 3.03, math.pi * 5 / 4)   # from tile (3,3) toward the corner of (2,2)
    s2, *_ , ev, sf = orc.step(g2, cfg, 1, s, 0)
    assert ev & orc.EV_BLOCKED_X and ev & orc.EV_BLOCKED_Y
    assert (s2.x, s2.y) == (3.03, 3.03)


def test_turns_wrap_and_cycle(orc):
    N = 8
    g, cfg = room(N), cfg_of(orc, side=N, n_actions=4)
    for th0 in (0.0, 1.0, 6.2):
        s = st(orc, 3.5, 3.5, th0)
        for _ in range(32):
            s = orc.step(g, cfg, 1, s, 3)[0]
            assert 0.0 <= s.theta < 2 * math.pi
        diff = (s.theta - th0 + math.pi) % (2 * math.pi) - math.pi
        assert abs(diff) < 4e-6
        assert (s.x, s.y) == (3.5, 3.5)
    s = orc.step(g, cfg, 1, st(orc, 3.5, 3.5, 0.0), 2)[0]
    assert abs(s.theta - (2 * math.pi - TURN32)) < 1e-15


def test_truncation_exactly_at_cap(orc):
    N, cap = 16, 40
    cfg = cfg_of(orc, side=N, n_actions=4, episode_cap=cap)
    g = room(N)
    s = st(orc, 1.5, 1.5, 0.0, goal=(N - 2) * N + (N - 2))
    rng = np.random.default_rng(0)
    for t in range(cap):
        a = int(rng.integers(0, 2)) + 2   # turns only: never reaches the goal
        s2, r, d, ev, sf = orc.step(g, cfg, 77, s, a)
        if t < cap - 1:
            assert not d and s2.t == t + 1
        else:
            assert d and ev & orc.EV_TRUNC and ev & orc.EV_RESET and r == 0.0
            assert s2.as_dict() == orc.reset(g, cfg, 77, 1).as_dict()
        s = s2


def test_goal_reward_and_reset(orc):
    N = 8
    g = room(N)
    cfg = cfg_of(orc, side=N, n_actions=4, r_goal=1.0)
    goal = 3 * N + 5
    s = st(orc, 4.95, 3.5, 0.0, goal=goal, t=10, episode=4)
    s2, r, d, ev, sf = orc.step(g, cfg, 5, s, 0)
    assert d == 1 and r == 1.0 and ev & orc.EV_GOAL and not ev & orc.EV_TRUNC
    assert s2.as_dict() == orc.reset(g, cfg, 5, 5).as_dict()
    s = st(orc, 4.85, 3.5, 0.0, goal=goal)
    s2, r, d, ev, sf = orc.step(g, cfg, 5, s, 0)       # 4.95: still outside
    assert d == 0 and r == 0.0


def test_key_pickup_radius_and_door(orc):
    N = 8
    g = room(N)
    cfg = cfg_of(orc, side=N, n_actions=4, key_door=1, r_key=0.5)
    key = 3 * N + 3                         # key centre (3.5, 3.5)
    door = 3 * N + 5
    # approach from x = 3.5 - 0.39: one step to 3.5 - 0.29 (inside 0.3)
    s = st(orc, 3.5 - 0.39, 3.5, 0.0, key=key, door=door)
    s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)
    assert ev & orc.EV_KEY and r == 0.5 and s2.key_taken == 1 and s2.door_open == 1
    # from 3.5 - 0.41 the step ends at 3.5 - 0.31: outside
    s = st(orc, 3.5 - 0.41, 3.5, 0.0, key=key, door=door)
    s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)
    assert not ev & orc.EV_KEY and r == 0.0 and s2.key_taken == 0
    # the shut door blocks; once open it does not
    s = st(orc, 4.95, 3.5, 0.0, key=key, door=door)
    s2, *_ , ev, sf = orc.step(g, cfg, 1, s, 0)
    assert ev & orc.EV_BLOCKED_X and s2.x == 4.95
    s = st(orc, 4.95, 3.5, 0.0, key=key, door=door, key_taken=1, door_open=1)
    s2, *_ , ev, sf = orc.step(g, cfg, 1, s, 0)
    assert not ev & orc.EV_BLOCKED_X and s2.x == 4.95 + M32


def test_key_and_goal_same_step_sum(orc):
    N = 8
    g = room(N)
    cfg = cfg_of(orc, side=N, n_actions=4, key_door=1, r_key=0.5, r_goal=1.0)
    t = 3 * N + 4
    s = st(orc, 4.15, 3.5, 0.0, key=t, goal=t, door=5 * N + 5)   # ends at 0.25 from the key
    s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)
    assert r == 1.5 and d and ev & orc.EV_KEY and ev & orc.EV_GOAL


def test_invalid_action_is_noop(orc):
    N = 8
    g, cfg = room(N), cfg_of(orc, side=N, n_actions=4)
    s = st(orc, 3.5, 3.5, 1.0, t=3)
    for a in (4, 5, 200, 255):
        s2, r, d, ev, sf = orc.step(g, cfg, 1, s, a)
        assert ev == orc.EV_INVALID and r == 0.0 and not d
        assert (s2.x, s2.y, s2.theta, s2.t) == (3.5, 3.5, 1.0, 4)


def test_step_flags_near_boundaries(orc):
    N = 8
    g, cfg = room(N), cfg_of(orc, side=N, n_actions=4)
    # a move landing within 1e-5 of the wall face is flagged
    s = st(orc, 7.0 - M32 + 3e-6, 3.5, 0.0)
    *_, sf = orc.step(g, cfg, 1, s, 0)
    assert sf & orc.SF_MOVE
    s = st(orc, 3.5, 3.5, 0.0)
    *_, sf = orc.step(g, cfg, 1, s, 0)
    assert sf == 0


def test_key_pickup_off_diagonal_tile(orc):
    # key tile with different x and y so the two axes of the distance are told apart
    N = 8
    g = room(N)
    cfg = cfg_of(orc, side=N, n_actions=4, key_door=1, r_key=0.5)
    key = 5 * N + 2                          # centre (2.5, 5.5)
    s = st(orc, 2.5, 5.5 - 0.38, math.pi / 2, key=key, door=1 * N + 6)
    s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)     # ends 0.28 above the centre
    assert ev & orc.EV_KEY and r == 0.5
    s = st(orc, 2.5 + 0.2, 5.5 - 0.33, math.pi / 2, key=key, door=1 * N + 6)
    s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)     # ends at (0.2, 0.23): 0.305 away
    assert not ev & orc.EV_KEY and r == 0.0


def test_y_check_uses_updated_x(orc):
    # x moves into column 4 first; the y move is then tested in column 4
    N = 8
    g = room(N)
    g[4, 4] = 1
    cfg = cfg_of(orc, side=N, n_actions=4)
    s = st(orc, 3.95, 3.95, math.pi / 4)
    s2, r, d, ev, sf = orc.step(g, cfg, 1, s, 0)
    assert not ev & orc.EV_BLOCKED_X and ev & orc.EV_BLOCKED_Y
    assert s2.x > 4.0 and s2.y == 3.95


def test_episode_stream_convention(orc):
    # Episode e draws from the stream started at seed XOR mix64(e + 1); its first
    # draw picks the spawn among the free tiles in row-major order.
    N = 16
    cfg = cfg_of(orc, side=N, loop_frac=0.1)
    for seed in (3, 99, 2**40 + 7):
        g = orc.maze(seed, N, 0.1)
        free = np.nonzero(g.reshape(-1) == 0)[0]
        for ep in (0, 1, 5):
            v, _ = orc.rng_range(seed ^ orc.mix64(ep + 1), len(free))
            s = orc.reset(g, cfg, seed, ep)
            assert int(s.y) * N + int(s.x) == free[v]
