"""Pins for the oracle's training-buffer formats (frames as a recurrent-PPO
learner stores them: NHWC or NCHW, bytes or the byte / 255 as bfloat16 or
float32) and for the previous-action rule.  The conversions are checked
against exact rational arithmetic for every byte; the layouts against numpy
transposes.  CPU only."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W


def f32_neighbours(v):
    v = np.float32(v)
    return np.nextafter(v, np.float32(-1)), np.nextafter(v, np.float32(2))


def bf16_value(bits):
    return float(np.array([bits << 16], np.uint32).view(np.float32)[0])


def test_f32_is_the_nearest_float_to_b_over_255(orc):
    for b in range(256):
        q = Fraction(b, 255)
        v = orc.norm_f32(b)
        err = abs(Fraction(v) - q)
        for nb in f32_neighbours(v):
            assert err < abs(Fraction(float(nb)) - q) or b in (0, 255), b
        assert 0.0 <= v <= 1.0


def test_bf16_is_the_nearest_bfloat16_to_b_over_255(orc):
    for b in range(256):
        q = Fraction(b, 255)
        bits = orc.norm_bf16(b)
        v = Fraction(bf16_value(bits))
        err = abs(v - q)
        # the neighbouring bfloat16 values one unit in the last place away
        for nbits in (bits - 1, bits + 1):
            if 0 <= nbits < 0x7F80:
                assert err < abs(Fraction(bf16_value(nbits)) - q) or b in (0, 255), b
        if b:
            # 8 significant bits: unit roundoff 2^-8
            assert err <= q / 256, b


def test_known_values(orc):
    assert orc.norm_f32(0) == 0.0 and orc.norm_f32(255) == 1.0
    assert orc.norm_f32(51) == float(np.float32(0.2))          # 51 / 255 = 1 / 5
    assert orc.norm_f32(85) == float(np.float32(1.0 / 3.0))    # 85 / 255 = 1 / 3
    assert orc.norm_bf16(0) == 0 and orc.norm_bf16(255) == 0x3F80
    # 128 / 255 = 0.50196...: 0.50390625 (0x3F01) is nearer than 0.5 (0x3F00)
    assert orc.norm_bf16(128) == 0x3F01
    assert orc.norm_bf16(51) == 0x3E4D                          # 0.2 -> 0.200195...


def test_layouts_are_transposes(orc):
    rng = np.random.default_rng(11)
    f = rng.integers(0, 256, (7, 12, 3), dtype=np.uint8)
    tab32 = np.array([orc.norm_f32(b) for b in range(256)], np.float32)
    tab16 = np.array([orc.norm_bf16(b) for b in range(256)], np.uint16)
    assert np.array_equal(orc.format_frame(f, orc.OBS_NHWC, orc.OBS_U8), f)
    assert np.array_equal(orc.format_frame(f, orc.OBS_NCHW, orc.OBS_U8), f.transpose(2, 0, 1))
    assert np.array_equal(orc.format_frame(f, orc.OBS_NHWC, orc.OBS_F32), tab32[f])
    assert np.array_equal(orc.format_frame(f, orc.OBS_NCHW, orc.OBS_F32), tab32[f].transpose(2, 0, 1))
    assert np.array_equal(orc.format_frame(f, orc.OBS_NHWC, orc.OBS_BF16), tab16[f])
    assert np.array_equal(orc.format_frame(f, orc.OBS_NCHW, orc.OBS_BF16), tab16[f].transpose(2, 0, 1))


def test_bad_format_rejected(orc):
    f = np.zeros((2, 2, 3), np.uint8)
    with pytest.raises(KeyError):
        orc.format_frame(f, orc.OBS_NHWC, 3)
    with pytest.raises(ValueError):
        orc.format_frame(f, 2, orc.OBS_U8)


def test_prev_action_rule_on_a_trajectory(orc):
    cfg_d = W.env_cfg(side=8, n_colors=4, loop_frac=0.0, n_actions=4, episode_cap=16,
                      obs_h=32, obs_w=32)
    cfg = orc.make_cfg(cfg_d)
    seed = 1234
    g = orc.maze(seed, 8, 0.0)
    s = orc.reset(g, cfg, seed, 0)
    rng = np.random.default_rng(5)
    saw_done = saw_invalid = 0
    for t in range(60):
        a = int(rng.integers(0, 5))                   # 4 is out of range for 4 actions
        s, r, d, ev, sf = orc.step(g, cfg, seed, s, a)
        p = orc.prev_action(cfg, a, d)
        if d:
            assert p == 4 and (ev & orc.EV_RESET)
            saw_done += 1
        elif a >= 4:
            assert p == 4 and (ev & orc.EV_INVALID)
            saw_invalid += 1
        else:
            assert p == a
        assert 0 <= p <= cfg.n_actions                 # a one-hot of width n_actions + 1
    assert saw_done >= 3 and saw_invalid >= 3
