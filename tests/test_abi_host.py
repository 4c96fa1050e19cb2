"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/jx.h, and its host-only entry points behave (layout
generator equal to the oracle's maze byte for byte; argument validation)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "jx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(jx_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def jx():
    from paper_2605_19926_amd import jx as m
    m.lib()
    return m


def test_every_declared_symbol_is_exported(jx):
    names = declared_functions()
    assert len(names) >= 25
    L = jx.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) <= set(jx._SIGS), set(names) - set(jx._SIGS)


def test_abi_version(jx):
    assert jx.lib().jx_abi_version() == jx.ABI_VERSION == 5


@pytest.mark.parametrize("side", [5, 8, 9, 16, 31, 32, 64])
def test_host_layout_equals_oracle_maze(jx, orc, side):
    for lf in (0.0, 0.1, 0.5):
        cfg = W.env_cfg(side=side, loop_frac=lf)
        for seed in range(60):
            s = seed * 7 + side * 1000 + 2**40
            assert (jx.make_layout(s, cfg) == orc.maze(s, side, lf)).all(), (side, lf, seed)


def test_workload_seeds_layouts_match(jx, orc):
    for wl in (W.TINY, W.SCALE, W.KEYDOOR):
        cfg = wl["cfg"]
        for s in W.seeds(wl["number"], 64):
            assert (jx.make_layout(int(s), cfg) == orc.maze(int(s), cfg["side"],
                                                            cfg["loop_frac"])).all()


@pytest.mark.parametrize("bad", [dict(side=4), dict(side=65), dict(n_colors=0), dict(n_colors=9),
                                 dict(loop_frac=1.5), dict(max_decor=3), dict(obs_h=3),
                                 dict(obs_w=6), dict(obs_w=132), dict(n_actions=5),
                                 dict(episode_cap=0), dict(fov_deg=180.0), dict(move=1.0),
                                 dict(obs_layout=2), dict(obs_layout=-1), dict(obs_dtype=3)])
def test_layout_rejects_bad_cfg(jx, bad):
    cfg = W.env_cfg(**bad)
    with pytest.raises(jx.JxError) as e:
        jx.make_layout(1, cfg)
    assert e.value.code == jx.JX_EINVAL
    assert jx.lib().jx_last_error()


def test_workspace_bytes(jx):
    cfg = W.SCALE["cfg"]
    one = jx.workspace_bytes(1, [cfg])
    many = jx.workspace_bytes(4096, [cfg])
    assert one > 0 and many > one
    assert many % 256 == 0
    # per-env maps grow with the side
    big = jx.workspace_bytes(4096, [W.env_cfg(side=64)])
    assert big - many >= 4096 * (64 * 64 - 256)
    # several configurations need an index
    arr = (jx.jx_env_cfg * 2)(jx.make_cfg(cfg), jx.make_cfg(W.KEYDOOR["cfg"]))
    assert jx.lib().jx_workspace_bytes(4, arr, 2, None) == 0
    idx = np.array([0, 1, 1, 0], np.int32)
    assert jx.lib().jx_workspace_bytes(4, arr, 2, idx.ctypes.data) > 0
    idx[2] = 5
    assert jx.lib().jx_workspace_bytes(4, arr, 2, idx.ctypes.data) == 0
    assert jx.lib().jx_workspace_bytes(0, arr, 1, None) > 0


def test_null_arguments_are_errors(jx):
    L = jx.lib()
    assert L.jx_step(None, None, None, None, None, None) == jx.JX_EINVAL
    assert L.jx_reset(None, 1, None, None, 1, None, None) == jx.JX_EINVAL
    assert L.jx_make_layout(1, None, None) == jx.JX_EINVAL
    assert L.jx_server_submit(None, 0, None, None) == jx.JX_EINVAL
    assert L.jx_server_replay(None, 1, None, None, None, None, 1, 0.0, None, None, None) == jx.JX_EINVAL
    assert L.jx_num_envs(None) == -1
    assert L.jx_obs_bytes(None) == -1


def test_binding_checks_buffer_extents():
    """The binding refuses buffers smaller than a launch touches (the C-ABI
    sees raw pointers only)."""
    import torch
    from paper_2605_19926_amd import jx
    t = torch.zeros(100, dtype=torch.float32)
    jx._need("reward", t, 400)
    with pytest.raises(jx.JxError):
        jx._need("reward", t, 401)
    with pytest.raises(jx.JxError):
        jx._need("reward", t[::2], 10)
    with pytest.raises(jx.JxError):
        jx._need("reward", None, 1)


@pytest.mark.parametrize("text,side", [(W.MAP16, 16), (W.MAP10, 10), (W.MAP10, 13)])
def test_host_ascii_layout_equals_oracle(jx, orc, text, side):
    """The library's ASCII front-end and the oracle's (independent parsers of
    the Table 2 format) produce the same tile grid."""
    cfg = W.env_cfg(side=side, ascii_map=text)
    g_host = jx.make_layout(0, cfg)
    g_orc, _, _ = orc.ascii_layout(text, side)
    assert np.array_equal(g_host, g_orc)


@pytest.mark.parametrize("text,kw", [
    ("#####\n#.x.#\n#####", {}),                       # unknown symbol
    ("#####\n#....\n#####", {"side": 5}),              # border tile (x = 4 of 5) not a wall
    ("#####\n#.R.#\n#####", {"key_door": 1}),          # generated key-door with a map
    ("##\"##\n#.R.#\n#####", {"side": 5}),             # a door on the border (row 0)
    ("#" * 17, {}),                                    # wider than the side
])
def test_host_ascii_rejects(jx, text, kw):
    kw = dict({"side": 16}, **kw)
    cfg = W.env_cfg(ascii_map=text, **kw)
    with pytest.raises(jx.JxError):
        jx.make_layout(0, cfg)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: asking for more exits with a message, before
    touching any device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU only" in r.stderr


def test_one_hip_runtime_whatever_the_import_order():
    """Loading the library before torch must not leave two HIP runtimes in the
    process (torch's own and the system's, under one soname): the binding loads
    torch first, so libjx.so binds to torch's runtime.  Checked in a fresh
    interpreter from the memory map; no device is touched."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_2605_19926_amd import jx\n"
            "jx.lib()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(sorted({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=root)
    assert r.returncode == 0, r.stderr[-2000:]
    import ast
    libs = ast.literal_eval(r.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs
