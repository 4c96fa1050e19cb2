"""Python binding of libjx (include/jx.h): argument marshalling only.

Every step of the path runs in the HIP kernels of libjx.so.  PyTorch provides
device memory (tensors whose ``data_ptr()`` is passed through) and the stream
(``torch.cuda.current_stream().cuda_stream``).  The library must have been built
in-tree (``python -m paper_2605_19926_amd.build``); importing this module without
it raises immediately.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjx.so")

JX_OK, JX_EINVAL, JX_ENOMEM, JX_EDEVICE, JX_ESTATE, JX_EBUSY = 0, -1, -2, -3, -4, -5
ABI_VERSION = 5  # the jx_env_cfg layout and signatures this binding marshals
JX_FORM_PLAIN, JX_FORM_PERSISTENT, JX_FORM_PIPELINE = 0, 1, 2
JX_ROLLOUT_GRAPH, JX_ROLLOUT_FUSED = 1, 2
JX_SERVE_COALESCE, JX_SERVE_PLAIN = 0, 1
JX_OBS_NHWC, JX_OBS_NCHW = 0, 1
JX_OBS_U8, JX_OBS_BF16, JX_OBS_F32 = 0, 1, 2
OBS_ELEM_BYTES = {JX_OBS_U8: 1, JX_OBS_BF16: 2, JX_OBS_F32: 4}

EV_BLOCKED_X, EV_BLOCKED_Y, EV_KEY, EV_GOAL = 0x01, 0x02, 0x04, 0x08
EV_TRUNC, EV_INVALID, EV_RESET = 0x10, 0x20, 0x40
FL_KEY, FL_DOOR_OPEN = 0x01, 0x02


class JxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"jx error {code}: {msg}")
        self.code = code


class jx_env_cfg(ctypes.Structure):
    _fields_ = [("side", ctypes.c_int32), ("n_colors", ctypes.c_int32),
                ("loop_frac", ctypes.c_float), ("key_door", ctypes.c_int32),
                ("goal_sprite", ctypes.c_int32), ("max_decor", ctypes.c_int32),
                ("obs_h", ctypes.c_int32), ("obs_w", ctypes.c_int32),
                ("fov_deg", ctypes.c_float), ("n_actions", ctypes.c_int32),
                ("episode_cap", ctypes.c_int32), ("move", ctypes.c_float),
                ("turn", ctypes.c_float), ("pickup_radius", ctypes.c_float),
                ("r_goal", ctypes.c_float), ("r_key", ctypes.c_float),
                ("shade_levels", ctypes.c_int32), ("shade_dist", ctypes.c_float),
                ("ascii_map", ctypes.c_char_p),
                ("obs_layout", ctypes.c_int32), ("obs_dtype", ctypes.c_int32)]


class jx_launch(ctypes.Structure):
    _fields_ = [("form", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("groups_per_cu", ctypes.c_int32), ("store_mode", ctypes.c_int32),
                ("waves_per_env", ctypes.c_int32)]


class jx_col_debug(ctypes.Structure):
    _fields_ = [("hit", ctypes.c_int32), ("side", ctypes.c_int32), ("t", ctypes.c_float),
                ("cell", ctypes.c_int32)]


class jx_field(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("offset", ctypes.c_int64),
                ("bytes", ctypes.c_int64), ("elem", ctypes.c_int32), ("count", ctypes.c_int32)]


class jx_server_stats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("requests", ctypes.c_int64),
                ("env_steps", ctypes.c_int64), ("admission_waits", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_int64), ("clients_active", ctypes.c_int64),
                ("clients_pending", ctypes.c_int64), ("failed_launches", ctypes.c_int64)]


COL_DEBUG_DTYPE = np.dtype([("hit", "<i4"), ("side", "<i4"), ("t", "<f4"), ("cell", "<i4")])

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_sz = ctypes.c_size_t

# name -> (restype, argtypes); names and order follow include/jx.h
_SIGS = {
    "jx_abi_version": (_i32, []),
    "jx_last_error": (ctypes.c_char_p, []),
    "jx_workspace_bytes": (_sz, [_i32, ctypes.POINTER(jx_env_cfg), _i32, _vp]),
    "jx_create": (_i32, [ctypes.POINTER(_vp), _i32, _vp, _vp, _sz]),
    "jx_destroy": (None, [_vp]),
    "jx_reset": (_i32, [_vp, _i32, _vp, ctypes.POINTER(jx_env_cfg), _i32, _vp, _vp]),
    "jx_num_envs": (_i32, [_vp]),
    "jx_obs_bytes": (_i64, [_vp]),
    "jx_obs_offsets": (_i32, [_vp, _vp]),
    "jx_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "jx_rollout": (_i32, [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _i32]),
    "jx_rollout_noalloc": (_i32, [_vp, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _i32]),
    "jx_render": (_i32, [_vp, _vp, _vp]),
    "jx_state_bytes": (_sz, [_vp]),
    "jx_state_layout": (_i32, [_vp, ctypes.POINTER(jx_field), _i32, ctypes.POINTER(_i32)]),
    "jx_get_state": (_i32, [_vp, _vp, _sz]),
    "jx_set_state": (_i32, [_vp, _vp, _sz]),
    "jx_set_launch": (_i32, [_vp, ctypes.POINTER(jx_launch)]),
    "jx_get_launch": (_i32, [_vp, ctypes.POINTER(jx_launch)]),
    "jx_autotune": (_i32, [_vp, _vp, _i32, _vp, ctypes.c_char_p, ctypes.POINTER(jx_launch)]),
    "jx_sync": (_i32, [_vp]),
    "jx_make_layout": (_i32, [_u64, ctypes.POINTER(jx_env_cfg), _vp]),
    "jx_server_create": (_i32, [ctypes.POINTER(_vp), _i32, _sz, _i32, _i32, _i32]),
    "jx_server_destroy": (None, [_vp]),
    "jx_server_open": (_i32, [_vp, _i32, _vp, ctypes.POINTER(jx_env_cfg), ctypes.POINTER(_i32)]),
    "jx_server_open_dev": (_i32, [_vp, _i32, _vp, ctypes.POINTER(jx_env_cfg), _vp, _vp, _vp, _i32,
                                  ctypes.POINTER(_i32)]),
    "jx_server_submit": (_i32, [_vp, _i32, _vp, ctypes.POINTER(_u64)]),
    "jx_server_wait": (_i32, [_vp, _u64, ctypes.c_double, _vp, _vp, _vp,
                              ctypes.POINTER(ctypes.c_double)]),
    "jx_server_close": (_i32, [_vp, _i32]),
    "jx_server_wait_any": (_i32, [_vp, ctypes.c_double, ctypes.POINTER(_u64), ctypes.POINTER(_i32)]),
    "jx_server_get_stats": (_i32, [_vp, ctypes.POINTER(jx_server_stats)]),
    "jx_server_replay": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _i32, ctypes.c_double, _vp,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libjx.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2605_19926_amd.build`")
        # torch bundles its own HIP runtime under the same soname as the
        # system's.  Loaded first, it satisfies libjx.so's dependency, so the
        # process holds one HIP runtime and torch's device memory and streams
        # are valid in the library's calls.  Loaded after libjx.so, torch would
        # bring a second runtime that cannot open the GPU.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            if not hasattr(L, name):
                raise ImportError(f"{LIB_PATH} lacks {name}: rebuild it")
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        if L.jx_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI version {L.jx_abi_version()}, this binding "
                              f"expects {ABI_VERSION}: rebuild it")
        _lib = L
    return _lib


def check(code: int) -> int:
    if code != JX_OK:
        raise JxError(code, lib().jx_last_error().decode(errors="replace"))
    return code


def make_cfg(d: dict) -> jx_env_cfg:
    """The configuration struct of a dict; "ascii_map" (optional) is a str or
    None (the struct keeps a reference to the encoded text)."""
    c = jx_env_cfg()
    for name, _ in jx_env_cfg._fields_:
        if name == "ascii_map":
            m = d.get("ascii_map")
            c.ascii_map = None if m is None else m.encode("ascii")
            continue
        if name in ("obs_layout", "obs_dtype"):
            setattr(c, name, d.get(name, 0))
            continue
        setattr(c, name, d[name])
    return c


def frame_bytes(d: dict) -> int:
    """Bytes of one frame of configuration d in its format."""
    return d["obs_h"] * d["obs_w"] * 3 * OBS_ELEM_BYTES[d.get("obs_dtype", JX_OBS_U8)]


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _nbytes(t) -> int:
    if isinstance(t, np.ndarray):
        return int(t.nbytes)
    return int(t.numel()) * int(t.element_size())


def _need(name: str, t, nbytes: int, device=None) -> None:
    """Host-side size (and device) check of a buffer the kernels will touch:
    the C-ABI takes raw pointers and cannot see extents."""
    if t is None:
        raise JxError(JX_EINVAL, f"{name} is required")
    if not t.is_contiguous():
        raise JxError(JX_EINVAL, f"{name} must be contiguous")
    if device is not None and t.device != device:
        raise JxError(JX_EINVAL, f"{name} is on {t.device}, expected {device}")
    have = _nbytes(t)
    if have < nbytes:
        raise JxError(JX_EINVAL, f"{name} holds {have} bytes, {nbytes} needed")


def make_layout(seed: int, cfg: dict) -> np.ndarray:
    """Host-only maze generator of the library (no device needed)."""
    c = make_cfg(cfg)
    g = np.zeros((cfg["side"], cfg["side"]), np.uint8)
    check(lib().jx_make_layout(seed & (2**64 - 1), ctypes.byref(c), g.ctypes.data))
    return g


def workspace_bytes(n: int, cfgs: list[dict], cfg_index=None) -> int:
    arr = (jx_env_cfg * len(cfgs))(*[make_cfg(c) for c in cfgs])
    idx = None if cfg_index is None else np.ascontiguousarray(cfg_index, np.int32)
    return int(lib().jx_workspace_bytes(n, arr, len(cfgs), _ptr(idx)))


class Env:
    """A batch of environments on one device, driven through the C-ABI.

    Holds the torch tensors that back the workspace, observations, rewards and
    dones.  ``step(actions)`` takes a uint8 device tensor [n]."""

    def __init__(self, seeds, cfgs, cfg_index=None, device: int = 0, stream=None,
                 obs_slots: int = 1):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", device)
        if isinstance(cfgs, dict):
            cfgs = [cfgs]
        self.cfgs = list(cfgs)
        self.seeds = np.ascontiguousarray(seeds, np.uint64)
        self.n = int(self.seeds.shape[0])
        self.cfg_index = None if cfg_index is None else np.ascontiguousarray(cfg_index, np.int32)
        self._carr = (jx_env_cfg * len(self.cfgs))(*[make_cfg(c) for c in self.cfgs])
        ws = lib().jx_workspace_bytes(self.n, self._carr, len(self.cfgs), _ptr(self.cfg_index))
        if ws == 0:
            raise JxError(JX_EINVAL, "invalid configuration for jx_workspace_bytes")
        self.workspace = torch.empty(int(ws) + 256, dtype=torch.uint8, device=self.dev)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._ws_ptr = aligned
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.dev)
        ctx = _vp()
        check(lib().jx_create(ctypes.byref(ctx), device, _vp(self.stream.cuda_stream),
                              _vp(aligned), ctypes.c_size_t(int(ws))))
        self.ctx = ctx
        self.obs_slots = obs_slots
        self._reset_done = False

    # -- lifecycle ---------------------------------------------------------------
    def reset(self, obs=None):
        torch = self.torch
        if obs is not None:
            per_cfg = [frame_bytes(c) for c in self.cfgs]
            need = (per_cfg[0] * self.n if self.cfg_index is None
                    else int(sum(per_cfg[i] for i in self.cfg_index)))
            _need("obs", obs, need, self.dev)
        check(lib().jx_reset(self.ctx, self.n, _ptr(self.seeds), self._carr, len(self.cfgs),
                             _ptr(self.cfg_index), _ptr(obs)))
        self.obs_bytes = int(lib().jx_obs_bytes(self.ctx))
        off = np.zeros(self.n + 1, np.int64)
        check(lib().jx_obs_offsets(self.ctx, off.ctypes.data))
        self.obs_offsets = off
        self.reward = torch.zeros(self.n, dtype=torch.float32, device=self.dev)
        self.done = torch.zeros(self.n, dtype=torch.uint8, device=self.dev)
        self._reset_done = True

    def close(self):
        if getattr(self, "ctx", None):
            lib().jx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping ----------------------------------------------------------------
    def new_obs(self, slots: int = 1):
        return self.torch.empty(slots * self.obs_bytes, dtype=torch_uint8(self.torch),
                                device=self.dev)

    def _check_frame(self, obs, name="obs"):
        if obs is not None and self._reset_done:
            _need(name, obs, self.obs_bytes, self.dev)

    def step(self, actions, obs, reward=None, done=None, prev=None):
        """One step; prev (optional uint8 [n]) receives the previous action to
        feed the policy beside each returned frame (n_actions at an episode start)."""
        reward = self.reward if reward is None else reward
        done = self.done if done is None else done
        _need("actions", actions, self.n, self.dev)
        _need("reward", reward, 4 * self.n, self.dev)
        _need("done", done, self.n, self.dev)
        if prev is not None:
            _need("prev", prev, self.n, self.dev)
        self._check_frame(obs)
        check(lib().jx_step(self.ctx, _ptr(actions), _ptr(obs), _ptr(reward), _ptr(done), _ptr(prev)))
        return reward, done

    def rollout(self, actions, obs, reward, done, T: int, obs_stride: int = 0, graph: bool = True,
                fused: bool = False, prev=None):
        flags = (JX_ROLLOUT_GRAPH if graph else 0) | (JX_ROLLOUT_FUSED if fused else 0)
        if T > 0:
            _need("actions", actions, T * self.n, self.dev)
            _need("reward", reward, 4 * T * self.n, self.dev)
            _need("done", done, T * self.n, self.dev)
            if prev is not None:
                _need("prev", prev, T * self.n, self.dev)
            if obs_stride and obs_stride < self.obs_bytes:
                raise JxError(JX_EINVAL, f"obs_stride {obs_stride} < frame bytes {self.obs_bytes}")
            if obs is not None:
                _need("obs", obs, (T - 1) * obs_stride + self.obs_bytes, self.dev)
        check(lib().jx_rollout(self.ctx, T, _ptr(actions), _ptr(obs), obs_stride, _ptr(reward),
                               _ptr(done), _ptr(prev), flags))

    def rollout_noalloc(self, actions, obs, reward, done, T: int, obs_stride: int = 0,
                        fused: bool = False, prev=None, flags: int | None = None):
        """jx_rollout_noalloc: the rollout of ``rollout(..., graph=False)`` with
        its work-queue counters in the library's static device array (no
        allocation); ``flags`` overrides the flags passed (for error tests)."""
        if flags is None:
            flags = JX_ROLLOUT_FUSED if fused else 0
        if T > 0:
            _need("actions", actions, T * self.n, self.dev)
            _need("reward", reward, 4 * T * self.n, self.dev)
            _need("done", done, T * self.n, self.dev)
            if prev is not None:
                _need("prev", prev, T * self.n, self.dev)
            if obs_stride and obs_stride < self.obs_bytes:
                raise JxError(JX_EINVAL, f"obs_stride {obs_stride} < frame bytes {self.obs_bytes}")
            if obs is not None:
                _need("obs", obs, (T - 1) * obs_stride + self.obs_bytes, self.dev)
        check(lib().jx_rollout_noalloc(self.ctx, T, _ptr(actions), _ptr(obs), obs_stride, _ptr(reward),
                                       _ptr(done), _ptr(prev), flags))

    def render(self, obs=None, debug=None):
        self._check_frame(obs)
        check(lib().jx_render(self.ctx, _ptr(obs), _ptr(debug)))

    def sync(self):
        check(lib().jx_sync(self.ctx))

    # -- launch mapping ----------------------------------------------------------
    def set_launch(self, form=JX_FORM_PLAIN, waves_per_group=1, groups_per_cu=4, store_mode=0, waves_per_env=1):
        l = jx_launch(form, waves_per_group, groups_per_cu, store_mode, waves_per_env)
        check(lib().jx_set_launch(self.ctx, ctypes.byref(l)))

    def get_launch(self) -> dict:
        l = jx_launch()
        check(lib().jx_get_launch(self.ctx, ctypes.byref(l)))
        return {k: getattr(l, k) for k, _ in jx_launch._fields_}

    def autotune(self, actions, iters: int, obs_scratch, cache_path: str | None = None) -> dict:
        l = jx_launch()
        check(lib().jx_autotune(self.ctx, _ptr(actions), iters, _ptr(obs_scratch),
                                None if cache_path is None else cache_path.encode(),
                                ctypes.byref(l)))
        return {k: getattr(l, k) for k, _ in jx_launch._fields_}

    # -- state -------------------------------------------------------------------
    def state_layout(self) -> dict:
        n = _i32()
        check(lib().jx_state_layout(self.ctx, None, 0, ctypes.byref(n)))
        arr = (jx_field * n.value)()
        check(lib().jx_state_layout(self.ctx, arr, n.value, ctypes.byref(n)))
        return {f.name.decode(): (f.offset, f.bytes, f.elem, f.count) for f in arr}

    def get_state_bytes(self) -> np.ndarray:
        nb = int(lib().jx_state_bytes(self.ctx))
        buf = np.zeros(nb, np.uint8)
        check(lib().jx_get_state(self.ctx, buf.ctypes.data, nb))
        return buf

    def set_state_bytes(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, np.uint8)
        check(lib().jx_set_state(self.ctx, buf.ctypes.data, buf.nbytes))

    def get_state(self) -> dict:
        """Per-env state arrays (numpy views into one host image)."""
        buf = self.get_state_bytes()
        return unpack_state(buf, self.state_layout())

    def set_state(self, fields: dict, image: np.ndarray | None = None):
        """Writes the given arrays (same names as get_state) into an image of the
        current state and uploads it."""
        buf = self.get_state_bytes() if image is None else image.copy()
        lay = self.state_layout()
        for name, arr in fields.items():
            off, nbytes, elem, count = lay[name]
            raw = np.ascontiguousarray(arr).view(np.uint8).reshape(-1)
            if raw.nbytes > nbytes:
                raise ValueError(f"{name}: {raw.nbytes} bytes > {nbytes}")
            buf[off:off + raw.nbytes] = raw
        self.set_state_bytes(buf)


_FIELD_DTYPES = {"x": np.float32, "y": np.float32, "theta": np.float32, "t": np.uint32,
                 "episode": np.uint32, "goal": np.int32, "door": np.int32, "key": np.int32,
                 "decor": np.int32, "flags": np.uint8, "events": np.uint8, "n_decor": np.uint8,
                 "invalid": np.uint32, "seed": np.uint64, "cfg_index": np.int32,
                 "map_offset": np.uint32, "obs_offset": np.int64, "order": np.int32,
                 "akey": np.int32, "doors": np.uint32}


def unpack_state(buf: np.ndarray, layout: dict) -> dict:
    out = {}
    for name, (off, nbytes, elem, count) in layout.items():
        raw = buf[off:off + nbytes]
        if name in _FIELD_DTYPES:
            out[name] = raw.view(_FIELD_DTYPES[name]).copy()
        else:
            out[name] = raw.copy()
    return out


def torch_uint8(torch):
    return torch.uint8


class Server:
    """Serving loop of libjx (jx_server_*): clients' env batches stay resident
    on the device; ready step requests are coalesced into shared launches."""

    def __init__(self, device: int = 0, hbm_budget: int = 8 << 30, n_streams: int = 4,
                 mode: int = JX_SERVE_COALESCE, max_batch_envs: int = 0):
        h = _vp()
        check(lib().jx_server_create(ctypes.byref(h), device, hbm_budget, n_streams, mode,
                                     max_batch_envs))
        self.h = h
        self.sizes = {}

    def open(self, seeds, cfg: dict) -> tuple[int, bool]:
        """Returns (client id, admitted now)."""
        seeds = np.ascontiguousarray(seeds, np.uint64)
        c = make_cfg(cfg)
        cid = _i32()
        rc = lib().jx_server_open(self.h, int(seeds.shape[0]), seeds.ctypes.data, ctypes.byref(c),
                                  ctypes.byref(cid))
        if rc not in (JX_OK, JX_EBUSY):
            check(rc)
        self.sizes[cid.value] = (int(seeds.shape[0]), cfg["obs_h"] * cfg["obs_w"] * 3)
        return cid.value, rc == JX_OK

    def open_dev(self, seeds, cfg: dict, obs, reward, done, slots: int) -> tuple[int, bool]:
        """A client whose results stay in device rings (torch tensors on the
        server's device): obs [slots * n * H * W * 3] uint8, reward [slots * n]
        float32, done [slots * n] uint8; request k writes slot k mod slots.
        Returns (client id, admitted now)."""
        seeds = np.ascontiguousarray(seeds, np.uint64)
        n = int(seeds.shape[0])
        fb = cfg["obs_h"] * cfg["obs_w"] * 3
        _need("obs", obs, slots * n * fb)
        _need("reward", reward, 4 * slots * n)
        _need("done", done, slots * n)
        c = make_cfg(cfg)
        cid = _i32()
        rc = lib().jx_server_open_dev(self.h, n, seeds.ctypes.data, ctypes.byref(c), _ptr(obs), _ptr(reward),
                                      _ptr(done), slots, ctypes.byref(cid))
        if rc not in (JX_OK, JX_EBUSY):
            check(rc)
        self.sizes[cid.value] = (n, fb)
        self.dev_clients = getattr(self, "dev_clients", set()) | {cid.value}
        return cid.value, rc == JX_OK

    def submit(self, client: int, actions: np.ndarray) -> int:
        a = np.ascontiguousarray(actions, np.uint8)
        t = _u64()
        check(lib().jx_server_submit(self.h, client, a.ctypes.data, ctypes.byref(t)))
        return t.value

    def wait(self, client: int, ticket: int, timeout: float = -1.0, want_obs: bool = True,
             out=None):
        """Returns (obs [n, H*W*3] or None, reward, done, latency_s), or None on
        timeout.  `out` = (obs, reward, done) arrays to fill instead of new ones."""
        n, fb = self.sizes[client]
        if client in getattr(self, "dev_clients", ()):
            # results are in the client's device rings: wait only
            lat = ctypes.c_double()
            rc = lib().jx_server_wait(self.h, ticket, timeout, None, None, None, ctypes.byref(lat))
            if rc == JX_EBUSY:
                return None
            check(rc)
            return None, None, None, lat.value
        if out is not None:
            obs, rew, done = out
            if (obs is not None and (obs.dtype != np.uint8 or obs.size != n * fb or
                                     not obs.flags.c_contiguous)) or \
                    rew.dtype != np.float32 or rew.size != n or not rew.flags.c_contiguous or \
                    done.dtype != np.uint8 or done.size != n or not done.flags.c_contiguous:
                raise JxError(JX_EINVAL, "out buffers do not match the client's sizes")
        else:
            obs = np.empty((n, fb), np.uint8) if want_obs else None
            rew = np.empty(n, np.float32)
            done = np.empty(n, np.uint8)
        lat = ctypes.c_double()
        rc = lib().jx_server_wait(self.h, ticket, timeout, _ptr(obs), rew.ctypes.data,
                                  done.ctypes.data, ctypes.byref(lat))
        if rc == JX_EBUSY:
            return None
        check(rc)
        return obs, rew, done, lat.value

    def wait_any(self, timeout: float = -1.0):
        """Next completed, not yet collected request as (client, ticket), in
        completion order, or None on timeout.  Collect it with wait()."""
        tk = _u64()
        cid = _i32()
        rc = lib().jx_server_wait_any(self.h, timeout, ctypes.byref(tk), ctypes.byref(cid))
        if rc == JX_EBUSY:
            return None
        check(rc)
        return cid.value, tk.value

    def replay(self, t_arrival, clients, actions, close_after=None, n_collectors: int = 4,
               timeout: float = 600.0):
        """Native load generator (jx_server_replay): submits request k at
        t_arrival[k] s for clients[k] with actions[k] (uint8 array of that
        client's size), closing the client after it when close_after[k].
        Returns (latency_s per request, submit seconds, wall seconds)."""
        n = len(t_arrival)
        t = np.ascontiguousarray(t_arrival, np.float64)
        c = np.ascontiguousarray(clients, np.int32)
        acts = [np.ascontiguousarray(a, np.uint8) for a in actions]
        for k, a in enumerate(acts):
            if a.size != self.sizes[int(c[k])][0]:
                raise JxError(JX_EINVAL, f"request {k}: {a.size} actions for a client of "
                                         f"{self.sizes[int(c[k])][0]} envs")
        ptrs = np.array([a.ctypes.data for a in acts], np.uint64)
        ca = None if close_after is None else np.ascontiguousarray(close_after, np.uint8)
        lat = np.zeros(n, np.float64)
        sub, wall = ctypes.c_double(), ctypes.c_double()
        check(lib().jx_server_replay(self.h, n, t.ctypes.data, c.ctypes.data, ptrs.ctypes.data,
                                     None if ca is None else ca.ctypes.data, n_collectors, timeout,
                                     lat.ctypes.data, ctypes.byref(sub), ctypes.byref(wall)))
        return lat, sub.value, wall.value

    def close_client(self, client: int):
        check(lib().jx_server_close(self.h, client))

    def stats(self) -> dict:
        s = jx_server_stats()
        check(lib().jx_server_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in jx_server_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            lib().jx_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
