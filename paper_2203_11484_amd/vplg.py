"""Python binding of libvplg.so (include/vplg.h): argument marshalling only.

Every function here forwards to the C ABI entry point of the same name
(without the ``vplg_`` prefix).  Device memory comes from torch tensors on a
ROCm device (their ``data_ptr()`` is passed in); streams are torch streams
(``torch.cuda.current_stream().cuda_stream`` by default).  All computation
runs in the library's HIP kernels; if the library is not built this module
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvplg.so")
_lib = None

OK, EINVAL, ENOMEM, EBUDGET, ENOTFOUND, EHIP, EBUSY, ECANCELLED, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7, -8

DEBUG_ARRAYS = {"pflags": (0, np.uint8), "sorted": (1, np.int32), "keys": (2, np.uint32), "prefix": (3, np.int64),
                "strata": (4, np.int32), "path": (5, np.int32), "bounce": (6, np.int32),
                "patch_off": (7, np.int64)}


class VplgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vplg error {code}: {msg}")
        self.code = code


class Light(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pos", C.c_float * 3), ("edge_u", C.c_float * 3), ("edge_v", C.c_float * 3),
                ("power", C.c_float * 3)]


class SceneInfo(C.Structure):
    _fields_ = [("n_tris", C.c_int32), ("n_nodes", C.c_int32), ("n_leaves", C.c_int32), ("max_depth", C.c_int32),
                ("device_bytes", C.c_uint64), ("lo", C.c_float * 3), ("hi", C.c_float * 3)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3), ("vfov_deg", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32)]


class GBufferStruct(C.Structure):
    _fields_ = [("pos", C.c_void_p * 3), ("nrm", C.c_void_p * 3), ("alb", C.c_void_p * 3), ("tri", C.c_void_p),
                ("width", C.c_int32), ("height", C.c_int32)]


class GenParams(C.Structure):
    _fields_ = [("k_near", C.c_int32), ("n_far", C.c_int32), ("max_bounces", C.c_int32), ("max_paths", C.c_int32),
                ("d_near", C.c_double), ("patch_h", C.c_double), ("t_eps", C.c_double), ("walk_near", C.c_int32),
                ("jitter", C.c_int32), ("brightness", C.c_int32), ("walk_schedule", C.c_int32)]


class GenStats(C.Structure):
    _fields_ = [("n_patches", C.c_int64), ("n_near", C.c_int64), ("n_eligible", C.c_int64), ("q_total", C.c_int64),
                ("k_eff", C.c_int64), ("n_far_target", C.c_int64), ("n_far", C.c_int64), ("n_paths", C.c_int64),
                ("far_by_bounce", C.c_int64 * 3), ("flags", C.c_int64), ("near_discarded", C.c_int64)]


class GatherParams(C.Structure):
    _fields_ = [("g_clamp", C.c_float), ("t_eps", C.c_float), ("tile_px", C.c_int32), ("tile_vpl", C.c_int32)]


class View(C.Structure):
    _fields_ = [("scene_id", C.c_uint64), ("vplset_id", C.c_uint64), ("gb", GBufferStruct),
                ("radiance", C.c_void_p * 3), ("params", GatherParams)]


class ServerParams(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_inflight", C.c_int32), ("n_streams", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("scene_id", C.c_uint64), ("camera", Camera), ("gen", GenParams), ("gather", GatherParams),
                ("radiance", C.c_void_p * 3)]


class Timing(C.Structure):
    _fields_ = [("state", C.c_int32), ("error", C.c_int32), ("submit_ns", C.c_int64), ("admit_ns", C.c_int64),
                ("done_ns", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("cancelled", C.c_int64), ("queued", C.c_int64), ("running", C.c_int64),
                ("peak_running", C.c_int64), ("pool_bytes", C.c_uint64), ("peak_bytes", C.c_uint64)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED, REQ_CANCELLED = 0, 1, 2, 3, 4

_p = C.c_void_p
_u64 = C.c_uint64
_SIGS = {
    "vplg_last_error": (C.c_char_p, []),
    "vplg_version": (C.c_int, []),
    "vplg_context_create": (C.c_int, [C.c_int, _u64, C.POINTER(_p)]),
    "vplg_context_destroy": (C.c_int, [_p]),
    "vplg_context_usage": (C.c_int, [_p, C.POINTER(_u64), C.POINTER(_u64)]),
    "vplg_scene_upload": (C.c_int, [_p, _p, _p, _p, C.c_int32, C.POINTER(Light), _p, C.POINTER(_u64)]),
    "vplg_scene_release": (C.c_int, [_p, _u64]),
    "vplg_scene_describe": (C.c_int, [_p, _u64, C.POINTER(SceneInfo)]),
    "vplg_gbuffer_render": (C.c_int, [_p, _u64, C.POINTER(Camera), C.POINTER(GBufferStruct), _p]),
    "vplg_vpls_generate": (C.c_int, [_p, _u64, C.POINTER(Camera), C.POINTER(GenParams), _p, C.POINTER(_u64)]),
    "vplg_vpls_regenerate": (C.c_int, [_p, _u64, C.POINTER(Camera), C.POINTER(GenParams), _p]),
    "vplg_vplset_stats": (C.c_int, [_p, _u64, C.POINTER(GenStats)]),
    "vplg_vplset_count": (C.c_int, [_p, _u64, C.POINTER(C.c_int32)]),
    "vplg_vpls_upload": (C.c_int, [_p, _p, _p, _p, _p, C.c_int32, _p, C.POINTER(_u64)]),
    "vplg_vpls_download": (C.c_int, [_p, _u64, _p, _p, _p, _p, C.c_int32, C.POINTER(C.c_int32)]),
    "vplg_vplset_debug": (C.c_int, [_p, _u64, C.c_int32, _p, C.c_int64, C.POINTER(C.c_int64)]),
    "vplg_vplset_release": (C.c_int, [_p, _u64]),
    "vplg_gather": (C.c_int, [_p, _u64, _u64, C.POINTER(GBufferStruct), C.POINTER(_p), C.POINTER(GatherParams), _p]),
    "vplg_gather_noalloc": (C.c_int, [_p, _u64, _u64, C.POINTER(GBufferStruct), C.POINTER(_p),
                                      C.POINTER(GatherParams), _p]),
    "vplg_gather_counted": (C.c_int, [_p, _u64, _u64, C.POINTER(GBufferStruct), C.POINTER(_p),
                                      C.POINTER(GatherParams), _p, _p]),
    "vplg_gather_visibility_dump": (C.c_int, [_p, _u64, _u64, C.POINTER(GBufferStruct), _p, C.c_int32, _p,
                                              C.POINTER(GatherParams), _p]),
    "vplg_direct": (C.c_int, [_p, _u64, C.POINTER(GBufferStruct), C.POINTER(_p), C.c_float, _p]),
    "vplg_gather_batch": (C.c_int, [_p, C.POINTER(View), C.c_int32, _p]),
    "vplg_autotune": (C.c_int, [_p, _u64, _u64, C.POINTER(GBufferStruct), C.POINTER(_p), C.POINTER(GatherParams), _p,
                                C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "vplg_autotune_batch": (C.c_int, [_p, C.POINTER(View), C.c_int32, _p, C.POINTER(C.c_int32)]),
    "vplg_autotune_lookup": (C.c_int, [_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]),
    "vplg_autotune_save": (C.c_int, [_p, C.c_char_p]),
    "vplg_autotune_load": (C.c_int, [_p, C.c_char_p]),
    "vplg_server_start": (C.c_int, [_p, C.POINTER(ServerParams), C.POINTER(_p)]),
    "vplg_server_submit": (C.c_int, [_p, C.POINTER(Request), C.POINTER(_u64)]),
    "vplg_server_poll": (C.c_int, [_p, _u64, C.POINTER(Timing)]),
    "vplg_server_wait": (C.c_int, [_p, _u64, C.c_int64, C.POINTER(Timing)]),
    "vplg_server_cancel": (C.c_int, [_p, _u64]),
    "vplg_server_query": (C.c_int, [_p, C.POINTER(ServerStats)]),
    "vplg_server_stop": (C.c_int, [_p]),
}


def lib():
    """Load libvplg.so (raises if it was not built; there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python paper_2203_11484_amd/build.py")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _check(rc):
    if rc != 0:
        msg = lib().vplg_last_error()
        raise VplgError(rc, msg.decode() if msg else "")


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(stream)


def _f32c(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# ---------------------------------------------------------------------------
# struct builders
# ---------------------------------------------------------------------------

def make_light(d):
    L = Light()
    L.kind = int(d["kind"])
    for k in ("pos", "edge_u", "edge_v", "power"):
        getattr(L, k)[:] = [float(x) for x in np.asarray(d[k], np.float32)]
    return L


def make_camera(d):
    c = Camera()
    c.eye[:] = [float(x) for x in np.asarray(d["eye"], np.float32)]
    c.target[:] = [float(x) for x in np.asarray(d["target"], np.float32)]
    c.up[:] = [float(x) for x in np.asarray(d["up"], np.float32)]
    c.vfov_deg = float(d["vfov_deg"])
    c.width = int(d["width"])
    c.height = int(d["height"])
    return c


def make_gen_params(p):
    g = GenParams()
    g.k_near, g.n_far, g.max_bounces = int(p["k_near"]), int(p["n_far"]), int(p["max_bounces"])
    g.max_paths = int(p["max_paths"])
    g.d_near, g.patch_h, g.t_eps = float(p["d_near"]), float(p["patch_h"]), float(p["t_eps"])
    g.walk_near = int(p.get("walk_near", 0))
    g.jitter = int(p.get("jitter", 0))
    g.brightness = int(p.get("brightness", 0))
    g.walk_schedule = int(p.get("walk_schedule", 0))
    return g


def make_gather_params(p=None, g_clamp=10.0, t_eps=1e-4):
    if p is not None:
        g_clamp, t_eps = p.get("g_clamp", g_clamp), p.get("t_eps", t_eps)
    g = GatherParams()
    g.g_clamp, g.t_eps, g.tile_px, g.tile_vpl = float(g_clamp), float(t_eps), 0, 0
    if p is not None:
        g.tile_px, g.tile_vpl = int(p.get("tile_px", 0)), int(p.get("tile_vpl", 0))
    return g


class GBuffer:
    """Device G-buffer planes held by torch tensors: ``planes`` (9, H, W) float32
    = position xyz, normal xyz, albedo rgb; ``tri`` (H, W) int32."""

    def __init__(self, width, height, device="cuda", planes=None, tri=None):
        import torch
        self.width, self.height = int(width), int(height)
        self.planes = planes if planes is not None else torch.empty((9, height, width), dtype=torch.float32,
                                                                    device=device)
        self.tri = tri if tri is not None else torch.empty((height, width), dtype=torch.int32, device=device)
        assert self.planes.is_contiguous() and self.tri.is_contiguous()
        s = GBufferStruct()
        base = self.planes.data_ptr()
        plane = self.width * self.height * 4
        for c in range(3):
            s.pos[c] = base + c * plane
            s.nrm[c] = base + (3 + c) * plane
            s.alb[c] = base + (6 + c) * plane
        s.tri = self.tri.data_ptr()
        s.width, s.height = self.width, self.height
        self.struct = s

    @classmethod
    def from_arrays(cls, pos, nrm, alb, tri, width, height, device="cuda"):
        """Upload AoS float arrays [P, 3] and tri [P] into device planes."""
        import torch
        P = width * height
        planes = np.empty((9, P), np.float32)
        planes[0:3] = _f32c(pos).reshape(P, 3).T
        planes[3:6] = _f32c(nrm).reshape(P, 3).T
        planes[6:9] = _f32c(alb).reshape(P, 3).T
        pt = torch.from_numpy(planes.reshape(9, height, width)).to(device)
        tt = torch.from_numpy(np.ascontiguousarray(tri, np.int32).reshape(height, width)).to(device)
        return cls(width, height, device, pt, tt)

    def to_numpy(self):
        pl = self.planes.cpu().numpy().reshape(9, -1)
        return dict(pos=pl[0:3].T.copy(), nrm=pl[3:6].T.copy(), alb=pl[6:9].T.copy(),
                    tri=self.tri.cpu().numpy().reshape(-1))


def radiance_planes(rad):
    """(3, H, W) float32 torch tensor -> array of 3 device pointers."""
    assert rad.is_contiguous() and rad.dtype.itemsize == 4
    plane = rad[0].numel() * 4
    arr = (C.c_void_p * 3)()
    for c in range(3):
        arr[c] = rad.data_ptr() + c * plane
    return arr


# ---------------------------------------------------------------------------
# ABI calls
# ---------------------------------------------------------------------------

def version():
    return lib().vplg_version()


def context_create(device=0, hbm_budget_bytes=0):
    h = C.c_void_p()
    _check(lib().vplg_context_create(int(device), int(hbm_budget_bytes), C.byref(h)))
    return h


def context_destroy(ctx):
    _check(lib().vplg_context_destroy(ctx))


def context_usage(ctx):
    used, budget = _u64(), _u64()
    _check(lib().vplg_context_usage(ctx, C.byref(used), C.byref(budget)))
    return used.value, budget.value


def scene_upload(ctx, tri, albedo, flags, light, stream=None):
    tri = _f32c(tri).reshape(-1, 9)
    alb = _f32c(albedo).reshape(-1, 3)
    fl = np.ascontiguousarray(flags, np.uint8)
    L = make_light(light)
    sid = _u64()
    _check(lib().vplg_scene_upload(ctx, tri.ctypes.data, alb.ctypes.data, fl.ctypes.data, len(tri), C.byref(L),
                                   _stream(stream), C.byref(sid)))
    return sid.value


def scene_release(ctx, scene_id):
    _check(lib().vplg_scene_release(ctx, scene_id))


def scene_describe(ctx, scene_id):
    info = SceneInfo()
    _check(lib().vplg_scene_describe(ctx, scene_id, C.byref(info)))
    return dict(n_tris=info.n_tris, n_nodes=info.n_nodes, n_leaves=info.n_leaves, max_depth=info.max_depth,
                device_bytes=info.device_bytes, lo=list(info.lo), hi=list(info.hi))


def gbuffer_render(ctx, scene_id, camera, gb, stream=None):
    cam = make_camera(camera)
    _check(lib().vplg_gbuffer_render(ctx, scene_id, C.byref(cam), C.byref(gb.struct), _stream(stream)))


def vpls_generate(ctx, scene_id, camera, params, stream=None):
    cam = make_camera(camera)
    gp = make_gen_params(params)
    vid = _u64()
    _check(lib().vplg_vpls_generate(ctx, scene_id, C.byref(cam), C.byref(gp), _stream(stream), C.byref(vid)))
    return vid.value


def vpls_regenerate(ctx, vplset_id, camera, params, stream=None):
    cam = make_camera(camera)
    gp = make_gen_params(params)
    _check(lib().vplg_vpls_regenerate(ctx, vplset_id, C.byref(cam), C.byref(gp), _stream(stream)))


def vplset_stats(ctx, vplset_id):
    st = GenStats()
    _check(lib().vplg_vplset_stats(ctx, vplset_id, C.byref(st)))
    d = {k: getattr(st, k) for k, _ in GenStats._fields_ if k != "far_by_bounce"}
    d["far_b1"], d["far_b2"], d["far_b3"] = list(st.far_by_bounce)
    return d


def vplset_count(ctx, vplset_id):
    n = C.c_int32()
    _check(lib().vplg_vplset_count(ctx, vplset_id, C.byref(n)))
    return n.value


def vpls_upload(ctx, pos, nrm, intensity, host_tri, stream=None):
    pos, nrm, I = _f32c(pos).reshape(-1, 3), _f32c(nrm).reshape(-1, 3), _f32c(intensity).reshape(-1, 3)
    tri = np.ascontiguousarray(host_tri, np.int32)
    n = len(pos)
    vid = _u64()
    _check(lib().vplg_vpls_upload(ctx, pos.ctypes.data, nrm.ctypes.data, I.ctypes.data, tri.ctypes.data, n,
                                  _stream(stream), C.byref(vid)))
    return vid.value


def vpls_download(ctx, vplset_id):
    n = vplset_count(ctx, vplset_id)
    pos = np.zeros((n, 3), np.float32)
    nrm = np.zeros((n, 3), np.float32)
    I = np.zeros((n, 3), np.float32)
    tri = np.zeros(n, np.int32)
    got = C.c_int32()
    _check(lib().vplg_vpls_download(ctx, vplset_id, pos.ctypes.data, nrm.ctypes.data, I.ctypes.data, tri.ctypes.data,
                                    n, C.byref(got)))
    return dict(pos=pos, nrm=nrm, I=I, tri=tri, n=got.value)


def vplset_debug(ctx, vplset_id, name):
    what, dt = DEBUG_ARRAYS[name]
    n = C.c_int64()
    rc = lib().vplg_vplset_debug(ctx, vplset_id, what, None, 0, C.byref(n))
    if rc not in (0, EINVAL):
        _check(rc)
    out = np.zeros(max(n.value, 1), dt)
    _check(lib().vplg_vplset_debug(ctx, vplset_id, what, out.ctypes.data, out.nbytes, C.byref(n)))
    return out[:n.value]


def vplset_release(ctx, vplset_id):
    _check(lib().vplg_vplset_release(ctx, vplset_id))


def gather(ctx, scene_id, vplset_id, gb, radiance, params=None, stream=None):
    gp = params if isinstance(params, GatherParams) else make_gather_params(params)
    _check(lib().vplg_gather(ctx, scene_id, vplset_id, C.byref(gb.struct), radiance_planes(radiance), C.byref(gp),
                             _stream(stream)))


def gather_noalloc(ctx, scene_id, vplset_id, gb, radiance, params=None, stream=None):
    """vplg_gather without device allocation: its work memory is the library's fixed per-device array."""
    gp = params if isinstance(params, GatherParams) else make_gather_params(params)
    _check(lib().vplg_gather_noalloc(ctx, scene_id, vplset_id, C.byref(gb.struct), radiance_planes(radiance),
                                     C.byref(gp), _stream(stream)))


def direct(ctx, scene_id, gb, radiance, t_eps=1e-4, stream=None):
    """Direct term L_e of eq. (1) into radiance (torch [3, H, W] float32 on the device)."""
    _check(lib().vplg_direct(ctx, scene_id, C.byref(gb.struct), radiance_planes(radiance), float(t_eps),
                             _stream(stream)))


N_COUNTERS = 14  # counters[0..13] of vplg_gather_counted


def gather_counted(ctx, scene_id, vplset_id, gb, radiance, counters, params=None, stream=None):
    """counters: torch int64 tensor of N_COUNTERS on the device (see vplg_gather_counted in include/vplg.h)."""
    if counters.numel() < N_COUNTERS:
        raise ValueError(f"gather_counted needs {N_COUNTERS} counters")
    gp = params if isinstance(params, GatherParams) else make_gather_params(params)
    _check(lib().vplg_gather_counted(ctx, scene_id, vplset_id, C.byref(gb.struct), radiance_planes(radiance),
                                     C.byref(gp), C.c_void_p(counters.data_ptr()), _stream(stream)))


def gather_visibility_dump(ctx, scene_id, vplset_id, gb, pixels, vis_bits, params=None, stream=None):
    """pixels: device int32 tensor [n]; vis_bits: device int32 tensor [n, ceil(M/32)]."""
    gp = params if isinstance(params, GatherParams) else make_gather_params(params)
    _check(lib().vplg_gather_visibility_dump(ctx, scene_id, vplset_id, C.byref(gb.struct),
                                             C.c_void_p(pixels.data_ptr()), int(pixels.numel()),
                                             C.c_void_p(vis_bits.data_ptr()), C.byref(gp), _stream(stream)))


def make_views(views):
    """views: list of dicts with scene, vplset, gb (GBuffer), radiance ((3, H, W) tensor), params (dict or
    GatherParams).  Returns the ctypes array (keep it alive while the call runs)."""
    arr = (View * len(views))()
    for i, v in enumerate(views):
        arr[i].scene_id = v["scene"]
        arr[i].vplset_id = v["vplset"]
        arr[i].gb = v["gb"].struct
        rp = radiance_planes(v["radiance"])
        for c in range(3):
            arr[i].radiance[c] = rp[c]
        p = v.get("params")
        arr[i].params = p if isinstance(p, GatherParams) else make_gather_params(p)
    return arr


def gather_batch(ctx, views, stream=None):
    arr = make_views(views)
    _check(lib().vplg_gather_batch(ctx, arr, len(views), _stream(stream)))
    return arr


def autotune(ctx, scene_id, vplset_id, gb, radiance, params=None, stream=None):
    """Returns the fastest (tile_vpl, tile_px) of a lone gather of this view, now the tuned shape of its bucket."""
    gp = params if isinstance(params, GatherParams) else make_gather_params(params)
    best, px = C.c_int32(), C.c_int32()
    _check(lib().vplg_autotune(ctx, scene_id, vplset_id, C.byref(gb.struct), radiance_planes(radiance), C.byref(gp),
                               _stream(stream), C.byref(best), C.byref(px)))
    return best.value, px.value


def autotune_batch(ctx, views, stream=None):
    """Tune the open views' shape buckets with the batched launch as the objective; returns the buckets kept."""
    arr = make_views(views)
    n = C.c_int32()
    _check(lib().vplg_autotune_batch(ctx, arr, len(views), _stream(stream), C.byref(n)))
    return n.value


def autotune_lookup(ctx, width, height, n_vpls, batched=False):
    """(tile_vpl, tile_px) a gather of this shape takes with tile_vpl 0."""
    w, px = C.c_int32(), C.c_int32()
    _check(lib().vplg_autotune_lookup(ctx, int(width), int(height), int(n_vpls), int(bool(batched)), C.byref(w),
                                      C.byref(px)))
    return w.value, px.value


def autotune_save(ctx, path):
    _check(lib().vplg_autotune_save(ctx, os.fsencode(path)))


def autotune_load(ctx, path):
    _check(lib().vplg_autotune_load(ctx, os.fsencode(path)))


def _timing(t):
    return dict(state=t.state, error=t.error, submit_ns=t.submit_ns, admit_ns=t.admit_ns, done_ns=t.done_ns)


def server_start(ctx, hbm_budget_bytes, max_inflight=8, n_streams=4):
    prm = ServerParams(int(hbm_budget_bytes), int(max_inflight), int(n_streams))
    h = C.c_void_p()
    _check(lib().vplg_server_start(ctx, C.byref(prm), C.byref(h)))
    return h


def make_request(scene_id, camera, gen_params, radiance, gather_params=None):
    r = Request()
    r.scene_id = scene_id
    r.camera = make_camera(camera)
    r.gen = make_gen_params(gen_params)
    gp = gather_params if isinstance(gather_params, GatherParams) else make_gather_params(gather_params or gen_params)
    r.gather = gp
    rp = radiance_planes(radiance)
    for c in range(3):
        r.radiance[c] = rp[c]
    return r


def server_submit(srv, request):
    t = C.c_uint64()
    _check(lib().vplg_server_submit(srv, C.byref(request), C.byref(t)))
    return t.value


def server_poll(srv, ticket):
    t = Timing()
    _check(lib().vplg_server_poll(srv, ticket, C.byref(t)))
    return _timing(t)


def server_wait(srv, ticket, timeout_ms=-1):
    t = Timing()
    _check(lib().vplg_server_wait(srv, ticket, int(timeout_ms), C.byref(t)))
    return _timing(t)


def server_cancel(srv, ticket):
    _check(lib().vplg_server_cancel(srv, ticket))


def server_query(srv):
    st = ServerStats()
    _check(lib().vplg_server_query(srv, C.byref(st)))
    return {k: getattr(st, k) for k, _ in ServerStats._fields_}


def server_stop(srv):
    _check(lib().vplg_server_stop(srv))
