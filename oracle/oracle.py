"""ctypes front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It takes the same
float32 arrays that the GPU library takes and returns float64 results.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

ST_NAMES = ("n_patches", "n_near", "n_eligible", "Q", "k_eff", "n_far_target", "n_far", "n_paths",
            "far_b1", "far_b2", "far_b3", "flags", "near_discarded")

_p = C.c_void_p


def _ptr(a):
    return a.ctypes.data_as(_p) if a is not None else None


def lib():
    global _LIB
    if _LIB is None:
        # ORACLE_LIB: another build of oracle.c (the sanitizer test loads an ASan/UBSan one)
        path = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            import importlib.util
            spec = importlib.util.spec_from_file_location("_oracle_build", os.path.join(_HERE, "build.py"))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            mod.build()
        _LIB = C.CDLL(path)
        L = _LIB
        L.oracle_scene_create.restype = _p
        L.oracle_scene_create.argtypes = [_p, _p, _p, C.c_int, C.c_int]
        L.oracle_scene_destroy.argtypes = [_p]
        L.oracle_scene_bvh_nodes.argtypes = [_p]
        L.oracle_face_normals.argtypes = [_p, _p]
        L.oracle_visibility.argtypes = [_p, _p, _p, _p, _p, C.c_int64, C.c_double, _p]
        L.oracle_grazing.argtypes = [_p, _p, _p, _p, _p, C.c_int64, C.c_double, C.c_double, _p]
        L.oracle_gbuffer.argtypes = [_p, _p, _p, _p, _p, _p]
        L.oracle_gbuffer_edges.argtypes = [_p, _p, C.c_double, _p]
        L.oracle_gather.argtypes = [_p, _p, _p, _p, _p, C.c_int64, _p, _p, _p, _p, C.c_int, C.c_double,
                                    C.c_double, _p, _p, _p, C.c_int64, C.c_int, _p]
        L.oracle_vis_matrix.argtypes = [_p, _p, _p, C.c_int64, _p, _p, C.c_int, C.c_double, _p]
        L.oracle_light_samples.argtypes = [_p, _p]
        L.oracle_light_samples.restype = C.c_int
        L.oracle_direct.argtypes = [_p, _p, _p, _p, _p, C.c_int64, _p, C.c_double, _p, _p, _p, C.c_int64, _p]
        L.oracle_halton.restype = C.c_double
        L.oracle_halton.argtypes = [C.c_int, C.c_int64]
        L.oracle_rho_bar.restype = C.c_double
        L.oracle_rho_bar.argtypes = [_p]
        L.oracle_patch_count.restype = C.c_int64
        L.oracle_patch_count.argtypes = [_p, C.c_double]
        L.oracle_generate.restype = C.c_int
        L.oracle_generate.argtypes = [_p, _p, _p, _p, _p, C.c_double] + [_p] * 12 + [C.c_int64, _p]
        L.oracle_morton30.restype = C.c_uint32
        L.oracle_morton30.argtypes = [C.c_int, C.c_int, C.c_int]
        L.oracle_num_threads.restype = C.c_int
    return _LIB


def _f32(a, shape_last=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def cam_array(cam):
    return np.array([*cam["eye"], *cam["target"], *cam["up"], cam["vfov_deg"], cam["width"], cam["height"]],
                    dtype=np.float64)


def light_array(light):
    return np.array([light["kind"], *light["pos"], *light["edge_u"], *light["edge_v"], *light["power"]],
                    dtype=np.float64)


def halton(b, i):
    return lib().oracle_halton(int(b), int(i))


def morton30(cx, cy, cz):
    return lib().oracle_morton30(int(cx), int(cy), int(cz))


def num_threads():
    return lib().oracle_num_threads()


def light_samples(light):
    """The light's sample points as eq. (2) uses them: [1, 3] or [16, 3] FP64."""
    la = light_array(light)
    out = np.zeros((16, 3), np.float64)
    n = lib().oracle_light_samples(_ptr(la), _ptr(out))
    return out[:n].copy()


class Scene:
    """FP64 copy of a float32 triangle scene (optionally with the oracle's own BVH)."""

    def __init__(self, tri, albedo, flags, use_bvh=None):
        self.tri = _f32(np.asarray(tri).reshape(-1, 9))
        self.albedo = _f32(np.asarray(albedo).reshape(-1, 3))
        self.flags = np.ascontiguousarray(flags, dtype=np.uint8)
        self.T = len(self.tri)
        if use_bvh is None:
            use_bvh = self.T > 1000
        self.use_bvh = bool(use_bvh)
        self.h = lib().oracle_scene_create(_ptr(self.tri), _ptr(self.albedo), _ptr(self.flags), self.T,
                                           int(self.use_bvh))
        lo = self.tri.reshape(-1, 3).astype(np.float64).min(0) if self.T else np.zeros(3)
        hi = self.tri.reshape(-1, 3).astype(np.float64).max(0) if self.T else np.zeros(3)
        self.diag = float(np.linalg.norm(hi - lo))

    @classmethod
    def from_dict(cls, sc, use_bvh=None):
        return cls(sc["tri"], sc["albedo"], sc["flags"], use_bvh)

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.oracle_scene_destroy(self.h)
            self.h = None

    def normals(self):
        out = np.zeros((self.T, 3), np.float64)
        lib().oracle_face_normals(self.h, _ptr(out))
        return out

    # -- visibility --------------------------------------------------------
    def visibility(self, x, tx, y, ty, eps=1e-4):
        x, y = _f32(x).reshape(-1, 3), _f32(y).reshape(-1, 3)
        tx, ty = _i32(tx), _i32(ty)
        n = len(x)
        out = np.zeros(n, np.uint8)
        lib().oracle_visibility(self.h, _ptr(x), _ptr(tx), _ptr(y), _ptr(ty), n, eps, _ptr(out))
        return out

    def grazing(self, x, tx, y, ty, eps=1e-4, delta_rel=1e-5):
        x, y = _f32(x).reshape(-1, 3), _f32(y).reshape(-1, 3)
        tx, ty = _i32(tx), _i32(ty)
        n = len(x)
        out = np.zeros(n, np.uint8)
        lib().oracle_grazing(self.h, _ptr(x), _ptr(tx), _ptr(y), _ptr(ty), n, eps, delta_rel * self.diag,
                             _ptr(out))
        return out

    # -- G-buffer ----------------------------------------------------------
    def gbuffer(self, cam):
        ca = cam_array(cam)
        P = cam["width"] * cam["height"]
        pos = np.zeros((P, 3)); nrm = np.zeros((P, 3)); alb = np.zeros((P, 3))
        tri = np.zeros(P, np.int32)
        lib().oracle_gbuffer(self.h, _ptr(ca), _ptr(pos), _ptr(nrm), _ptr(alb), _ptr(tri))
        return dict(pos=pos, nrm=nrm, alb=alb, tri=tri)

    def gbuffer_edges(self, cam, delta=1e-5):
        ca = cam_array(cam)
        out = np.zeros(cam["width"] * cam["height"], np.uint8)
        lib().oracle_gbuffer_edges(self.h, _ptr(ca), delta, _ptr(out))
        return out

    # -- gather ------------------------------------------------------------
    def gather(self, gpos, gnrm, galb, gtri, vpos, vnrm, vI, vtri, C=10.0, eps=1e-4, overrides=None,
               nthreads=0):
        gpos, gnrm, galb = (_f32(a).reshape(-1, 3) for a in (gpos, gnrm, galb))
        gtri = _i32(gtri)
        vpos, vnrm, vI = (_f32(a).reshape(-1, 3) for a in (vpos, vnrm, vI))
        vtri = _i32(vtri)
        n = len(gpos)
        M = len(vpos)
        if overrides is not None:
            op, ov, ob = overrides
            order = np.lexsort((ov, op))
            op, ov, ob = _i32(np.asarray(op)[order]), _i32(np.asarray(ov)[order]), \
                np.ascontiguousarray(np.asarray(ob)[order], np.uint8)
            nov = len(op)
        else:
            op = ov = ob = None
            nov = 0
        L = np.zeros((n, 3), np.float64)
        lib().oracle_gather(self.h, _ptr(gpos), _ptr(gnrm), _ptr(galb), _ptr(gtri), n, _ptr(vpos), _ptr(vnrm),
                            _ptr(vI), _ptr(vtri), M, float(C), float(eps), _ptr(op), _ptr(ov), _ptr(ob), nov,
                            int(nthreads), _ptr(L))
        return L

    def direct(self, gpos, gnrm, galb, gtri, light, eps=1e-4, overrides=None):
        """Direct term L_e of eq. (1) (light model of eq. (2)) per G-buffer entry, [n, 3] FP64;
        overrides = (pixel, sample, visibility) replace V for listed pairs."""
        gpos, gnrm, galb = (_f32(a).reshape(-1, 3) for a in (gpos, gnrm, galb))
        gtri = _i32(gtri)
        n = len(gpos)
        if overrides is not None:
            op, os_, ob = overrides
            order = np.lexsort((os_, op))
            op, os_, ob = _i32(np.asarray(op)[order]), _i32(np.asarray(os_)[order]), \
                np.ascontiguousarray(np.asarray(ob)[order], np.uint8)
            nov = len(op)
        else:
            op = os_ = ob = None
            nov = 0
        la = light_array(light)
        L = np.zeros((n, 3), np.float64)
        lib().oracle_direct(self.h, _ptr(gpos), _ptr(gnrm), _ptr(galb), _ptr(gtri), n, _ptr(la), float(eps),
                            _ptr(op), _ptr(os_), _ptr(ob), nov, _ptr(L))
        return L

    def vis_matrix(self, gpos, gtri, vpos, vtri, eps=1e-4):
        gpos, vpos = _f32(gpos).reshape(-1, 3), _f32(vpos).reshape(-1, 3)
        gtri, vtri = _i32(gtri), _i32(vtri)
        out = np.zeros((len(gpos), len(vpos)), np.uint8)
        lib().oracle_vis_matrix(self.h, _ptr(gpos), _ptr(gtri), len(gpos), _ptr(vpos), _ptr(vtri), len(vpos),
                                float(eps), _ptr(out))
        return out

    def rho_bar(self):
        """The scene's mean albedo of Keller's path schedule (area-weighted over non-emitting faces)."""
        return float(lib().oracle_rho_bar(self.h))

    # -- generation --------------------------------------------------------
    def generate(self, cam, light, params):
        p = params
        ca, la = cam_array(cam), light_array(light)
        ip = np.array([p["k_near"], p["n_far"], p["max_bounces"], p["max_paths"], p.get("walk_near", 0),
                       p.get("jitter", 0), p.get("brightness", 0), p.get("walk_schedule", 0)], np.int64)
        dp = np.array([p["d_near"], p["patch_h"]], np.float64)
        NP = int(lib().oracle_patch_count(self.h, float(p["patch_h"])))
        cap = int(p["k_near"] + p["n_far"])
        patch_off = np.zeros(self.T + 1, np.int64)
        pflags = np.zeros(max(NP, 1), np.uint8)
        sorted_ = np.zeros(max(NP, 1), np.int32)
        keys = np.zeros(max(NP, 1), np.uint32)
        F = np.zeros(max(NP, 1), np.int64)
        m = np.zeros(max(int(p["k_near"]), 1), np.int32)
        vpos = np.zeros((cap, 3)); vnrm = np.zeros((cap, 3)); vI = np.zeros((cap, 3))
        vtri = np.zeros(cap, np.int32); vpath = np.zeros(cap, np.int32); vb = np.zeros(cap, np.int32)
        stats = np.zeros(len(ST_NAMES), np.int64)
        nv = lib().oracle_generate(self.h, _ptr(ca), _ptr(la), _ptr(ip), _ptr(dp), float(p["t_eps"]),
                                   _ptr(patch_off), _ptr(pflags), _ptr(sorted_), _ptr(keys), _ptr(F), _ptr(m),
                                   _ptr(vpos), _ptr(vnrm), _ptr(vI), _ptr(vtri), _ptr(vpath), _ptr(vb), cap,
                                   _ptr(stats))
        if nv < 0:
            raise RuntimeError(f"oracle_generate failed ({nv})")
        st = dict(zip(ST_NAMES, (int(v) for v in stats)))
        ne = st["n_eligible"]
        return dict(stats=st, patch_off=patch_off, pflags=pflags[:NP], sorted=sorted_[:ne], keys=keys[:ne],
                    F=F[:ne], m=m[:st["k_eff"]], pos=vpos[:nv], nrm=vnrm[:nv], I=vI[:nv], tri=vtri[:nv],
                    path=vpath[:nv], bounce=vb[:nv], n=nv)
