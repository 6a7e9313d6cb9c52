"""Small scene builders and tolerance checks shared by the tests (no method arithmetic)."""
import numpy as np

from paper_2203_11484_amd import scenes


def floor_quad(x0, x1, z0, z1, y=0.0, nu=1, nv=1):
    """Rectangle at height y, front facing +y, split into nu x nv cells (2 triangles each)."""
    return scenes._quad_grid((x0, y, z0), (x1 - x0, 0, 0), (0, 0, z1 - z0), (0, 1, 0), nu, nv)


def closed_box(lo, hi, cells=1):
    """Six inward-facing walls of an axis-aligned box."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    ex = hi - lo
    walls = [
        (lo, (ex[0], 0, 0), (0, 0, ex[2]), (0, 1, 0)),
        ((lo[0], hi[1], lo[2]), (ex[0], 0, 0), (0, 0, ex[2]), (0, -1, 0)),
        (lo, (ex[0], 0, 0), (0, ex[1], 0), (0, 0, 1)),
        ((lo[0], lo[1], hi[2]), (ex[0], 0, 0), (0, ex[1], 0), (0, 0, -1)),
        (lo, (0, ex[1], 0), (0, 0, ex[2]), (1, 0, 0)),
        ((hi[0], lo[1], lo[2]), (0, ex[1], 0), (0, 0, ex[2]), (-1, 0, 0)),
    ]
    return np.concatenate([scenes._quad_grid(p, u, v, n, cells, cells) for p, u, v, n in walls])


def scene_dict(tri, albedo, flags=None, light=None, camera=None, params=None):
    tri = np.ascontiguousarray(np.asarray(tri, np.float32).reshape(-1, 3, 3))
    T = len(tri)
    alb = np.ascontiguousarray(np.broadcast_to(np.asarray(albedo, np.float32), (T, 3)))
    fl = np.zeros(T, np.uint8) if flags is None else np.asarray(flags, np.uint8)
    return dict(name="test", tri=tri, albedo=alb, flags=fl, light=light, camera=camera,
                params=params or scenes.default_params())


def radiance_close(L_gpu, L_ref, rel=1e-4, floor_frac=1e-3):
    """Per channel |dL| <= rel * max(L_ref, floor_frac * mean(L_ref)); exact zeros stay zero.

    Returns a boolean mask of pixels that pass."""
    L_gpu = np.asarray(L_gpu, np.float64)
    L_ref = np.asarray(L_ref, np.float64)
    mean = np.maximum(L_ref.mean(axis=0, keepdims=True), 1e-300)
    tol = rel * np.maximum(np.abs(L_ref), floor_frac * mean)
    ok = np.abs(L_gpu - L_ref) <= tol
    ok &= ~((L_ref == 0) & (L_gpu != 0))
    return ok.all(axis=-1)
