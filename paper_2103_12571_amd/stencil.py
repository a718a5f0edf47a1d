"""Stencil taps (dx, dy, coef, dcoef/dnu) of the workloads' operators A.

The taps describe the periodic finite-difference matrices of the synthetic
workloads (grid x_j = j/n, h = 1/n), in the form the C ABI takes them.
"""
import numpy as np


def _pack(taps, dtaps=None):
    keys = sorted(taps)
    dx = np.array([k[0] for k in keys], dtype=np.int32)
    dy = np.array([k[1] for k in keys], dtype=np.int32)
    c = np.array([taps[k] for k in keys], dtype=np.float64)
    d = None if dtaps is None else np.array([dtaps.get(k, 0.0) for k in keys], dtype=np.float64)
    return dx, dy, c, d


def _add(t, k, v):
    t[k] = t.get(k, 0.0) + v


def taps_for(kind, nx, ny=1, nu=0.0, vel=(0.0, 0.0)):
    """(dx, dy, coef, dcoef_dnu) of A for a workload kind.

    heat1d: nu D2 (second-order central); heat2d: nu times the 5-point
    Laplacian; adv1d_c4: -c times the fourth-order central first derivative;
    advdiff2d: nu Lap - v_x Dx - v_y Dy with second-order central Dx, Dy.
    """
    t = {}
    if kind == "heat1d":
        s = nu * nx * nx
        for k, v in (((-1, 0), s), ((0, 0), -2 * s), ((1, 0), s)):
            _add(t, k, v)
        return _pack(t)
    if kind in ("heat2d", "advdiff2d"):
        lap = {}
        sx, sy = nx * nx, ny * ny
        for k, v in (((-1, 0), sx), ((1, 0), sx), ((0, -1), sy), ((0, 1), sy), ((0, 0), -2 * (sx + sy))):
            _add(lap, k, v)
        for k, v in lap.items():
            _add(t, k, nu * v)
        if kind == "heat2d":
            return _pack(t)
        vx, vy = vel
        _add(t, (1, 0), -vx * nx / 2)
        _add(t, (-1, 0), vx * nx / 2)
        _add(t, (0, 1), -vy * ny / 2)
        _add(t, (0, -1), vy * ny / 2)
        return _pack(t, lap)
    if kind == "adv1d_c4":
        c = vel[0]
        s = -c * nx / 12.0
        for k, v in (((-2, 0), s), ((-1, 0), -8 * s), ((1, 0), 8 * s), ((2, 0), -s)):
            _add(t, k, v)
        return _pack(t)
    raise ValueError("unknown operator kind %r" % kind)


def plan_for(workload, **overrides):
    """A binding.Plan for a workload (keyword overrides go to Plan)."""
    from .binding import Plan
    w = workload
    kw = dict(M=w.M, L=w.L, dt=w.dt, batch=w.batch, precision=w.precision, inner=w.inner,
              inner_tol=w.inner_tol)
    kw.update(overrides)
    return Plan(taps_for(w.kind, w.nx, w.ny, nu=w.nu, vel=w.vel), w.nx, w.ny, **kw)
