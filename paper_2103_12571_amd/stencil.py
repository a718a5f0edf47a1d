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


# Central second differences of order 2, 4, 6 (h^2 f'' ~ sum w_j f_{x+j}) and
# upwind first differences of order 1..5 for a positive velocity
# (h f' ~ sum w_j f_{x+j}), the classical rational weights.
CENTRAL_D2 = {
    2: {-1: 1.0, 0: -2.0, 1: 1.0},
    4: {-2: -1 / 12, -1: 4 / 3, 0: -5 / 2, 1: 4 / 3, 2: -1 / 12},
    6: {-3: 1 / 90, -2: -3 / 20, -1: 3 / 2, 0: -49 / 18, 1: 3 / 2, 2: -3 / 20, 3: 1 / 90},
}
UPWIND_D1 = {
    1: {-1: -1.0, 0: 1.0},
    2: {-2: 1 / 2, -1: -2.0, 0: 3 / 2},
    3: {-2: 1 / 6, -1: -1.0, 0: 1 / 2, 1: 1 / 3},
    4: {-3: -1 / 12, -2: 1 / 2, -1: -3 / 2, 0: 5 / 6, 1: 1 / 4},
    5: {-3: -1 / 30, -2: 1 / 4, -1: -1.0, 0: 1 / 3, 1: 1 / 2, 2: -1 / 20},
}


def taps_for(kind, nx, ny=1, nu=0.0, vel=(0.0, 0.0), order=2):
    """(dx, dy, coef, dcoef_dnu) of A for a workload kind.

    heat1d: nu D2 (second-order central); heat2d: nu times the 5-point
    Laplacian; adv1d_c4: -c times the fourth-order central first derivative;
    advdiff2d: nu Lap - v_x Dx - v_y Dy with second-order central Dx, Dy;
    heat2d_central: nu Lap with central differences of order `order` (the heat
    problem of Sec. 5); adv2d_upwind: -(v_x Dx + v_y Dy) with upwind
    differences of order `order` (the advection problem of Sec. 5).
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
    if kind == "heat2d_central":
        lap = {}
        for o, v in CENTRAL_D2[order].items():
            _add(lap, (o, 0), v * nx * nx)
            _add(lap, (0, o), v * ny * ny)
        for k, v in lap.items():
            _add(t, k, nu * v)
        return _pack(t, lap)
    if kind == "adv2d_upwind":
        vx, vy = vel
        for o, v in UPWIND_D1[order].items():
            _add(t, (o, 0), -vx * v * nx)
            _add(t, (0, o), -vy * v * ny)
        return _pack(t)
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
    return Plan(taps_for(w.kind, w.nx, w.ny, nu=w.nu, vel=w.vel, order=w.order), w.nx, w.ny, **kw)
