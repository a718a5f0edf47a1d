"""Periodic finite-difference operators A (oracle; test infrastructure only).

The paper's problems are linear IVPs u_t = A u with a constant matrix A
(Sec. 2, eq. (genericlinearform)); the workloads use periodic central stencils
on the unit interval or unit square with x_j = j / n, h = 1 / n.  A is built
here as an explicit scipy.sparse matrix row by row; its Fourier symbol (used by
the per-mode back-end) is the DFT of its first column, which holds for any
circulant matrix.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import scipy.sparse as sp


class PeriodicStencil:
    """A periodic constant-coefficient operator on an nx (x ny) grid.

    ``weights`` maps an offset (dx,) or (dx, dy) to a real coefficient; the
    operator is (A u)[x, y] = sum w * u[x + dx, y + dy] with periodic wrap and
    the flattened index n = y * nx + x.
    """

    def __init__(self, nx, ny, weights, d_dnu=None):
        self.nx = int(nx)
        self.ny = int(ny)
        self.ndim = 1 if self.ny == 1 else 2
        self.weights = dict(weights)
        self.d_dnu = None if d_dnu is None else dict(d_dnu)

    @property
    def N(self):
        return self.nx * self.ny

    def _build(self, weights):
        nx, ny = self.nx, self.ny
        n = np.arange(nx * ny)
        x, y = n % nx, n // nx
        rows, cols, vals = [], [], []
        for off, w in weights.items():
            dx = off[0]
            dy = off[1] if len(off) > 1 else 0
            cols.append(((y + dy) % ny) * nx + (x + dx) % nx)
            rows.append(n)
            vals.append(np.full(n.size, float(w)))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(nx * ny, nx * ny))

    def matrix(self):
        return self._build(self.weights)

    def matrix_d_dnu(self):
        """dA/dnu (only for operators that carry a nu derivative)."""
        if self.d_dnu is None:
            raise ValueError("operator has no nu derivative")
        return self._build(self.d_dnu)

    def symbol(self):
        """Eigenvalues of the circulant A indexed like numpy's fft (ny, nx)."""
        e0 = np.zeros(self.N)
        e0[0] = 1.0
        col = self.matrix() @ e0
        return np.fft.fft2(col.reshape(self.ny, self.nx))


def _lap1d(nu, n):
    s = nu * n * n
    return {(-1,): s, (0,): -2.0 * s, (1,): s}


def _lap2d(nu, nx, ny):
    sx = nu * nx * nx
    sy = nu * ny * ny
    return {(-1, 0): sx, (1, 0): sx, (0, -1): sy, (0, 1): sy, (0, 0): -2.0 * (sx + sy)}


def fd_weights(offsets, deriv):
    """Weights w_j on the integer offsets j with sum_j w_j f(x + j h) =
    h^deriv f^(deriv)(x) + O(h^(len(offsets))): the moment conditions
    sum_j w_j j^p = deriv! [p == deriv], p = 0 .. len(offsets) - 1, solved
    exactly in rationals (Gauss-Jordan on the Vandermonde system)."""
    offs = [int(o) for o in offsets]
    n = len(offs)
    a = [[Fraction(o) ** p for o in offs] + [Fraction(factorial(deriv) if p == deriv else 0)] for p in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        inv = 1 / a[col][col]
        a[col] = [v * inv for v in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [v - f * w for v, w in zip(a[r], a[col])]
    return {o: a[i][n] for i, o in enumerate(offs)}


def central_d2(order):
    """Central second derivative of even order: offsets -order/2 .. order/2."""
    h = order // 2
    return fd_weights(range(-h, h + 1), 2)


def upwind_d1(order):
    """Upwind-biased first derivative of order 1..5 for a positive velocity:
    order + 1 offsets, one more upwind (negative) than downwind for odd
    orders, two more for even ones."""
    lo = -((order + 2) // 2)
    return fd_weights(range(lo, lo + order + 1), 1)


def stencil_for(kind, nx, ny=1, nu=0.0, c=(0.0, 0.0), order=2):
    """Operators of the synthetic workloads.

    * ``heat1d``:   nu (u_{j-1} - 2u_j + u_{j+1}) / h^2
    * ``heat2d``:   nu / h^2 times the 5-point Laplacian
    * ``adv1d_c4``: -c (-u_{j+2} + 8u_{j+1} - 8u_{j-1} + u_{j-2}) / (12 h)
    * ``advdiff2d``: nu Lap_h - c_x D_x - c_y D_y, 5-point Laplacian and
      second-order central first derivatives (u_{j+1} - u_{j-1}) / (2h);
      carries dA/dnu = Lap_h for the gradient with respect to nu.
    * ``heat2d_central``: nu Lap_h with central differences of order
      ``order`` (2, 4, 6), the heat problem of Sec. 5 (eq. (heat)).
    * ``adv2d_upwind``: -(c_x D_x + c_y D_y) with upwind differences of order
      ``order`` (1..5), the advection problem of Sec. 5 (eq. (advection)).
    """
    if kind == "heat1d":
        return PeriodicStencil(nx, 1, _lap1d(nu, nx))
    if kind == "heat2d":
        return PeriodicStencil(nx, ny, _lap2d(nu, nx, ny))
    if kind == "adv1d_c4":
        cx = c[0] if np.ndim(c) else c
        s = -cx * nx / 12.0
        return PeriodicStencil(nx, 1, {(-2,): s * 1.0, (-1,): s * -8.0, (1,): s * 8.0, (2,): s * -1.0})
    if kind == "advdiff2d":
        lap = _lap2d(nu, nx, ny)
        cx, cy = c
        w = dict(lap)
        w[(1, 0)] += -cx * nx / 2.0
        w[(-1, 0)] += cx * nx / 2.0
        w[(0, 1)] += -cy * ny / 2.0
        w[(0, -1)] += cy * ny / 2.0
        d = _lap2d(1.0, nx, ny)
        return PeriodicStencil(nx, ny, w, d_dnu=d)
    if kind == "heat2d_central":
        # nu Lap_h with central second differences of order `order` in x and y
        w = {}
        for o, v in central_d2(order).items():
            w[(o, 0)] = w.get((o, 0), 0.0) + nu * float(v) * nx * nx
            w[(0, o)] = w.get((0, o), 0.0) + nu * float(v) * ny * ny
        return PeriodicStencil(nx, ny, w)
    if kind == "adv2d_upwind":
        # -(c_x D_x + c_y D_y) with upwind differences of order `order`
        # (velocities c_x, c_y > 0)
        cx, cy = c
        w = {}
        for o, v in upwind_d1(order).items():
            w[(o, 0)] = w.get((o, 0), 0.0) - cx * float(v) * nx
            w[(0, o)] = w.get((0, o), 0.0) - cy * float(v) * ny
        return PeriodicStencil(nx, ny, w)
    raise ValueError("unknown operator kind %r" % kind)
