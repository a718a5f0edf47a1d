"""Periodic finite-difference operators A (oracle; test infrastructure only).

The paper's problems are linear IVPs u_t = A u with a constant matrix A
(Sec. 2, eq. (genericlinearform)); the workloads use periodic central stencils
on the unit interval or unit square with x_j = j / n, h = 1 / n.  A is built
here as an explicit scipy.sparse matrix row by row; its Fourier symbol (used by
the per-mode back-end) is the DFT of its first column, which holds for any
circulant matrix.
"""
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


def stencil_for(kind, nx, ny=1, nu=0.0, c=(0.0, 0.0)):
    """Operators of the synthetic workloads.

    * ``heat1d``:   nu (u_{j-1} - 2u_j + u_{j+1}) / h^2
    * ``heat2d``:   nu / h^2 times the 5-point Laplacian
    * ``adv1d_c4``: -c (-u_{j+2} + 8u_{j+1} - 8u_{j-1} + u_{j-2}) / (12 h)
    * ``advdiff2d``: nu Lap_h - c_x D_x - c_y D_y, 5-point Laplacian and
      second-order central first derivatives (u_{j+1} - u_{j-1}) / (2h);
      carries dA/dnu = Lap_h for the gradient with respect to nu.
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
    raise ValueError("unknown operator kind %r" % kind)
