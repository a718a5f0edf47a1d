"""Adjoint of the composite collocation system (oracle; test infrastructure).

For the loss J = 1/2 ||u_{L,M} - u_target||^2 with C(nu) U = w(u0)
(eq. (globalsys), b = 0), the adjoint state solves C^T lambda = g with
g = e_{L,M} (x) (U_{L,M} - u_target).  C^T is block upper bidiagonal with
diagonal blocks C_coll^T and super-diagonal blocks -H^T, so lambda follows
from a backward sequential sweep:

    C_coll^T lambda_L = g_L,   C_coll^T lambda_l = g_l + H^T lambda_{l+1},

where (H^T v)_m = [m = M] sum_{m'} v_{m'}.  Then
dJ/du0 = sum_m lambda_{1,m} (w_1 = 1_M (x) u0) and
dJ/dnu = -lambda^T (dC/dnu) U = dT sum_l lambda_l^T (Q (x) dA/dnu) U_l.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import PeriodicStencil


def _transposed(op):
    w = {tuple(-o for o in off): v for off, v in op.weights.items()}
    return PeriodicStencil(op.nx, op.ny, w)


def adjoint_solve(op, Q, dt, g_last, L, backend="sparse"):
    """lambda[L, M, N] solving C^T lambda = e_{L,M} (x) g_last."""
    Q = np.asarray(Q, dtype=np.float64)
    M = Q.shape[0]
    N = op.N
    g_last = np.asarray(g_last)
    lam = np.zeros((L, M, N), dtype=np.result_type(g_last, np.float64))
    if backend == "sparse":
        A = op.matrix()
        CcT = (sp.identity(M * N, format="csc")
               - dt * sp.kron(sp.csr_matrix(Q.T), A.T.tocsr())).tocsc()
        lu = spla.splu(CcT)
        solve = lambda rhs: lu.solve(rhs.reshape(-1)).reshape(M, N)
    elif backend == "spectral":
        opT = _transposed(op)
        mu = opT.symbol().reshape(-1)
        sysm = np.eye(M)[None] - dt * mu[:, None, None] * Q.T[None]
        real_in = np.isrealobj(g_last)

        def solve(rhs):
            rh = np.stack([np.fft.fft2(rhs[m].reshape(op.ny, op.nx)).reshape(-1) for m in range(M)], 1)
            sol = np.linalg.solve(sysm, rh[..., None])[..., 0]
            out = np.stack([np.fft.ifft2(sol[:, m].reshape(op.ny, op.nx)).reshape(-1) for m in range(M)])
            return out.real if real_in else out
    else:
        raise ValueError("unknown backend %r" % backend)
    for l in range(L - 1, -1, -1):
        rhs = np.zeros((M, N), dtype=lam.dtype)
        if l == L - 1:
            rhs[M - 1] += g_last
        else:
            rhs[M - 1] += lam[l + 1].sum(axis=0)
        lam[l] = solve(rhs)
    return lam


def gradients(op, Q, dt, U, lam):
    """(dJ/du0 [N], dJ/dnu scalar) from the forward and adjoint states."""
    Q = np.asarray(Q, dtype=np.float64)
    L, M, N = U.shape
    g_u0 = lam[0].sum(axis=0)
    dA = op.matrix_d_dnu()
    g_nu = 0.0
    for l in range(L):
        dAU = np.stack([dA @ U[l, m] for m in range(M)])
        g_nu += dt * np.sum(lam[l] * (Q @ dAU))
    return g_u0, g_nu
