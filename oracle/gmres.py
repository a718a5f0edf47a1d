"""Outer Krylov solver for C u = w preconditioned by C_alpha (oracle; test
infrastructure only).

The paper points to Krylov acceleration of the alpha-circulant iteration as an
alternative to Richardson (introduction, Sec. 6).  Written here from the
definition of flexible GMRES with right preconditioning (Saad, "A flexible
inner-outer preconditioned GMRES algorithm", 1993): after j steps of a cycle
that starts at x0 with r0 = b - C x0, the iterate is x0 + Z_j y with
z_i = M_i^{-1} v_i, where v_1 = r0 / ||r0|| and the v_i are orthonormalised
by Arnoldi (modified Gram-Schmidt) against C z_i; y minimises
|| ||r0|| e_1 - H_j y || for the (j+1) x j Hessenberg matrix H_j, which equals
|| b - C (x0 + Z_j y) ||.  The small least-squares problem is solved with
numpy's lstsq.  Pinned by finite termination on tiny systems, by the
minimal-residual property against an explicit Krylov basis, and by the
closed form of one GMRES(1) step.
"""
import numpy as np
import scipy.sparse.linalg as spla

from .allatonce import assemble_C, assemble_C_alpha, assemble_w


def fgmres(apply_C, apply_prec, b, x0, restart, tol, max_steps):
    """Flexible GMRES(restart) for C x = b; apply_prec(v, k) = M_k^{-1} v for
    the k-th step overall (k = 0, 1, ...).  Stops when the least-squares
    residual of a step is at most tol ||b||, or after max_steps steps.

    Returns (x, hist, Z): hist[k] = estimated ||b - C x|| / ||b|| after step
    k + 1; Z the preconditioned vectors of the last cycle.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    bnorm = np.linalg.norm(b)
    hist = []
    k = 0
    Z = []
    while k < max_steps:
        r0 = b - apply_C(x)
        beta = np.linalg.norm(r0)
        if beta <= tol * bnorm:
            break
        V = [r0 / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        y = np.zeros(0)
        for j in range(restart):
            z = apply_prec(V[j], k)
            Z.append(z)
            w = apply_C(z)
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y = np.linalg.lstsq(H[:j + 2, :j + 1], e1, rcond=None)[0]
            res = np.linalg.norm(e1 - H[:j + 2, :j + 1] @ y)
            hist.append(res / bnorm)
            k += 1
            if res <= tol * bnorm or k >= max_steps or H[j + 1, j] == 0:
                break
        x = x + np.array(Z).T @ y
        if hist and hist[-1] <= tol:
            break
    return x, hist, Z


def gmres_solve(op, Q, dt, u0, L, alphas, restart, tol, max_steps, forcing=None):
    """Solve C U = w (eq. (globalsys)) by flexible GMRES with right
    preconditioner C_alpha (eq. (prec)); alphas[k] is used at step k (the
    last value repeats).  Starts from u0 at every node.  Returns (U, hist)."""
    M = Q.shape[0]
    N = op.N
    C = assemble_C(op, Q, dt, L).tocsr()
    w = assemble_w(u0, L, M, forcing, Q, dt).reshape(-1)
    lus = {}

    def prec(v, k):
        a = float(alphas[min(k, len(alphas) - 1)])
        if a not in lus:
            lus[a] = spla.splu(assemble_C_alpha(op, Q, dt, L, a).tocsc())
        return lus[a].solve(v)

    x0 = np.tile(np.asarray(u0, dtype=np.float64), L * M)
    x, hist, _ = fgmres(lambda v: C @ v, prec, w, x0, restart, tol, max_steps)
    return x.reshape(L, M, N), hist
