"""All-at-once operators (oracle; test infrastructure only).

eq. (globalsys):  C = I_L (x) C_coll + E (x) H,  C_coll = I_MN - dT Q (x) A,
H = H_M (x) I_N with H_M's last column all ones (eq. (Hm)), E with -1 on the
lower sub-diagonal; w_1 = 1_M (x) u0 + dT (Q (x) I) b_1, w_l = dT (Q (x) I) b_l
(eq. (collocation); b = 0 unless a forcing array is given).
eq. (prec):  C_alpha = I_L (x) C_coll + E_alpha (x) H, E_alpha = E plus
-alpha in the top-right corner.
The preconditioned Richardson iteration (eq. (Riteration)) applies
C_alpha^{-1}; its defect-correction form u <- u + C_alpha^{-1}(w - C u) is
algebraically identical.  Here C_alpha^{-1} r is a plain sparse direct solve
of the assembled matrix - no diagonalisation, no transform over l.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _HM(M):
    H = np.zeros((M, M))
    H[:, M - 1] = 1.0
    return H


def _E(L, alpha=None):
    E = sp.diags([-np.ones(L - 1)], [-1], shape=(L, L), format="lil")
    if alpha is not None:
        E[0, L - 1] += -alpha
    return E.tocsr()


def _parts(op, Q, dt):
    A = op.matrix()
    M = Q.shape[0]
    N = A.shape[0]
    Ccoll = sp.identity(M * N, format="csr") - dt * sp.kron(sp.csr_matrix(Q), A, format="csr")
    H = sp.kron(sp.csr_matrix(_HM(M)), sp.identity(N), format="csr")
    return Ccoll, H


def assemble_C(op, Q, dt, L, batch_dims=()):
    """Sparse C of eq. (globalsys), size LMN x LMN."""
    Ccoll, H = _parts(op, Q, dt)
    return (sp.kron(sp.identity(L), Ccoll) + sp.kron(_E(L), H)).tocsr()


def assemble_C_alpha(op, Q, dt, L, alpha):
    """Sparse C_alpha of eq. (prec)."""
    Ccoll, H = _parts(op, Q, dt)
    return (sp.kron(sp.identity(L), Ccoll) + sp.kron(_E(L, alpha), H)).tocsr()


def assemble_w(u0, L, M, forcing=None, Q=None, dt=None):
    """w as an array [L, M, N]: u0 in every node of step 1, plus dT Q b_l in
    step l when forcing (b at the collocation times, [L, M, N]) is given."""
    u0 = np.asarray(u0)
    w = np.zeros((L, M, u0.size), dtype=u0.dtype)
    w[0, :, :] = u0[None, :]
    if forcing is not None:
        Q = np.asarray(Q, dtype=np.float64)
        for l in range(L):
            w[l] += dt * (Q @ np.asarray(forcing[l]).reshape(M, -1))
    return w


def residual(op, Q, dt, u0, U, forcing=None):
    """w - C U for U[L, M, N] (row a1 of the sweep), by sparse matvec."""
    L, M, N = U.shape
    C = assemble_C(op, Q, dt, L)
    return (assemble_w(u0, L, M, forcing, Q, dt).reshape(-1) - C @ U.reshape(-1)).reshape(L, M, N)


def precond_solve(op, Q, dt, alpha, R):
    """delta = C_alpha^{-1} R for R[L, M, N], by sparse LU of C_alpha."""
    L, M, N = R.shape
    Ca = assemble_C_alpha(op, Q, dt, L, alpha).tocsc()
    return spla.splu(Ca).solve(np.ascontiguousarray(R.reshape(-1))).reshape(L, M, N)


def brute_force_solve(op, Q, dt, u0, L, forcing=None):
    """Dense LAPACK solve of C U = w (tiny sizes only)."""
    M = Q.shape[0]
    C = assemble_C(op, Q, dt, L).toarray()
    w = assemble_w(u0, L, M, forcing, Q, dt).reshape(-1)
    return np.linalg.solve(C, w).reshape(L, M, -1)
