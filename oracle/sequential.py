"""Sequential step-by-step collocation (oracle; test infrastructure only).

Sec. 2.1, eq. (seq_collocation_problem): for l = 1..L solve

    (I_MN - dT Q (x) A) U_l = 1_M (x) u_{l-1} + dT (Q (x) I_N) b_l,    u_l := U_{l,M},

starting from u_0, where b_l holds the source b(t) at the step's collocation
times t_{l-1} + tau_m dT (eq. (collocation); b = 0 unless ``forcing`` is given).  The result U is the unique solution of the composite
system C U = w (eq. (globalsys)); it is the converged answer of the
alpha-circulant Richardson iteration, which therefore is compared with it on U only.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _rhs(prev, Q, dt, forcing, l):
    M = Q.shape[0]
    r = np.tile(prev, M)
    if forcing is not None:
        r = r + dt * (Q @ np.asarray(forcing[l]).reshape(M, -1)).reshape(-1)
    return r


def _solve_dense(A, Q, dt, u0, L, forcing):
    M = Q.shape[0]
    N = A.shape[0]
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    Ccoll = np.eye(M * N) - dt * np.kron(Q, Ad)
    U = np.empty((L, M, N), dtype=np.result_type(Ccoll, u0))
    prev = np.asarray(u0)
    for l in range(L):
        U[l] = np.linalg.solve(Ccoll, _rhs(prev, Q, dt, forcing, l)).reshape(M, N)
        prev = U[l, M - 1]
    return U


def _solve_sparse(A, Q, dt, u0, L, forcing):
    M = Q.shape[0]
    N = A.shape[0]
    Ccoll = (sp.identity(M * N, format="csc") - dt * sp.kron(sp.csr_matrix(Q), A)).tocsc()
    lu = spla.splu(Ccoll)
    U = np.empty((L, M, N), dtype=np.result_type(Ccoll.dtype, u0))
    prev = np.asarray(u0)
    for l in range(L):
        U[l] = lu.solve(_rhs(prev, Q, dt, forcing, l)).reshape(M, N)
        prev = U[l, M - 1]
    return U


def _solve_spectral(op, Q, dt, u0, L, forcing):
    """Per Fourier mode k: (I_M - dT lam_k Q) U_l(k) = 1_M U_{l-1,M}(k) + dT Q b_l(k).

    A periodic constant-coefficient stencil is circulant, so the DFT in space
    block-diagonalises I - dT Q (x) A into one M x M system per mode.
    """
    M = Q.shape[0]
    ny, nx = op.ny, op.nx
    lam = op.symbol().reshape(-1)
    K = lam.size
    sysm = np.eye(M)[None, :, :] - dt * lam[:, None, None] * Q[None, :, :]
    uh = np.fft.fft2(np.asarray(u0).reshape(ny, nx)).reshape(-1)
    real_in = np.isrealobj(u0)
    U = np.empty((L, M, K), dtype=np.float64 if real_in else np.complex128)
    for l in range(L):
        rhs = np.repeat(uh[:, None], M, axis=1)
        if forcing is not None:
            bh = np.stack([np.fft.fft2(np.asarray(forcing[l][m]).reshape(ny, nx)).reshape(-1) for m in range(M)], 1)
            rhs = rhs + dt * (bh @ Q.T)
        Uh = np.linalg.solve(sysm, rhs[..., None])[..., 0]  # (K, M)
        for m in range(M):
            v = np.fft.ifft2(Uh[:, m].reshape(ny, nx)).reshape(-1)
            U[l, m] = v.real if real_in else v
        uh = Uh[:, M - 1]
    return U


def sequential_solve(op, Q, dt, u0, L, backend="sparse", forcing=None):
    """Composite collocation solution U[l, m, n] (l = 0..L-1 is step l+1).

    backend: ``dense`` (LAPACK on I - dT Q (x) A, tiny sizes), ``sparse``
    (scipy splu, factorised once) or ``spectral`` (per-Fourier-mode M x M
    solves; exact for the circulant operators of the workloads).
    forcing: None (b = 0) or b at the collocation times, array [L, M, N].
    """
    Q = np.asarray(Q, dtype=np.float64)
    if backend == "dense":
        return _solve_dense(op.matrix(), Q, dt, u0, L, forcing)
    if backend == "sparse":
        return _solve_sparse(op.matrix(), Q, dt, u0, L, forcing)
    if backend == "spectral":
        return _solve_spectral(op, Q, dt, u0, L, forcing)
    raise ValueError("unknown backend %r" % backend)
