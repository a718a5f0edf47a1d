"""Collocation nodes and integration matrix (oracle; test infrastructure only).

Sec. 2.1, eq. (collocation): q_{mi} = int_0^{t_m} c_i(s) ds with c_i the
Lagrange polynomials of the nodes.  Sec. 2.3: the Radau-right nodes on [0, 1]
are the roots of P_{M-1} + P_M on [-1, 1] under x = -2t + 1, and the monic
node polynomial w_M(t) = prod (t - t_m).
"""
import numpy as np
from numpy.polynomial import legendre as _leg


def radau_right_nodes(M):
    """Radau IIA nodes 0 < t_1 < ... < t_M = 1 (Sec. 2.3, node polynomial).

    Roots of P_{M-1}(x) + P_M(x) (Legendre series, numpy), polished by Newton
    in FP64, mapped by t = (1 - x) / 2.  Pinned by the closed forms for M = 1,
    2, 3 in the tests.
    """
    if M < 1:
        raise ValueError("M must be >= 1")
    c = np.zeros(M + 1)
    c[M] = 1.0
    c[M - 1] += 1.0
    x = np.real(_leg.legroots(c))
    dc = _leg.legder(c)
    for _ in range(4):  # Newton polish on the Legendre series itself
        fx = _leg.legval(x, c)
        d = _leg.legval(x, dc)
        step = np.where(np.abs(x + 1.0) < 1e-14, 0.0, fx / np.where(d == 0, 1.0, d))
        x = x - step
    t = np.sort((1.0 - x) / 2.0)
    t[-1] = 1.0  # x = -1 is an exact root of P_{M-1} + P_M
    return t


def collocation_matrix(t):
    """Q with q_{mi} = int_0^{t_m} c_i(s) ds (Sec. 2.1, eq. (collocation)).

    Uses the property stated in the proof of Lemma 2: Q maps the nodal values
    of s^j to the nodal values of s^{j+1}/(j+1), j = 0..M-1, so Q W = W_int with
    the Vandermonde W_{mj} = t_m^j and (W_int)_{mj} = t_m^{j+1}/(j+1).
    """
    t = np.asarray(t, dtype=np.float64)
    M = t.size
    j = np.arange(M)
    W = t[:, None] ** j[None, :]
    W_int = t[:, None] ** (j[None, :] + 1) / (j[None, :] + 1)
    return np.linalg.solve(W.T, W_int.T).T


def node_polynomial(t):
    """Coefficients b_0..b_M (b_M = 1) of w_M(t) = prod (t - t_m) (Lemma 2)."""
    return np.poly(np.asarray(t, dtype=np.float64))[::-1].copy()
