"""Alpha schedule of Alg. 2 (oracle; test infrastructure only).

Sec. 3.3: gamma = L (3 eps + tau) ||w||_inf; for k = 0, 1, ...:
m_{k+1} = 2 sqrt(m_k gamma) and alpha_{k+1} = sqrt(gamma / m_k), while
m_k > tol.  Pinned by the alpha sequence printed for Fig. 3 and by the
closed form m_k = (4 gamma)^(1 - 2^-k) m_0^(2^-k) of Sec. 3.3.
"""
import math


def alpha_schedule(gamma, m0, n, tol=0.0):
    """First n pairs (alpha_{k+1}, m_{k+1}) of Alg. 2 (stops early if m_k <= tol)."""
    out = []
    m = float(m0)
    for _ in range(n):
        if m <= tol:
            break
        alpha = math.sqrt(gamma / m)
        m = 2.0 * math.sqrt(m * gamma)
        out.append((alpha, m))
    return out
