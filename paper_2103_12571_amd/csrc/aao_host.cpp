// Host-side collocation math (see aao_host.hpp).
#include "aao_host.hpp"

#include <algorithm>
#include <cmath>

namespace aao {

namespace {

using ld = long double;

// P_{M-1}(x) + P_M(x) and its derivative by the three-term recurrence.
void legendre_sum(int M, ld x, ld& f, ld& df) {
  ld p0 = 1, p1 = x, d0 = 0, d1 = 1;  // P_0, P_1 and derivatives
  if (M == 1) {
    f = p0 + p1;
    df = d0 + d1;
    return;
  }
  for (int n = 1; n < M; ++n) {  // produce P_{n+1}
    ld p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1);
    ld d2 = ((2 * n + 1) * (p1 + x * d1) - n * d0) / (n + 1);
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  f = p0 + p1;  // P_{M-1} + P_M
  df = d0 + d1;
}

// Evaluate a monic-or-not complex polynomial sum c[k] z^k and derivative.
void poly_eval(const std::vector<cd>& c, cd z, cd& p, cd& dp) {
  p = 0;
  dp = 0;
  for (int k = (int)c.size() - 1; k >= 0; --k) {
    dp = dp * z + p;
    p = p * z + c[k];
  }
}

// All roots of sum c[k] z^k (degree n = c.size()-1 >= 1) by the Aberth-Ehrlich
// simultaneous iteration, each root then polished by Newton's method.
std::vector<cd> poly_roots(const std::vector<cd>& c) {
  const int n = (int)c.size() - 1;
  std::vector<cd> z(n);
  // start on a circle of radius bounded by Cauchy's bound, slightly rotated
  double R = 0;
  for (int k = 0; k < n; ++k) R = std::max(R, std::abs(c[k] / c[n]));
  R = 1 + R;
  for (int k = 0; k < n; ++k) z[k] = std::polar(0.5 * R, 2 * M_PI * (k + 0.25) / n + 0.4);
  for (int it = 0; it < 200; ++it) {  // cubic convergence: typically < 20 sweeps
    double maxstep = 0;
    for (int k = 0; k < n; ++k) {
      cd p, dp;
      poly_eval(c, z[k], p, dp);
      if (p == cd(0)) continue;
      cd ratio = p / dp;
      cd s = 0;
      for (int j = 0; j < n; ++j)
        if (j != k) s += 1.0 / (z[k] - z[j]);
      cd w = ratio / (1.0 - ratio * s);
      z[k] -= w;
      maxstep = std::max(maxstep, std::abs(w) / std::max(1.0, std::abs(z[k])));
    }
    if (maxstep < 1e-15) break;  // then Newton polishing below
  }
  for (int k = 0; k < n; ++k) {
    for (int it = 0; it < 3; ++it) {
      cd p, dp;
      poly_eval(c, z[k], p, dp);
      if (dp == cd(0)) break;
      z[k] -= p / dp;
    }
  }
  return z;
}

ld factorial(int n) {
  ld f = 1;
  for (int k = 2; k <= n; ++k) f *= k;
  return f;
}

}  // namespace

bool radau_right_nodes(int M, std::vector<double>& t) {
  if (M < 1 || M > 16) return false;
  t.assign(M, 0.0);
  // x = -1 is always a root; bracket the other M-1 roots on a fine grid in
  // (-1, 1] and refine by bisection + Newton.
  std::vector<ld> roots;
  const int G = 20000;
  ld xa = -1 + 1e-9L, fa, da;
  legendre_sum(M, xa, fa, da);
  for (int g = 1; g <= G && (int)roots.size() < M - 1; ++g) {
    ld xb = -1 + 2.0L * g / G, fb, db;
    legendre_sum(M, xb, fb, db);
    if ((fa < 0) != (fb < 0) || fb == 0) {
      ld lo = xa, hi = xb, flo = fa;
      for (int it = 0; it < 200; ++it) {
        ld mid = 0.5L * (lo + hi), fm, dm;
        legendre_sum(M, mid, fm, dm);
        if ((fm < 0) == (flo < 0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      ld x = 0.5L * (lo + hi);
      for (int it = 0; it < 3; ++it) {
        ld f, d;
        legendre_sum(M, x, f, d);
        if (d != 0) x -= f / d;
      }
      roots.push_back(x);
    }
    xa = xb;
    fa = fb;
  }
  if ((int)roots.size() != M - 1) return false;
  std::vector<double> tt;
  for (ld x : roots) tt.push_back((double)((1 - x) / 2));
  tt.push_back(1.0);
  std::sort(tt.begin(), tt.end());
  t = tt;
  return true;
}

void collocation_matrix(const std::vector<double>& t, std::vector<double>& Q) {
  const int M = (int)t.size();
  Q.assign(M * M, 0.0);
  for (int i = 0; i < M; ++i) {
    // monomial coefficients of the Lagrange polynomial c_i
    std::vector<ld> c(1, 1.0L);
    ld denom = 1;
    for (int k = 0; k < M; ++k) {
      if (k == i) continue;
      std::vector<ld> nc(c.size() + 1, 0.0L);
      for (size_t e = 0; e < c.size(); ++e) {
        nc[e + 1] += c[e];
        nc[e] -= (ld)t[k] * c[e];
      }
      c.swap(nc);
      denom *= (ld)t[i] - (ld)t[k];
    }
    for (int m = 0; m < M; ++m) {
      ld tm = t[m], acc = 0, pw = tm;
      for (size_t e = 0; e < c.size(); ++e) {
        acc += c[e] * pw / (ld)(e + 1);
        pw *= tm;
      }
      Q[m * M + i] = (double)(acc / denom);
    }
  }
}

bool invert(int n, const std::vector<cd>& A, std::vector<cd>& Ainv) {
  std::vector<cd> a(A);
  Ainv.assign(n * n, cd(0));
  for (int i = 0; i < n; ++i) Ainv[i * n + i] = 1;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::abs(a[r * n + col]) > std::abs(a[piv * n + col])) piv = r;
    if (std::abs(a[piv * n + col]) == 0) return false;
    if (piv != col)
      for (int k = 0; k < n; ++k) {
        std::swap(a[piv * n + k], a[col * n + k]);
        std::swap(Ainv[piv * n + k], Ainv[col * n + k]);
      }
    cd inv = 1.0 / a[col * n + col];
    for (int k = 0; k < n; ++k) {
      a[col * n + k] *= inv;
      Ainv[col * n + k] *= inv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      cd f = a[r * n + col];
      if (f == cd(0)) continue;
      for (int k = 0; k < n; ++k) {
        a[r * n + k] -= f * a[col * n + k];
        Ainv[r * n + k] -= f * Ainv[col * n + k];
      }
    }
  }
  return true;
}

std::string freq_table(const std::vector<double>& t, const std::vector<double>& Q, double alpha,
                       int L, int j, FreqTable& out) {
  const int M = (int)t.size();
  // Lemma 1: d_j = -alpha^{1/L} e^{-2 pi i j / L}; eq. (QGL): r_j = d_j / (1 + d_j).
  const double a = std::pow(alpha, 1.0 / L);
  out.d = -a * std::exp(cd(0, -2.0 * M_PI * (double)j / (double)L));
  out.r = out.d / (1.0 + out.d);
  // K = Q G_j^{-1} = Q - r_j D_t H_M: column M-1 gets -r_j t_m.
  std::vector<cd> K(M * M);
  for (int m = 0; m < M; ++m)
    for (int i = 0; i < M; ++i) K[m * M + i] = Q[m * M + i] - (i == M - 1 ? out.r * t[m] : cd(0));
  out.lam.assign(M, 0);
  out.S.assign(M * M, 0);
  if (M == 1) {
    out.lam[0] = K[0];
    out.S[0] = 1;
  } else {
    // Lemma 2 with the sign of eq. (QGL): the eigenvalues of Q - r D_t H_M are
    // the roots of p_M(lambda) with r replaced by -r, where w_M = prod(t - t_m)
    // = sum b_k t^k and c_0 = (1 - r) b_0, c_m = m! b_m + r sum_{k>=1}
    // (m+k)!/k! b_{m+k}, c_M = M!.
    std::vector<ld> b(1, 1.0L);
    for (int k = 0; k < M; ++k) {
      std::vector<ld> nb(b.size() + 1, 0.0L);
      for (size_t e = 0; e < b.size(); ++e) {
        nb[e + 1] += b[e];
        nb[e] -= (ld)t[k] * b[e];
      }
      b.swap(nb);
    }
    const cd r = out.r;
    std::vector<cd> c(M + 1);
    c[M] = (double)factorial(M);
    c[0] = (1.0 - r) * (double)b[0];
    for (int m = 1; m < M; ++m) {
      cd s = 0;
      for (int k = 1; k <= M - m; ++k) s += (double)(factorial(m + k) / factorial(k) * b[m + k]);
      c[m] = (double)(factorial(m) * b[m]) + r * s;
    }
    std::vector<cd> lam = poly_roots(c);
    // Eigenvector of lambda (proof of Lemma 2): g(t) = sum_{k=1}^M a_k t^k with
    // a_M = 1, a_k = sum_{i=0}^{M-k} lambda^i (k+i)!/k! b_{k+i} (k >= 2),
    // a_1 = -b_0 / lambda; the eigenvector is h = g' at the nodes.
    for (int e = 0; e < M; ++e) {
      const cd lm = lam[e];
      std::vector<cd> acoef(M + 1, 0.0);
      acoef[M] = 1.0;
      for (int k = M - 1; k >= 2; --k) acoef[k] = (double)b[k] + (double)(k + 1) * lm * acoef[k + 1];
      acoef[1] = -(double)b[0] / lm;
      double nrm = 0;
      for (int m = 0; m < M; ++m) {
        cd h = 0, pw = 1;
        for (int k = 1; k <= M; ++k) {
          h += (double)k * acoef[k] * pw;
          pw *= t[m];
        }
        out.S[m * M + e] = h;
        nrm += std::norm(h);
      }
      nrm = std::sqrt(nrm);
      for (int m = 0; m < M; ++m) out.S[m * M + e] /= nrm;
    }
    out.lam = lam;
  }
  if (!invert(M, out.S, out.Sinv)) return "eigenvector matrix S_j is singular";
  double n1 = 0, n1i = 0, kmax = 0, lmax = 0;
  for (int col = 0; col < M; ++col) {
    double s1 = 0, s2 = 0;
    for (int row = 0; row < M; ++row) {
      s1 += std::abs(out.S[row * M + col]);
      s2 += std::abs(out.Sinv[row * M + col]);
    }
    n1 = std::max(n1, s1);
    n1i = std::max(n1i, s2);
  }
  out.cond = n1 * n1i;
  out.gap = 1e300;
  for (int e = 0; e < M; ++e) lmax = std::max(lmax, std::abs(out.lam[e]));
  for (int e = 0; e < M; ++e)
    for (int f = e + 1; f < M; ++f) out.gap = std::min(out.gap, std::abs(out.lam[e] - out.lam[f]) / lmax);
  if (M == 1) out.gap = 1.0;
  double err = 0;
  for (int m = 0; m < M; ++m)
    for (int i = 0; i < M; ++i) {
      cd v = 0;
      for (int e = 0; e < M; ++e) v += out.S[m * M + e] * out.lam[e] * out.Sinv[e * M + i];
      err = std::max(err, std::abs(v - K[m * M + i]));
      kmax = std::max(kmax, std::abs(K[m * M + i]));
    }
  out.recon = err / kmax;
  if (!(out.cond < 1e8) || !(out.gap > 1e-8) || !(out.recon < 1e-9))
    return "Q G_j^{-1} is not well diagonalisable (cond(S)=" + std::to_string(out.cond) +
           ", rel. eigenvalue gap=" + std::to_string(out.gap) + ", reconstruction error=" +
           std::to_string(out.recon) + ")";
  return "";
}

namespace {

// In-place unnormalised forward DFT (e^{-2 pi i jk / P}) of a power-of-two
// length: bit-reversal permutation, then radix-2 butterflies.
void dft_pow2(std::vector<cd>& v) {
  const int P = (int)v.size();
  for (int i = 1, j = 0; i < P; ++i) {
    int bit = P >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(v[i], v[j]);
  }
  for (int len = 2; len <= P; len <<= 1) {
    for (int k = 0; k < len / 2; ++k) {
      const double ang = -2.0 * M_PI * k / len;
      const cd w(std::cos(ang), std::sin(ang));
      for (int i = 0; i < P; i += len) {
        const cd a = v[i + k], b = w * v[i + k + len / 2];
        v[i + k] = a + b;
        v[i + k + len / 2] = a - b;
      }
    }
  }
}

}  // namespace

void bluestein_tables(int n, int P, std::vector<cd>& W, std::vector<cd>& ch, std::vector<cd>& Bf,
                      std::vector<cd>& Bi) {
  W.resize(P);
  for (int k = 0; k < P; ++k) W[k] = cd(std::cos(2.0 * M_PI * k / P), std::sin(2.0 * M_PI * k / P));
  ch.resize(n);
  for (int j = 0; j < n; ++j) {
    const long long q = ((long long)j * j) % (2LL * n);  // e^{-i pi j^2 / n} has period 2n in j^2
    const double ang = -M_PI * (double)q / n;
    ch[j] = cd(std::cos(ang), std::sin(ang));
  }
  Bf.assign(P, cd(0, 0));
  Bi.assign(P, cd(0, 0));
  for (int m = 0; m < n; ++m) {
    Bf[m] = std::conj(ch[m]);
    Bi[m] = ch[m];
    if (m > 0) {
      Bf[P - m] = std::conj(ch[m]);
      Bi[P - m] = ch[m];
    }
  }
  dft_pow2(Bf);
  dft_pow2(Bi);
}

}  // namespace aao
