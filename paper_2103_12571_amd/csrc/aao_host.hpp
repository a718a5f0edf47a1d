// Host-side collocation math for the alpha-circulant sweep (FP64, small M).
//
// Nodes and Q follow Sec. 2.1 (eq. (collocation)) and Sec. 2.3 (Radau-right
// node polynomial); the per-alpha tables follow Lemma 1 (d_l), eq. (QGL)
// (G_l^{-1} = I - r_l H_M, Q G_l^{-1} = Q - r_l D_t H_M) and Lemma 2
// (eigenvalues as roots of a degree-M polynomial, eigenvectors as the
// derivative of a polynomial g evaluated at the nodes).
#pragma once
#include <complex>
#include <string>
#include <vector>

namespace aao {

using cd = std::complex<double>;

// Radau-right nodes 0 < t_1 < ... < t_M = 1: roots of P_{M-1} + P_M on [-1, 1]
// under x = 1 - 2t (Sec. 2.3).  Returns false if M is out of range.
bool radau_right_nodes(int M, std::vector<double>& t);

// Q[m][i] = int_0^{t_m} c_i(s) ds (eq. (collocation)); row-major M x M, by exact
// integration of the Lagrange polynomials in extended precision.
void collocation_matrix(const std::vector<double>& t, std::vector<double>& Q);

// One frequency j of the alpha-circulant diagonalisation.
struct FreqTable {
  cd d;                     // d_j = -alpha^{1/L} exp(-2 pi i j / L)          (Lemma 1)
  cd r;                     // r_j = d_j / (1 + d_j)                           (eq. (QGL))
  std::vector<cd> lam;      // eigenvalues d_jm of Q G_j^{-1}, M               (Lemma 2)
  std::vector<cd> S;        // eigenvectors as columns, row-major M x M, unit 2-norm
  std::vector<cd> Sinv;     // S^{-1}
  double cond;              // ||S||_1 ||S^{-1}||_1
  double gap;               // min |lam_a - lam_b| / max |lam|
  double recon;             // max |S D S^{-1} - Q G^{-1}| / max |Q G^{-1}|
};

// Builds the eigen-table of Q G_j^{-1} for frequency j.  Returns an empty string
// on success, else the reason the matrix is not (well) diagonalisable.
std::string freq_table(const std::vector<double>& t, const std::vector<double>& Q, double alpha,
                       int L, int j, FreqTable& out);

// Small dense complex inverse (Gauss-Jordan, partial pivoting).  False if singular.
bool invert(int n, const std::vector<cd>& A, std::vector<cd>& Ainv);

// Tables of Bluestein's chirp-z DFT of length n through cyclic convolutions of
// length P (a power of two >= 2n - 1): W[k] = e^{+2 pi i k / P} (k < P),
// ch[j] = e^{-i pi j^2 / n} (j < n, with j^2 reduced mod 2n first), and the
// length-P DFTs Bf of the forward filter (conj(ch_m) at m and P - m) and Bi of
// the inverse filter (ch_m at m and P - m).
void bluestein_tables(int n, int P, std::vector<cd>& W, std::vector<cd>& ch, std::vector<cd>& Bf,
                      std::vector<cd>& Bi);

}  // namespace aao
