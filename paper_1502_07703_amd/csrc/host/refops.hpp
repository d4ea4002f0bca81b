// Host-side FP64 builders: quadrature, Jacobi and Lagrange polynomials, the
// semi-nodal basis of Lemma 3 and the reference operators of Algorithms 1-3.
#pragma once

#include <cstdint>
#include <vector>

namespace dgpyr {

inline int n_basis(int N) { return (N + 1) * (N + 2) * (2 * N + 3) / 6; }

// n-point Gauss-Jacobi rule for the weight (1 - x)^alpha (beta = 0), nodes
// ascending.  alpha = 0 gives Gauss-Legendre.
void gauss_jacobi(int n, double alpha, std::vector<double>& x, std::vector<double>& w);

// P_n^{(alpha, 0)}(x), standard normalisation P_n(1) = binom(n + alpha, n), and
// its derivative.
double jacobi_p(int n, double alpha, double beta, double x);
double jacobi_dp(int n, double alpha, double beta, double x);

// Lagrange polynomial i on the given nodes, and its derivative.
double lagrange(const std::vector<double>& nodes, int i, double x);
double lagrange_d(const std::vector<double>& nodes, int i, double x);

// Reference data for degree N.  Point orders used on the device:
//   volume point q = p + (N+1) * (m + (N+1) * r): a = xg[p], b = xg[m],
//     c = xc[r] (Gauss-Jacobi(2,0)); reference weight wv[q] = wg wg wc / 4.
//   face f point q = p + (N+1) * m within the face, faces ordered
//     0: base c = -1, (a, b) = (xg[p], xg[m]), weight wg[p] wg[m];
//     1: a = -1, 2: a = +1 with (b, c) = (xg[p], xt[m]);
//     3: b = -1, 4: b = +1 with (a, c) = (xg[p], xt[m]);
//     triangle weight wg[p] wt[m] / 2 (Gauss-Jacobi(1,0) in c).
struct RefOps {
  int N = 0, Np = 0, Nq1 = 0, Nc = 0, Nfq = 0, Nfc = 0;
  std::vector<double> xg, wg;   // (N+1)-point Gauss-Legendre
  std::vector<double> xc, wc;   // (N+1)-point Gauss-Jacobi (2,0)
  std::vector<double> xt, wt;   // (N+1)-point Gauss-Jacobi (1,0)
  std::vector<double> wv;       // [Nc] volume weights
  std::vector<double> wf;       // [Nfc] face parameter weights
  std::vector<double> fa, fb, fc;  // [Nfc] collapsed coordinates of face points
  // Row-major operators
  std::vector<double> V;        // [Nc][Np]   phi_n at volume points
  std::vector<double> Dr, Ds, Dt;  // [Nc][Np] reference derivatives
  std::vector<double> Vf;       // [Nfc][Np]  phi_n at face points
  // Diagonal of the reference mass matrix and the (a, b) node of each basis
  // function: M_nn(K) = J_K(na[n], nb[n]) * wwc[n].
  std::vector<double> wwc, na, nb;
  std::vector<int> bi, bj, bk;  // (i, j, k) of each basis index
  // One-dimensional factors of the basis for sum factorisation, with
  // n1 = N + 1 and h = (1 - c)/2, g_k = h^k P_{N-k}^{(2k+3,0)}:
  std::vector<double> sfLa;  // [k][p][i] l^k_i(xg[p]), zero for i > k
  std::vector<double> sfDa;  // [k][p][i] d/da l^k_i(xg[p])
  std::vector<double> sfLe;  // [k][s][i] l^k_i(-1) (s = 0), l^k_i(+1) (s = 1)
  std::vector<double> sfG;   // [r][k] g_k(xc[r])
  std::vector<double> sfGt;  // [r][k] h^(k-1) P_{N-k}(xc[r]) (zero for k = 0)
  std::vector<double> sfGp;  // [r][k] g_k'(xc[r])
  std::vector<double> sfGb;  // [k]    g_k(-1)
  std::vector<double> sfGf;  // [m][k] g_k(xt[m])
};

// Values of all Np basis functions of degree N at collapsed (a, b, c).
void eval_basis(int N, double a, double b, double c, double* v);

// Builds all reference data; returns false (with a message) if an internal
// consistency check fails (Lemma 2 constant, reference mass diagonality).
bool build_refops(int N, RefOps& ops, char* msg, int msglen);

// Face-point permutations between two sides of a face.  For a quad face the
// orientation o in 0..7 encodes the signed permutation (a, b) -> (a', b');
// for a triangle o in {0, 1} flips the edge coordinate.  Writes the
// neighbour-side point index of each own point.
void quad_perm(int N, int o, int* perm);
void tri_perm(int N, int o, int* perm);

}  // namespace dgpyr
