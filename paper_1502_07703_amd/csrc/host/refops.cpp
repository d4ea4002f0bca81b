// Host-side FP64 reference builders (Section 2, Lemmas 2-3, Section 4.1).
#include "refops.hpp"

#include <cmath>
#include <cstdio>

namespace dgpyr {

double jacobi_p(int n, double alpha, double beta, double x) {
  // Three-term recurrence in the standard normalisation.
  if (n == 0) return 1.0;
  double p0 = 1.0;
  double p1 = 0.5 * ((alpha + beta + 2.0) * x + (alpha - beta));
  for (int k = 1; k < n; ++k) {
    const double ab = alpha + beta;
    const double a1 = 2.0 * (k + 1) * (k + ab + 1) * (2 * k + ab);
    const double a2 = (2 * k + ab + 1) * (alpha * alpha - beta * beta);
    const double a3 = (2 * k + ab) * (2 * k + ab + 1) * (2 * k + ab + 2);
    const double a4 = 2.0 * (k + alpha) * (k + beta) * (2 * k + ab + 2);
    const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

double jacobi_dp(int n, double alpha, double beta, double x) {
  if (n == 0) return 0.0;
  return 0.5 * (n + alpha + beta + 1.0) * jacobi_p(n - 1, alpha + 1.0, beta + 1.0, x);
}

void gauss_jacobi(int n, double alpha, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration with deflation by the roots already found, started from
  // Chebyshev-Gauss points (the zero-finding scheme of Karniadakis and
  // Sherwin); weights w_i = 2^(alpha+1) / ((1 - x_i^2) P_n'(x_i)^2) for beta = 0.
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < n; ++k) {
    double r = -std::cos((2.0 * k + 1.0) * pi / (2.0 * n));
    if (k > 0) r = 0.5 * (r + x[k - 1]);
    for (int it = 0; it < 200; ++it) {
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += 1.0 / (r - x[i]);
      const double p = jacobi_p(n, alpha, 0.0, r);
      const double dp = jacobi_dp(n, alpha, 0.0, r);
      const double delta = -p / (dp - s * p);
      r += delta;
      if (std::fabs(delta) < 1e-17) break;
    }
    x[k] = r;
  }
  if (alpha == 0.0) {
    // Gauss-Legendre nodes are symmetric about 0; make them exactly so, so that
    // reflected face parametrisations land on the same floating-point points.
    for (int i = 0; i < n / 2; ++i) {
      const double s = 0.5 * (x[n - 1 - i] - x[i]);
      x[i] = -s;
      x[n - 1 - i] = s;
    }
    if (n % 2) x[n / 2] = 0.0;
  }
  for (int i = 0; i < n; ++i) {
    const double dp = jacobi_dp(n, alpha, 0.0, x[i]);
    w[i] = std::pow(2.0, alpha + 1.0) / ((1.0 - x[i] * x[i]) * dp * dp);
  }
}

double lagrange(const std::vector<double>& nodes, int i, double x) {
  double v = 1.0;
  for (size_t q = 0; q < nodes.size(); ++q)
    if ((int)q != i) v *= (x - nodes[q]) / (nodes[i] - nodes[q]);
  return v;
}

double lagrange_d(const std::vector<double>& nodes, int i, double x) {
  double d = 0.0;
  for (size_t q = 0; q < nodes.size(); ++q) {
    if ((int)q == i) continue;
    double t = 1.0 / (nodes[i] - nodes[q]);
    for (size_t l = 0; l < nodes.size(); ++l)
      if ((int)l != i && l != q) t *= (x - nodes[l]) / (nodes[i] - nodes[l]);
    d += t;
  }
  return d;
}

namespace {

// phi_ijk(a, b, c) = l_i^k(a) l_j^k(b) h^k P_{N-k}^{(2k+3,0)}(c), h = (1-c)/2,
// with derivatives taken directly in (r, s, t): since 2/(1-c) h^k = h^(k-1),
//   d/dr = l'(a) l(b) h^(k-1) P,  d/ds = l(a) l'(b) h^(k-1) P,
//   d/dt = l l g'(c) + (1+a)/2 l' l h^(k-1) P + (1+b)/2 l l' h^(k-1) P,
// with g = h^k P and g' = -k/2 h^(k-1) P + h^k P'.  No division by 1 - c.
struct BasisEval {
  int N;
  std::vector<std::vector<double>> lev;  // GL nodes of each level k
  explicit BasisEval(int N_) : N(N_), lev(N_ + 1) {
    std::vector<double> w;
    for (int k = 0; k <= N; ++k) gauss_jacobi(k + 1, 0.0, lev[k], w);
  }
  void eval(double a, double b, double c, double* v, double* dr, double* ds, double* dt) const {
    const double h = 0.5 * (1.0 - c);
    int n = 0;
    for (int k = 0; k <= N; ++k) {
      const double alpha = 2.0 * k + 3.0;
      const double P = jacobi_p(N - k, alpha, 0.0, c);
      const double dP = jacobi_dp(N - k, alpha, 0.0, c);
      const double hk = std::pow(h, k);
      const double hk1 = k > 0 ? std::pow(h, k - 1) : 0.0;
      const double g = hk * P;
      const double dg = hk * dP - 0.5 * k * hk1 * P;
      for (int j = 0; j <= k; ++j) {
        const double lb = k > 0 ? lagrange(lev[k], j, b) : 1.0;
        const double dlb = k > 0 ? lagrange_d(lev[k], j, b) : 0.0;
        for (int i = 0; i <= k; ++i, ++n) {
          const double la = k > 0 ? lagrange(lev[k], i, a) : 1.0;
          const double dla = k > 0 ? lagrange_d(lev[k], i, a) : 0.0;
          if (v) v[n] = la * lb * g;
          if (dr) {
            const double ea = dla * lb * hk1 * P;
            const double eb = la * dlb * hk1 * P;
            dr[n] = ea;
            ds[n] = eb;
            dt[n] = la * lb * dg + 0.5 * (1.0 + a) * ea + 0.5 * (1.0 + b) * eb;
          }
        }
      }
    }
  }
};

}  // namespace

void eval_basis(int N, double a, double b, double c, double* v) {
  BasisEval be(N);
  be.eval(a, b, c, v, nullptr, nullptr, nullptr);
}

bool build_refops(int N, RefOps& o, char* msg, int msglen) {
  o.N = N;
  o.Np = n_basis(N);
  o.Nq1 = N + 1;
  o.Nc = o.Nq1 * o.Nq1 * o.Nq1;
  o.Nfq = o.Nq1 * o.Nq1;
  o.Nfc = 5 * o.Nfq;
  const int n1 = o.Nq1, Np = o.Np;
  gauss_jacobi(n1, 0.0, o.xg, o.wg);
  gauss_jacobi(n1, 2.0, o.xc, o.wc);
  gauss_jacobi(n1, 1.0, o.xt, o.wt);

  BasisEval be(N);
  o.wv.assign(o.Nc, 0.0);
  o.V.assign((size_t)o.Nc * Np, 0.0);
  o.Dr.assign((size_t)o.Nc * Np, 0.0);
  o.Ds.assign((size_t)o.Nc * Np, 0.0);
  o.Dt.assign((size_t)o.Nc * Np, 0.0);
  for (int r = 0; r < n1; ++r)
    for (int m = 0; m < n1; ++m)
      for (int p = 0; p < n1; ++p) {
        const int q = p + n1 * (m + n1 * r);
        o.wv[q] = o.wg[p] * o.wg[m] * o.wc[r] / 4.0;
        be.eval(o.xg[p], o.xg[m], o.xc[r], &o.V[(size_t)q * Np], &o.Dr[(size_t)q * Np],
                &o.Ds[(size_t)q * Np], &o.Dt[(size_t)q * Np]);
      }

  o.wf.assign(o.Nfc, 0.0);
  o.fa.assign(o.Nfc, 0.0);
  o.fb.assign(o.Nfc, 0.0);
  o.fc.assign(o.Nfc, 0.0);
  o.Vf.assign((size_t)o.Nfc * Np, 0.0);
  for (int f = 0; f < 5; ++f)
    for (int m = 0; m < n1; ++m)
      for (int p = 0; p < n1; ++p) {
        const int q = f * o.Nfq + p + n1 * m;
        double a, b, c, w;
        if (f == 0) {
          a = o.xg[p]; b = o.xg[m]; c = -1.0; w = o.wg[p] * o.wg[m];
        } else {
          const double sg = o.xg[p];
          c = o.xt[m];
          w = o.wg[p] * o.wt[m] / 2.0;
          if (f == 1) { a = -1.0; b = sg; }
          else if (f == 2) { a = 1.0; b = sg; }
          else if (f == 3) { a = sg; b = -1.0; }
          else { a = sg; b = 1.0; }
        }
        o.wf[q] = w;
        o.fa[q] = a; o.fb[q] = b; o.fc[q] = c;
        be.eval(a, b, c, &o.Vf[(size_t)q * Np], nullptr, nullptr, nullptr);
      }

  // One-dimensional factors for the sum-factorised kernels.
  o.sfLa.assign((size_t)n1 * n1 * n1, 0.0);
  o.sfDa.assign((size_t)n1 * n1 * n1, 0.0);
  o.sfLe.assign((size_t)n1 * 2 * n1, 0.0);
  o.sfG.assign((size_t)n1 * n1, 0.0);
  o.sfGt.assign((size_t)n1 * n1, 0.0);
  o.sfGp.assign((size_t)n1 * n1, 0.0);
  o.sfGb.assign((size_t)n1, 0.0);
  o.sfGf.assign((size_t)n1 * n1, 0.0);
  for (int k = 0; k <= N; ++k) {
    const std::vector<double>& lev = be.lev[k];
    for (int i = 0; i <= k; ++i) {
      for (int p = 0; p < n1; ++p) {
        o.sfLa[((size_t)k * n1 + p) * n1 + i] = k > 0 ? lagrange(lev, i, o.xg[p]) : 1.0;
        o.sfDa[((size_t)k * n1 + p) * n1 + i] = k > 0 ? lagrange_d(lev, i, o.xg[p]) : 0.0;
      }
      o.sfLe[((size_t)k * 2 + 0) * n1 + i] = k > 0 ? lagrange(lev, i, -1.0) : 1.0;
      o.sfLe[((size_t)k * 2 + 1) * n1 + i] = k > 0 ? lagrange(lev, i, 1.0) : 1.0;
    }
    const double alpha = 2.0 * k + 3.0;
    for (int r = 0; r < n1; ++r) {
      const double c = o.xc[r], h = 0.5 * (1.0 - c);
      const double P = jacobi_p(N - k, alpha, 0.0, c), dP = jacobi_dp(N - k, alpha, 0.0, c);
      const double hk = std::pow(h, k), hk1 = k > 0 ? std::pow(h, k - 1) : 0.0;
      o.sfG[(size_t)r * n1 + k] = hk * P;
      o.sfGt[(size_t)r * n1 + k] = hk1 * P;
      o.sfGp[(size_t)r * n1 + k] = hk * dP - 0.5 * k * hk1 * P;
      const double ct = o.xt[r], ht = 0.5 * (1.0 - ct);
      o.sfGf[(size_t)r * n1 + k] = std::pow(ht, k) * jacobi_p(N - k, alpha, 0.0, ct);
    }
    o.sfGb[k] = jacobi_p(N - k, alpha, 0.0, -1.0);
  }

  // Diagonal of the reference mass matrix (Lemma 3 with J = 1), by quadrature,
  // checked against w_i^k w_j^k 2/(2k+3) and against diagonality.
  o.wwc.assign(Np, 0.0);
  o.na.assign(Np, 0.0);
  o.nb.assign(Np, 0.0);
  o.bi.assign(Np, 0);
  o.bj.assign(Np, 0);
  o.bk.assign(Np, 0);
  double maxdiag = 0.0, maxoff = 0.0, maxclosed = 0.0;
  std::vector<double> M((size_t)Np * Np, 0.0);
  for (int q = 0; q < o.Nc; ++q)
    for (int i = 0; i < Np; ++i) {
      const double vi = o.wv[q] * o.V[(size_t)q * Np + i];
      for (int j = 0; j < Np; ++j) M[(size_t)i * Np + j] += vi * o.V[(size_t)q * Np + j];
    }
  int n = 0;
  for (int k = 0; k <= N; ++k) {
    std::vector<double> xk, wk;
    gauss_jacobi(k + 1, 0.0, xk, wk);
    for (int j = 0; j <= k; ++j)
      for (int i = 0; i <= k; ++i, ++n) {
        o.bi[n] = i; o.bj[n] = j; o.bk[n] = k;
        o.na[n] = xk[i];
        o.nb[n] = xk[j];
        o.wwc[n] = wk[i] * wk[j] * 2.0 / (2.0 * k + 3.0);
        maxclosed = std::fmax(maxclosed, std::fabs(M[(size_t)n * Np + n] - o.wwc[n]));
        maxdiag = std::fmax(maxdiag, std::fabs(M[(size_t)n * Np + n]));
      }
  }
  for (int i = 0; i < Np; ++i)
    for (int j = 0; j < Np; ++j)
      if (i != j) maxoff = std::fmax(maxoff, std::fabs(M[(size_t)i * Np + j]));
  if (maxoff > 1e-12 * maxdiag || maxclosed > 1e-12 * maxdiag) {
    std::snprintf(msg, msglen, "reference mass check failed (N=%d): offdiag %.3e, closed form %.3e",
                  N, maxoff, maxclosed);
    return false;
  }
  return true;
}

void quad_perm(int N, int o, int* perm) {
  const int n1 = N + 1;
  const bool neg0 = o & 1, neg1 = (o >> 1) & 1, swap = (o >> 2) & 1;
  for (int m = 0; m < n1; ++m)
    for (int p = 0; p < n1; ++p) {
      int X = swap ? m : p;  // index of the coordinate that becomes a'
      int Y = swap ? p : m;
      const int p2 = neg0 ? N - X : X;
      const int m2 = neg1 ? N - Y : Y;
      perm[p + n1 * m] = p2 + n1 * m2;
    }
}

void tri_perm(int N, int o, int* perm) {
  const int n1 = N + 1;
  for (int m = 0; m < n1; ++m)
    for (int p = 0; p < n1; ++p) perm[p + n1 * m] = (o ? N - p : p) + n1 * m;
}

}  // namespace dgpyr
