// Host tabulation of the 1D reference tables (Section II-B, eq. tensorDense).
//
// Gauss-Lobatto nodes: end points plus the roots of L_p', found by Newton iteration
// using the Legendre equation (1-x^2) L'' = 2x L' - p(p+1) L for the second
// derivative.  Gauss-Legendre points: roots of L_Q by Newton iteration, weights
// 2 / ((1-x^2) L_Q'(x)^2) (Golub & Welsch 1969 give the same rule).  Lagrange values and
// derivatives come from the product formula.  The collocated derivative is
// B_xi B_I^+ with the least-squares pseudo-inverse (B_I^T B_I)^{-1} B_I^T.
#include <cmath>
#include <vector>

#include "common.h"

namespace hpmg {
namespace {

// Legendre L_n(x) and its derivative by the three-term recurrence.
void legendre(int n, double x, double *L, double *dL) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *L = 1.0;
    *dL = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *L = p1;
  // L_n' = n (x L_n - L_{n-1}) / (x^2 - 1); valid away from the end points, which
  // the Newton iterations below never reach.
  *dL = n * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_rule(int Q, double *x, double *w) {
  for (int i = 0; i < Q; ++i) {
    double z = -std::cos(M_PI * (i + 0.75) / (Q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double L, dL;
      legendre(Q, z, &L, &dL);
      double dz = L / dL;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double L, dL;
    legendre(Q, z, &L, &dL);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dL * dL);
  }
}

void lobatto_nodes(int P, double *x) {
  const int p = P - 1;
  x[0] = -1.0;
  x[p] = 1.0;
  for (int j = 1; j < p; ++j) {
    double z = -std::cos(M_PI * j / p);
    for (int it = 0; it < 100; ++it) {
      double L, dL;
      legendre(p, z, &L, &dL);
      double d2L = (2.0 * z * dL - p * (p + 1.0) * L) / (1.0 - z * z);
      double dz = dL / d2L;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[j] = z;
  }
}

// B[q][i] = l_i(x_q), G[q][i] = l_i'(x_q) for Lagrange polynomials on `nodes`.
void lagrange_tables(int P, const double *nodes, int Q, const double *x, double *B, double *G) {
  for (int q = 0; q < Q; ++q) {
    for (int i = 0; i < P; ++i) {
      double v = 1.0;
      for (int j = 0; j < P; ++j)
        if (j != i) v *= (x[q] - nodes[j]) / (nodes[i] - nodes[j]);
      double d = 0.0;
      for (int k = 0; k < P; ++k) {
        if (k == i) continue;
        double t = 1.0 / (nodes[i] - nodes[k]);
        for (int j = 0; j < P; ++j)
          if (j != i && j != k) t *= (x[q] - nodes[j]) / (nodes[i] - nodes[j]);
        d += t;
      }
      if (B) B[q * P + i] = v;
      if (G) G[q * P + i] = d;
    }
  }
}

// Solves A X = R for X (n x n, n x m) by Gaussian elimination with partial pivoting.
bool solve_dense(int n, int m, std::vector<double> A, std::vector<double> &R) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (std::fabs(A[piv * n + c]) < 1e-300) return false;
    if (piv != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[piv * n + k]);
      for (int k = 0; k < m; ++k) std::swap(R[c * m + k], R[piv * m + k]);
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c] / A[c * n + c];
      if (f == 0.0) continue;
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      for (int k = 0; k < m; ++k) R[r * m + k] -= f * R[c * m + k];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int k = 0; k < m; ++k) R[r * m + k] /= A[r * n + r];
  return true;
}

}  // namespace

int tabulate(int P, int Q, double *B, double *G, double *D, double *xq, double *wq, double *gll) {
  if (P < 2 || Q < P || Q > 16) return fail(HPMG_ERR_ARG, "tabulate: need 2 <= P <= Q <= 16");
  std::vector<double> nodes(P), x(Q), w(Q), b(Q * P), g(Q * P);
  lobatto_nodes(P, nodes.data());
  gauss_rule(Q, x.data(), w.data());
  lagrange_tables(P, nodes.data(), Q, x.data(), b.data(), g.data());
  if (B) for (int k = 0; k < Q * P; ++k) B[k] = b[k];
  if (G) for (int k = 0; k < Q * P; ++k) G[k] = g[k];
  if (xq) for (int k = 0; k < Q; ++k) xq[k] = x[k];
  if (wq) for (int k = 0; k < Q; ++k) wq[k] = w[k];
  if (gll) for (int k = 0; k < P; ++k) gll[k] = nodes[k];
  if (D) {
    // D = G (B^T B)^{-1} B^T : solve (B^T B) Y = B^T for Y = B^+ (P x Q).
    std::vector<double> BtB(P * P, 0.0), Bt(P * Q);
    for (int i = 0; i < P; ++i)
      for (int j = 0; j < P; ++j)
        for (int q = 0; q < Q; ++q) BtB[i * P + j] += b[q * P + i] * b[q * P + j];
    for (int i = 0; i < P; ++i)
      for (int q = 0; q < Q; ++q) Bt[i * Q + q] = b[q * P + i];
    if (!solve_dense(P, Q, BtB, Bt)) return fail(HPMG_ERR_ARG, "tabulate: singular B^T B");
    for (int q = 0; q < Q; ++q)
      for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int i = 0; i < P; ++i) s += g[q * P + i] * Bt[i * Q + r];
        D[q * Q + r] = s;
      }
  }
  return HPMG_OK;
}

int ctof_table(int Pf, int Pc, double *M) {
  if (Pc < 2 || Pf < Pc || Pf > 16) return fail(HPMG_ERR_ARG, "ctof: need 2 <= Pc <= Pf <= 16");
  std::vector<double> nf(Pf), nc(Pc);
  lobatto_nodes(Pf, nf.data());
  lobatto_nodes(Pc, nc.data());
  lagrange_tables(Pc, nc.data(), Pf, nf.data(), M, nullptr);
  return HPMG_OK;
}

}  // namespace hpmg

extern "C" int hpmg_basis_tabulate(int P, int Q, double *interp, double *grad, double *colloc,
                                   double *qref, double *qweight, double *gll) {
  return hpmg::tabulate(P, Q, interp, grad, colloc, qref, qweight, gll);
}

extern "C" int hpmg_basis_ctof(int Pf, int Pc, double *ctof) {
  if (!ctof) return hpmg::fail(HPMG_ERR_ARG, "ctof: null output");
  return hpmg::ctof_table(Pf, Pc, ctof);
}
