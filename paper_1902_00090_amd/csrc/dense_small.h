// Host-side dense complex linear algebra for the small eigenproblem of
// subspace recycling: Householder least squares, Hessenberg reduction, the
// shifted QR algorithm to complex Schur form, and reordering of the Schur
// form (textbook algorithms: Golub and Van Loan, Matrix Computations, the
// chapters on orthogonalization and on the unsymmetric eigenvalue problem).
// Matrices are row-major std::complex<double> arrays.
#pragma once

#include <cmath>
#include <complex>
#include <vector>

namespace dd_small {

using cd = std::complex<double>;

inline double abs1(cd z) { return std::fabs(z.real()) + std::fabs(z.imag()); }

// Rotation G = [[c, s], [-conj(s), c]] (c real) with G [x; y] = [r; 0].
inline void givens(cd x, cd y, double& c, cd& s) {
  const double ax = std::abs(x), ay = std::abs(y);
  if (ay == 0.0) { c = 1.0; s = 0.0; return; }
  if (ax == 0.0) { c = 0.0; s = 1.0; return; }
  const double nrm = std::hypot(ax, ay);
  c = ax / nrm;
  s = (x / ax) * std::conj(y) / nrm;
}

// Rows a, b of the n-column matrix H (columns j0..j1-1) <- G [row a; row b].
inline void rot_rows(cd* H, int n, int a, int b, int j0, int j1, double c, cd s) {
  for (int j = j0; j < j1; ++j) {
    const cd h1 = H[(size_t)a * n + j], h2 = H[(size_t)b * n + j];
    H[(size_t)a * n + j] = c * h1 + s * h2;
    H[(size_t)b * n + j] = -std::conj(s) * h1 + c * h2;
  }
}

// Columns a, b of the n-column matrix H (rows i0..i1-1) <- [col a, col b] G^H.
inline void rot_cols(cd* H, int n, int a, int b, int i0, int i1, double c, cd s) {
  for (int i = i0; i < i1; ++i) {
    const cd h1 = H[(size_t)i * n + a], h2 = H[(size_t)i * n + b];
    H[(size_t)i * n + a] = c * h1 + std::conj(s) * h2;
    H[(size_t)i * n + b] = -s * h1 + c * h2;
  }
}

// Least squares X = G^+ M for G (m x n, full column rank, m >= n) and
// M (m x p): Householder QR of G, Q^H applied to M, back substitution.
// Returns false when R has a zero diagonal entry.
inline bool lsq(int m, int n, int p, std::vector<cd> G, std::vector<cd> M, std::vector<cd>& X) {
  std::vector<cd> v(m);
  for (int c = 0; c < n; ++c) {
    double nx = 0.0;
    for (int i = c; i < m; ++i) nx += std::norm(G[(size_t)i * n + c]);
    nx = std::sqrt(nx);
    if (nx == 0.0) return false;
    const cd x0 = G[(size_t)c * n + c];
    const cd ph = (std::abs(x0) > 0.0) ? x0 / std::abs(x0) : cd(1.0, 0.0);
    // v = x + ph ||x|| e_1 ; H = I - 2 v v^H / (v^H v) maps x to -ph ||x|| e_1
    for (int i = c; i < m; ++i) v[i] = G[(size_t)i * n + c];
    v[c] += ph * nx;
    double vv = 0.0;
    for (int i = c; i < m; ++i) vv += std::norm(v[i]);
    auto apply = [&](std::vector<cd>& A, int ncol, int j0) {
      for (int j = j0; j < ncol; ++j) {
        cd d = 0.0;
        for (int i = c; i < m; ++i) d += std::conj(v[i]) * A[(size_t)i * ncol + j];
        d *= 2.0 / vv;
        for (int i = c; i < m; ++i) A[(size_t)i * ncol + j] -= d * v[i];
      }
    };
    apply(G, n, c);
    apply(M, p, 0);
  }
  X.assign((size_t)n * p, cd(0.0, 0.0));
  for (int j = 0; j < p; ++j)
    for (int i = n - 1; i >= 0; --i) {
      cd s = M[(size_t)i * p + j];
      for (int l = i + 1; l < n; ++l) s -= G[(size_t)i * n + l] * X[(size_t)l * p + j];
      const cd r = G[(size_t)i * n + i];
      if (r == cd(0.0, 0.0)) return false;
      X[(size_t)i * p + j] = s / r;
    }
  return true;
}

// A (n x n) <- Z^H A Z upper Hessenberg by Householder reflections; Z is
// set to the accumulated unitary factor.
inline void hessenberg(int n, std::vector<cd>& A, std::vector<cd>& Z) {
  Z.assign((size_t)n * n, cd(0.0, 0.0));
  for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
  std::vector<cd> v(n);
  for (int c = 0; c + 2 < n; ++c) {
    double nx = 0.0;
    for (int i = c + 1; i < n; ++i) nx += std::norm(A[(size_t)i * n + c]);
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const cd x0 = A[(size_t)(c + 1) * n + c];
    const cd ph = (std::abs(x0) > 0.0) ? x0 / std::abs(x0) : cd(1.0, 0.0);
    for (int i = c + 1; i < n; ++i) v[i] = A[(size_t)i * n + c];
    v[c + 1] += ph * nx;
    double vv = 0.0;
    for (int i = c + 1; i < n; ++i) vv += std::norm(v[i]);
    const double f = 2.0 / vv;
    // A <- P A
    for (int j = 0; j < n; ++j) {
      cd d = 0.0;
      for (int i = c + 1; i < n; ++i) d += std::conj(v[i]) * A[(size_t)i * n + j];
      d *= f;
      for (int i = c + 1; i < n; ++i) A[(size_t)i * n + j] -= d * v[i];
    }
    // A <- A P, Z <- Z P
    for (int i = 0; i < n; ++i) {
      cd d = 0.0, e = 0.0;
      for (int l = c + 1; l < n; ++l) {
        d += A[(size_t)i * n + l] * v[l];
        e += Z[(size_t)i * n + l] * v[l];
      }
      d *= f;
      e *= f;
      for (int l = c + 1; l < n; ++l) {
        A[(size_t)i * n + l] -= d * std::conj(v[l]);
        Z[(size_t)i * n + l] -= e * std::conj(v[l]);
      }
    }
    for (int i = c + 2; i < n; ++i) A[(size_t)i * n + c] = 0.0;
  }
}

// Upper Hessenberg H (n x n) <- its complex Schur form T = Z^H H Z by the
// implicit single-shift QR algorithm with Wilkinson shifts (an exceptional
// shift every tenth iteration without deflation); Z accumulates the
// rotations (Z <- Z G^H).  Returns false without convergence.
inline bool schur(int n, std::vector<cd>& H, std::vector<cd>& Z) {
  const double ulp = 2.220446049250313e-16;
  int hi = n - 1, it = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    for (; l > 0; --l) {
      double s = abs1(H[(size_t)(l - 1) * n + l - 1]) + abs1(H[(size_t)l * n + l]);
      if (s == 0.0) {
        for (int i = 0; i <= hi; ++i) s += abs1(H[(size_t)i * n + i]);
        if (s == 0.0) s = 1.0;
      }
      if (abs1(H[(size_t)l * n + l - 1]) <= ulp * s) {
        H[(size_t)l * n + l - 1] = 0.0;
        break;
      }
    }
    if (l == hi) { --hi; it = 0; continue; }
    if (++total > 60 * n) return false;
    ++it;
    cd mu;
    if (it % 10 == 0) {
      mu = H[(size_t)hi * n + hi] + 0.75 * std::abs(H[(size_t)hi * n + hi - 1]);
    } else {
      const cd a = H[(size_t)(hi - 1) * n + hi - 1], b = H[(size_t)(hi - 1) * n + hi];
      const cd c = H[(size_t)hi * n + hi - 1], d = H[(size_t)hi * n + hi];
      const cd half = 0.5 * (a - d);
      const cd disc = std::sqrt(half * half + b * c);
      const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
    }
    cd x = H[(size_t)l * n + l] - mu, y = H[(size_t)(l + 1) * n + l];
    for (int k = l; k < hi; ++k) {
      double c;
      cd s;
      givens(x, y, c, s);
      rot_rows(H.data(), n, k, k + 1, (k > l) ? k - 1 : l, n, c, s);
      rot_cols(H.data(), n, k, k + 1, 0, std::min(k + 3, hi + 1), c, s);
      rot_cols(Z.data(), n, k, k + 1, 0, n, c, s);
      if (k > l) H[(size_t)(k + 1) * n + k - 1] = 0.0;
      if (k + 1 < hi) {
        x = H[(size_t)(k + 1) * n + k];
        y = H[(size_t)(k + 2) * n + k];
      }
    }
  }
  for (int i = 1; i < n; ++i)
    for (int j = 0; j < i; ++j) H[(size_t)i * n + j] = 0.0;
  return true;
}

// Swap the adjacent diagonal entries k, k+1 of the upper triangular T
// (n x n) by one rotation; Z <- Z G^H keeps A = Z T Z^H.
inline void swap_diag(int n, std::vector<cd>& T, std::vector<cd>& Z, int k) {
  const cd t11 = T[(size_t)k * n + k], t22 = T[(size_t)(k + 1) * n + k + 1];
  double c;
  cd s;
  givens(T[(size_t)k * n + k + 1], t22 - t11, c, s);
  rot_rows(T.data(), n, k, k + 1, k, n, c, s);
  rot_cols(T.data(), n, k, k + 1, 0, k + 2, c, s);
  rot_cols(Z.data(), n, k, k + 1, 0, n, c, s);
  T[(size_t)k * n + k] = t22;
  T[(size_t)(k + 1) * n + k + 1] = t11;
  T[(size_t)(k + 1) * n + k] = 0.0;
}

// Moves the kr diagonal entries of largest magnitude of the Schur form to
// the leading positions, largest first (ties keep their order).
inline void select_largest(int n, std::vector<cd>& T, std::vector<cd>& Z, int kr) {
  for (int pos = 0; pos < kr; ++pos) {
    int q = pos;
    double best = std::abs(T[(size_t)pos * n + pos]);
    for (int i = pos + 1; i < n; ++i) {
      const double a = std::abs(T[(size_t)i * n + i]);
      if (a > best) { best = a; q = i; }
    }
    for (int i = q - 1; i >= pos; --i) swap_diag(n, T, Z, i);
  }
}

// The small problem of harmonic Ritz recycling.  G (nw x ns) and M = W^H S
// (nw x ns) describe A S = W G with W orthonormal; the harmonic Ritz pairs
// (theta, S u) solve G^H G u = theta G^H M u, i.e. T u = u / theta with
// T = G^+ M.  Returns in Z (ns x kr) an orthonormal basis of the invariant
// subspace of T for its kr eigenvalues of largest magnitude (the harmonic
// Ritz values of smallest magnitude), each column scaled so that
// ||G z|| = 1, and in theta their harmonic Ritz values (infinite for a
// zero eigenvalue).  Returns false if G is rank deficient or QR fails.
inline bool harmonic_ritz(int ns, int nw, const std::vector<cd>& G, const std::vector<cd>& M,
                          int kr, std::vector<cd>& Z, std::vector<cd>& theta) {
  std::vector<cd> T;
  if (!lsq(nw, ns, ns, G, M, T)) return false;
  std::vector<cd> U;
  hessenberg(ns, T, U);
  if (!schur(ns, T, U)) return false;
  select_largest(ns, T, U, kr);
  Z.assign((size_t)ns * kr, cd(0.0, 0.0));
  theta.assign(kr, cd(0.0, 0.0));
  for (int o = 0; o < kr; ++o) {
    const cd mu = T[(size_t)o * ns + o];
    theta[o] = (mu == cd(0.0, 0.0)) ? cd(INFINITY, 0.0) : 1.0 / mu;
    double g2 = 0.0;
    for (int i = 0; i < nw; ++i) {
      cd s = 0.0;
      for (int l = 0; l < ns; ++l) s += G[(size_t)i * ns + l] * U[(size_t)l * ns + o];
      g2 += std::norm(s);
    }
    const double f = (g2 > 0.0) ? 1.0 / std::sqrt(g2) : 1.0;
    for (int l = 0; l < ns; ++l) Z[(size_t)l * kr + o] = U[(size_t)l * ns + o] * f;
  }
  return true;
}

}  // namespace dd_small
