// Host-side set-up mathematics (see host_math.hpp).
#include "host_math.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace dgbgk {

void symmetric_eigen(int n, std::vector<double> A, std::vector<double> &evals,
                     std::vector<double> &V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        (i == j ? diag : off) += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    if (off <= 1e-34 * std::max(diag, 1e-300)) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[(size_t)p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
        // rotation angle zeroing a_pq: cot(2 phi) = (a_qq - a_pp) / (2 a_pq)
        double zeta = (aqq - app) / (2.0 * apq);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- A G (columns p, q)
          double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * akp - s * akq;
          A[(size_t)k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- G^T A (rows p, q)
          double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * apk - s * aqk;
          A[(size_t)q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {  // V <- V G
          double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = c * vkp - s * vkq;
          V[(size_t)k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  // sort ascending, permuting eigenvector columns alongside
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(),
            [&](int a, int b) { return A[(size_t)a * n + a] < A[(size_t)b * n + b]; });
  evals.resize(n);
  std::vector<double> Vs((size_t)n * n);
  for (int c = 0; c < n; ++c) {
    evals[c] = A[(size_t)idx[c] * n + idx[c]];
    for (int r = 0; r < n; ++r) Vs[(size_t)r * n + c] = V[(size_t)r * n + idx[c]];
  }
  V.swap(Vs);
}

// Orthonormal (w.r.t. the standard normal) Hermite polynomials h_k and
// derivatives: h_{k+1} = (x h_k - sqrt(k) h_{k-1}) / sqrt(k+1).
static void hermite_orthonormal(int n, double x, std::vector<double> &h, double &dh_n) {
  h.assign(n + 1, 0.0);
  std::vector<double> d(n + 1, 0.0);
  h[0] = 1.0;
  if (n >= 1) { h[1] = x; d[1] = 1.0; }
  for (int k = 1; k < n; ++k) {
    double a = std::sqrt((double)k), b = std::sqrt((double)(k + 1));
    h[k + 1] = (x * h[k] - a * h[k - 1]) / b;
    d[k + 1] = (h[k] + x * d[k] - a * d[k - 1]) / b;
  }
  dh_n = d[n];
}

bool gauss_hermite_rule(int n, std::vector<double> &x, std::vector<double> &w) {
  if (n < 1 || n > 40) return false;
  // Jacobi matrix of the monic recurrence x He_k = He_{k+1} + k He_{k-1}.
  std::vector<double> J((size_t)n * n, 0.0), ev, V;
  for (int k = 1; k < n; ++k) J[(size_t)(k - 1) * n + k] = J[(size_t)k * n + k - 1] = std::sqrt((double)k);
  symmetric_eigen(n, J, ev, V);
  x.resize(n);
  w.resize(n);
  std::vector<double> h;
  for (int i = 0; i < n; ++i) {
    double xi = ev[i];
    for (int it = 0; it < 4; ++it) {  // Newton polish on h_n
      double dh;
      hermite_orthonormal(n, xi, h, dh);
      if (dh == 0.0) break;
      xi -= h[n] / dh;
    }
    double dh;
    hermite_orthonormal(n, xi, h, dh);
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += h[k] * h[k];  // Christoffel function
    x[i] = xi;
    w[i] = 1.0 / s;
  }
  // exact symmetry about zero
  for (int i = 0; i < n / 2; ++i) {
    double a = 0.5 * (x[n - 1 - i] - x[i]), b = 0.5 * (w[i] + w[n - 1 - i]);
    x[i] = -a; x[n - 1 - i] = a; w[i] = w[n - 1 - i] = b;
  }
  if (n % 2) x[n / 2] = 0.0;
  return true;
}

bool newton_cotes_rule(int m, double vmax, std::vector<double> &x, std::vector<double> &w) {
  if (m < 2 || m > 64 || !(vmax > 0.0)) return false;
  x.resize(m);
  w.resize(m);
  const double h = 2.0 * vmax / (m - 1);
  double sum = 0.0;
  for (int j = 0; j < m; ++j) {
    x[j] = vmax * (double)(2 * j - (m - 1)) / (double)(m - 1);
    const double coef = (j == 0 || j == m - 1) ? 0.5 * h : h;
    w[j] = coef * std::exp(-0.5 * x[j] * x[j]);
    sum += w[j];
  }
  for (int j = 0; j < m; ++j) w[j] /= sum;
  return true;
}

bool gll_points(int p, std::vector<double> &r) {
  if (p < 1 || p > 16) return false;
  r.assign(p + 1, 0.0);
  r[0] = -1.0;
  r[p] = 1.0;
  int n = p - 1;  // interior points: zeros of P_p' = Jacobi(1,1) polynomial of degree p-1
  if (n > 0) {
    std::vector<double> J((size_t)n * n, 0.0), ev, V;
    for (int k = 1; k < n; ++k) {
      double b = std::sqrt((double)k * (k + 2) / ((2.0 * k + 1.0) * (2.0 * k + 3.0)));
      J[(size_t)(k - 1) * n + k] = J[(size_t)k * n + k - 1] = b;
    }
    symmetric_eigen(n, J, ev, V);
    for (int i = 0; i < n; ++i) r[i + 1] = ev[i];
    for (int i = 0; i < (p + 1) / 2; ++i) {
      double a = 0.5 * (r[p - i] - r[i]);
      r[i] = -a;
      r[p - i] = a;
    }
    if (p % 2 == 0) r[p / 2] = 0.0;
  }
  return true;
}

bool gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w) {
  if (n < 1 || n > 64) return false;
  std::vector<double> J((size_t)n * n, 0.0), ev, V;
  for (int k = 1; k < n; ++k) {
    double b = k / std::sqrt(4.0 * k * k - 1.0);
    J[(size_t)(k - 1) * n + k] = J[(size_t)k * n + k - 1] = b;
  }
  symmetric_eigen(n, J, ev, V);
  x = ev;
  w.resize(n);
  for (int i = 0; i < n; ++i) w[i] = 2.0 * V[i] * V[i];  // first component of eigenvector i
  return true;
}

void lagrange_values(const std::vector<double> &r, double t, std::vector<double> &out) {
  const int n = (int)r.size();
  out.assign(n, 0.0);
  for (int i = 0; i < n; ++i)
    if (t == r[i]) { out[i] = 1.0; return; }
  std::vector<double> lam(n);
  double den = 0.0;
  for (int i = 0; i < n; ++i) {
    double prod = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != i) prod *= (r[i] - r[m]);
    lam[i] = 1.0 / prod;
    den += lam[i] / (t - r[i]);
  }
  for (int i = 0; i < n; ++i) out[i] = (lam[i] / (t - r[i])) / den;
}

void differentiation_matrix(const std::vector<double> &r, std::vector<double> &D) {
  const int n = (int)r.size();
  std::vector<double> lam(n);
  for (int i = 0; i < n; ++i) {
    double prod = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != i) prod *= (r[i] - r[m]);
    lam[i] = 1.0 / prod;
  }
  D.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double v = (lam[j] / lam[i]) / (r[i] - r[j]);
      D[(size_t)i * n + j] = v;
      diag -= v;
    }
    D[(size_t)i * n + i] = diag;
  }
}

void mass_matrix(const std::vector<double> &r, std::vector<double> &M) {
  const int n = (int)r.size();
  std::vector<double> xg, wg, l;
  gauss_legendre_rule(n + 1, xg, wg);  // exact for degree 2n+1 >= 2(n-1)
  M.assign((size_t)n * n, 0.0);
  for (size_t g = 0; g < xg.size(); ++g) {
    lagrange_values(r, xg[g], l);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) M[(size_t)i * n + j] += wg[g] * l[i] * l[j];
  }
}

bool spd_solve(int n, const std::vector<double> &M, const std::vector<double> &b,
               std::vector<double> &x) {
  std::vector<double> L((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = M[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[(size_t)i * n + i] = std::sqrt(s);
      } else {
        L[(size_t)i * n + j] = s / L[(size_t)j * n + j];
      }
    }
  std::vector<double> y(n);
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * y[k];
    y[i] = s / L[(size_t)i * n + i];
  }
  x.assign(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * x[k];
    x[i] = s / L[(size_t)i * n + i];
  }
  return true;
}

}  // namespace dgbgk
