// Host set-up of the Chebyshev wall-normal direction (see cheb.hpp).
#include "cheb.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace vd {

namespace {

using LD = long double;
const LD kPi = 3.14159265358979323846264338327950288L;

// Legendre P_n and P_{n-1} at x by the three-term recurrence.
void legendre2(int n, LD x, LD* pn, LD* pn1) {
  LD p0 = 1, p1 = x;
  if (n == 0) {
    *pn = 1;
    *pn1 = 0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    LD p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *pn = p1;
  *pn1 = p0;
}

// Symmetric eigen-decomposition by cyclic Jacobi rotations: A = Q diag(w) Q^T.
// Each rotation zeroes a_pq with t = sgn(th) / (|th| + sqrt(th^2 + 1)),
// th = (a_qq - a_pp) / (2 a_pq), c = 1/sqrt(1 + t^2), s = t c.
bool jacobi_eig(int n, std::vector<double>& A, std::vector<double>& Q, std::vector<double>& w) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  double fro = 0;
  for (double v : A) fro += v * v;
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a(p, q) * a(p, q);
    if (std::sqrt(off) <= 1e-15 * fro) {
      w.resize(n);
      for (int i = 0; i < n; ++i) w[i] = a(i, i);
      return true;
    }
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (std::fabs(apq) <= 1e-300) continue;
        const double th = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < n; ++r) {  // columns p, q
          const double arp = a(r, p), arq = a(r, q);
          a(r, p) = c * arp - s * arq;
          a(r, q) = s * arp + c * arq;
        }
        for (int r = 0; r < n; ++r) {  // rows p, q
          const double apr = a(p, r), aqr = a(q, r);
          a(p, r) = c * apr - s * aqr;
          a(q, r) = s * apr + c * aqr;
        }
        a(p, q) = a(q, p) = 0.0;
        for (int r = 0; r < n; ++r) {
          double* qr = &Q[(size_t)r * n];
          const double vp = qr[p], vq = qr[q];
          qr[p] = c * vp - s * vq;
          qr[q] = s * vp + c * vq;
        }
      }
    }
  }
  return false;
}

}  // namespace

bool cheb_setup(int nz, ChebSetup* o) {
  const int M = nz - 1, n = nz;
  o->nz = nz;
  o->zc.resize(n);
  for (int j = 0; j < n; ++j) o->zc[j] = (double)cosl(kPi * j / M);
  // differentiation matrix; node differences from the product formula
  // z_i - z_j = 2 sin(pi (i+j) / 2M) sin(pi (j-i) / 2M), diagonal by the
  // negative-sum rule
  o->D.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    const LD ci = (i == 0 || i == M) ? 2 : 1;
    LD rowsum = 0;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      const LD cj = (j == 0 || j == M) ? 2 : 1;
      const LD dz = 2 * sinl(kPi * (i + j) / (2 * M)) * sinl(kPi * (j - i) / (2 * M));
      const LD v = (ci / cj) * (((i + j) % 2) ? -1 : 1) / dz;
      o->D[(size_t)i * n + j] = (double)v;
      rowsum += v;
    }
    o->D[(size_t)i * n + i] = (double)(-rowsum);
  }
  // Legendre-Gauss-Lobatto nodes: zeros of (1 - x^2) P_M'(x), by Newton on
  // x P_M - P_{M-1} (which vanishes exactly there) from the Chebyshev nodes
  o->zl.resize(n);
  o->wl.resize(n);
  for (int j = 0; j < n; ++j) {
    LD x = cosl(kPi * j / M);
    if (j != 0 && j != M) {
      for (int it = 0; it < 100; ++it) {
        LD pn, pn1;
        legendre2(M, x, &pn, &pn1);
        const LD dx = (x * pn - pn1) / ((M + 1) * pn);
        x -= dx;
        if (fabsl(dx) < 1e-19L) break;
      }
    }
    LD pn, pn1;
    legendre2(M, x, &pn, &pn1);
    o->zl[j] = (double)x;
    o->wl[j] = (double)(2.0L / ((LD)M * (M + 1) * pn * pn));
  }
  // barycentric interpolation CGL -> LGL, weights (-1)^j delta_j
  o->I.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    const LD xi = o->zl[i];
    int hit = -1;
    for (int j = 0; j < n; ++j)
      if ((double)xi == o->zc[j]) hit = j;
    if (hit >= 0) {
      o->I[(size_t)i * n + hit] = 1.0;
      continue;
    }
    LD tot = 0;
    std::vector<LD> t(n);
    for (int j = 0; j < n; ++j) {
      LD bw = (j % 2) ? -1 : 1;
      if (j == 0 || j == M) bw *= 0.5L;
      t[j] = bw / (xi - (LD)o->zc[j]);
      tot += t[j];
    }
    for (int j = 0; j < n; ++j) o->I[(size_t)i * n + j] = (double)(t[j] / tot);
  }
  // G = I D
  o->G.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double v = o->I[(size_t)i * n + k];
      if (v == 0.0) continue;
      for (int j = 0; j < n; ++j) o->G[(size_t)i * n + j] += v * o->D[(size_t)k * n + j];
    }
  // mass and stiffness: Mz = I^T W I, Sz = G^T W G
  std::vector<double> Mz((size_t)n * n, 0.0), Sz((size_t)n * n, 0.0);
  for (int l = 0; l < n; ++l) {
    const double wlv = o->wl[l];
    const double* Il = &o->I[(size_t)l * n];
    const double* Gl = &o->G[(size_t)l * n];
    for (int i = 0; i < n; ++i) {
      const double a = wlv * Il[i], b = wlv * Gl[i];
      for (int j = 0; j < n; ++j) {
        Mz[(size_t)i * n + j] += a * Il[j];
        Sz[(size_t)i * n + j] += b * Gl[j];
      }
    }
  }
  // Cholesky Mz = L L^T
  std::vector<double> L((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = Mz[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(s > 0)) return false;
    const double ljj = std::sqrt(s);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = Mz[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = t / ljj;
    }
  }
  // C = L^-1 Sz L^-T  (X = L^-1 Sz, then C = L^-1 X^T since C is symmetric)
  auto lsolve = [&](std::vector<double>& B) {  // B <- L^-1 B, column by column
    for (int c = 0; c < n; ++c)
      for (int i = 0; i < n; ++i) {
        double t = B[(size_t)i * n + c];
        for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * B[(size_t)k * n + c];
        B[(size_t)i * n + c] = t / L[(size_t)i * n + i];
      }
  };
  std::vector<double> X = Sz;
  lsolve(X);
  std::vector<double> Xt((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Xt[(size_t)i * n + j] = X[(size_t)j * n + i];
  lsolve(Xt);
  for (int i = 0; i < n; ++i)  // symmetrise rounding
    for (int j = i + 1; j < n; ++j) {
      const double v = 0.5 * (Xt[(size_t)i * n + j] + Xt[(size_t)j * n + i]);
      Xt[(size_t)i * n + j] = Xt[(size_t)j * n + i] = v;
    }
  std::vector<double> Q, w;
  if (!jacobi_eig(n, Xt, Q, w)) return false;
  // V = L^-T Q, columns sorted by eigenvalue
  std::vector<double> Vq = Q;
  for (int c = 0; c < n; ++c)
    for (int i = n - 1; i >= 0; --i) {
      double t = Vq[(size_t)i * n + c];
      for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * Vq[(size_t)k * n + c];
      Vq[(size_t)i * n + c] = t / L[(size_t)i * n + i];
    }
  std::vector<int> ord(n);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return w[a] < w[b]; });
  o->V.assign((size_t)n * n, 0.0);
  o->lam.resize(n);
  for (int c = 0; c < n; ++c) {
    o->lam[c] = w[ord[c]];
    for (int i = 0; i < n; ++i) o->V[(size_t)i * n + c] = Vq[(size_t)i * n + ord[c]];
  }
  return true;
}

}  // namespace vd
