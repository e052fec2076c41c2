// 1D bases and quadrature rules on the host, FP64.
//
// Benchmarks section: C0 Lagrange bases of degree p on the p+1
// Gauss-Lobatto-Legendre (GLL) nodes; q = p+2 Gauss-Legendre points for
// BP1-BP4, integration on the GLL nodes for BP5-BP6.
//
// Legendre values come from the three-term (Bonnet) recurrence. Gauss points
// are the roots of P_q found by Newton's method from Chebyshev-like initial
// guesses; GLL interior nodes are the roots of (1 - x^2) P_p'(x) =
// p (P_{p-1}(x) - x P_p(x)), whose derivative is -p (p+1) P_p(x) by the
// Legendre equation, again by Newton's method.
#include <cmath>

#include "hx_internal.h"

namespace hx {

namespace {

// P_n(x) and P_{n-1}(x)
void legendre(int n, double x, double &pn, double &pnm1) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    pn = 1.0;
    pnm1 = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  pnm1 = p0;
}

}  // namespace

void gauss_nodes_weights(int q, std::vector<double> &x, std::vector<double> &w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    // root i counted from the left
    double t = -std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn, pm;
      legendre(q, t, pn, pm);
      double dp = q * (t * pn - pm) / (t * t - 1.0);
      double dt = pn / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double pn, pm;
    legendre(q, t, pn, pm);
    double dp = q * (t * pn - pm) / (t * t - 1.0);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  // exact symmetry about 0 (the even-odd kernels rely on it)
  for (int i = 0; i < q / 2; ++i) {
    const double s = 0.5 * (x[q - 1 - i] - x[i]), ws = 0.5 * (w[i] + w[q - 1 - i]);
    x[i] = -s;
    x[q - 1 - i] = s;
    w[i] = w[q - 1 - i] = ws;
  }
  if (q % 2 == 1) x[q / 2] = 0.0;
}

void gll_nodes_weights(int p, std::vector<double> &x, std::vector<double> &w) {
  const int n = p + 1;
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 1; i < p; ++i) {
    double t = -std::cos(M_PI * i / p);
    for (int it = 0; it < 100; ++it) {
      double pn, pm;
      legendre(p, t, pn, pm);
      // Newton on f = P_{p-1} - t P_p (proportional to (1-t^2) P_p'), f' = -(p+1) P_p
      double dt = (pm - t * pn) / ((p + 1.0) * pn);
      t += dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = t;
  }
  if (p % 2 == 0) x[p / 2] = 0.0;
  for (int i = 1; i < n / 2; ++i) {
    const double s = 0.5 * (x[n - 1 - i] - x[i]);
    x[i] = -s;
    x[n - 1 - i] = s;
  }
  for (int i = 0; i < n; ++i) {
    double pn, pm;
    legendre(p, x[i], pn, pm);
    w[i] = 2.0 / (p * (p + 1.0) * pn * pn);
  }
}

void lagrange_tables(const std::vector<double> &nodes, const std::vector<double> &pts,
                     std::vector<double> &val, std::vector<double> &der) {
  const int P = (int)nodes.size(), Q = (int)pts.size();
  val.assign((size_t)Q * P, 0.0);
  der.assign((size_t)Q * P, 0.0);
  for (int a = 0; a < Q; ++a) {
    const double t = pts[a];
    for (int i = 0; i < P; ++i) {
      double v = 1.0, d = 0.0;
      for (int m = 0; m < P; ++m) {
        if (m == i) continue;
        const double f = (t - nodes[m]) / (nodes[i] - nodes[m]);
        // product rule: d(v * f) = d * f + v * f'
        d = d * f + v / (nodes[i] - nodes[m]);
        v *= f;
      }
      val[(size_t)a * P + i] = v;
      der[(size_t)a * P + i] = d;
    }
  }
}

bool make_basis(int p, int q, int rule, Basis1D &out, std::string &err) {
  if (p < 1 || p > kMaxP - 1) {
    err = "polynomial degree p must be in 1..8";
    return false;
  }
  if (rule == HX_GLL) {
    if (q != p + 1) {
      err = "HX_GLL supports only the collocated rule q = p+1";
      return false;
    }
  } else if (rule == HX_GAUSS) {
    if (q != p + 1 && q != p + 2) {
      err = "HX_GAUSS supports q = p+1 or q = p+2";
      return false;
    }
  } else {
    err = "qrule must be HX_GAUSS or HX_GLL";
    return false;
  }
  out.p = p;
  out.P = p + 1;
  out.q = q;
  out.rule = rule;
  std::vector<double> wn;
  gll_nodes_weights(p, out.nodes, wn);
  if (rule == HX_GLL) {
    out.qpts = out.nodes;
    out.qw = wn;
  } else {
    gauss_nodes_weights(q, out.qpts, out.qw);
  }
  lagrange_tables(out.nodes, out.qpts, out.interp, out.grad);
  std::vector<double> cv;
  lagrange_tables(out.qpts, out.qpts, cv, out.colloc);
  return true;
}

}  // namespace hx
