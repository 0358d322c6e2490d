// Host point-set construction (see geometry.h).
//
// Readings of passages the paper leaves open (shared with the CPU reference,
// implemented independently here):
//  - equispaced grids start at angle 0 in the global frame and do not rotate with
//    the pair (Sec. 5, remark on combining fine sources);
//  - the ellipse focus a equals R_acc(delta), so the singular segment [0, R_acc]
//    lies between the foci (Sec. 5);
//  - every contact pair gets a_ell n_ell Moebius nodes per disk, the dense end
//    facing the neighbour;
//  - the peanut is made of the two far-side arcs of the disks and the two concave
//    arcs of the unit circle rolled around the pair (Sec. 3.3, Fig. peanut).
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <unordered_map>

namespace mfs {

static const double kPi = 3.14159265358979323846;

void ring_points(Pt c, double rad, int n, std::vector<Pt>& out) {
  out.resize(n);
  for (int j = 0; j < n; ++j) {
    double t = 2.0 * kPi * j / n;
    out[j] = {c.x + rad * std::cos(t), c.y + rad * std::sin(t)};
  }
}

double ring_rule(int n, double eps) { return 1.0 - std::log(1.0 / eps) / n; }

double accumulation_radius(double delta) { return 1.0 + 0.5 * delta - std::sqrt(delta + 0.25 * delta * delta); }

bool find_contacts(int P, const double* c, const double* a, double delta_c, std::vector<int32_t>& pairs, int* bad_i,
                   int* bad_k, double* bad_gap) {
  pairs.clear();
  if (P < 2) return true;
  double amax = 0, xmin = c[0], ymin = c[1];
  for (int i = 0; i < P; ++i) {
    amax = std::max(amax, a[i]);
    xmin = std::min(xmin, c[2 * i]);
    ymin = std::min(ymin, c[2 * i + 1]);
  }
  const double h = 2.0 * amax + std::max(delta_c, 0.0);
  auto key = [](int64_t ix, int64_t iy) { return (ix << 32) ^ (iy & 0xffffffffLL); };
  std::unordered_map<int64_t, std::vector<int>> cells;
  cells.reserve(P * 2);
  std::vector<int64_t> cx(P), cy(P);
  for (int i = 0; i < P; ++i) {
    cx[i] = (int64_t)std::floor((c[2 * i] - xmin) / h);
    cy[i] = (int64_t)std::floor((c[2 * i + 1] - ymin) / h);
    cells[key(cx[i], cy[i])].push_back(i);
  }
  bool ok = true;
  double worst = 1e300;
  for (int i = 0; i < P; ++i) {
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        auto it = cells.find(key(cx[i] + dx, cy[i] + dy));
        if (it == cells.end()) continue;
        for (int k : it->second) {
          if (k <= i) continue;
          double ex = c[2 * k] - c[2 * i], ey = c[2 * k + 1] - c[2 * i + 1];
          double d = std::sqrt(ex * ex + ey * ey);
          double gap = d - a[i] - a[k];
          if (!(gap > 0.0)) {
            if (gap < worst) {
              worst = gap;
              *bad_i = i;
              *bad_k = k;
              *bad_gap = gap;
            }
            ok = false;
          }
          if (gap <= delta_c) {
            pairs.push_back(i);
            pairs.push_back(k);
          }
        }
      }
  }
  // lexicographic order (i, k)
  size_t np = pairs.size() / 2;
  std::vector<std::pair<int32_t, int32_t>> v(np);
  for (size_t p = 0; p < np; ++p) v[p] = {pairs[2 * p], pairs[2 * p + 1]};
  std::sort(v.begin(), v.end());
  for (size_t p = 0; p < np; ++p) {
    pairs[2 * p] = v[p].first;
    pairs[2 * p + 1] = v[p].second;
  }
  return ok;
}

double limit_point(double a1, double a2, double d) {
  const double b = d * d + a1 * a1 - a2 * a2;
  return (b - std::sqrt(b * b - 4.0 * d * d * a1 * a1)) / (2.0 * d);
}

int fine_count(double radius, const FineParams& fp) { return (int)std::lround(fp.n_fp * radius); }

// Ellipse nodes of the disk of radius a1 toward its neighbour (radius a2) at gap delta, in the
// disk's frame with the pair axis along +x: foci 0 and the limit point x1, tip x1 + gamma (a1 - x1).
static void ellipse_nodes(double delta, double a1, double a2, const FineParams& fp,
                          std::vector<std::complex<double>>& z) {
  z.clear();
  const double Rf = a1 * ring_rule(fine_count(a1, fp), fp.eps_ring);
  const double x1 = (a1 == 1.0 && a2 == 1.0) ? accumulation_radius(delta) : limit_point(a1, a2, a1 + a2 + delta);
  if (!(x1 > Rf)) return;
  const double alpha = std::acosh(1.0 + 2.0 * fp.gamma * (a1 - x1) / x1);
  const double ch = std::cosh(alpha), sh = std::sinh(alpha);
  for (int j = 0; j < 2 * fp.n_ell; ++j) {
    double th = (j + 0.5) * kPi / fp.n_ell;
    // cos(th + i alpha) = cos th cosh alpha - i sin th sinh alpha
    std::complex<double> w(0.5 * x1 * (1.0 + std::cos(th) * ch), -0.5 * x1 * std::sin(th) * sh);
    if (std::abs(w) > Rf) z.push_back(w);
  }
}

int ellipse_count(double delta, const FineParams& fp, double a1, double a2) {
  std::vector<std::complex<double>> z;
  ellipse_nodes(delta, a1, a2, fp, z);
  return (int)z.size();
}

void pair_fine_sources(Pt ci, Pt ck, const FineParams& fp, std::vector<Pt>& yi, std::vector<Pt>& yk, double ai,
                       double ak) {
  double ex = ck.x - ci.x, ey = ck.y - ci.y;
  double d = std::sqrt(ex * ex + ey * ey);
  ex /= d;
  ey /= d;
  std::vector<std::complex<double>> z;
  for (int side = 0; side < 2; ++side) {
    const double a0 = side ? ak : ai, a1 = side ? ai : ak, sgn = side ? -1.0 : 1.0;
    const Pt c0 = side ? ck : ci;
    std::vector<Pt>& y = side ? yk : yi;
    const int nf = fine_count(a0, fp);
    ring_points(c0, a0 * ring_rule(nf, fp.eps_ring), nf, y);
    ellipse_nodes(d - ai - ak, a0, a1, fp, z);
    for (auto& w : z) {
      const double rx = ex * w.real() - ey * w.imag();
      const double ry = ey * w.real() + ex * w.imag();
      y.push_back({c0.x + sgn * rx, c0.y + sgn * ry});
    }
  }
}

void pair_fine_nodes(Pt ci, Pt ck, const FineParams& fp, std::vector<Pt>& xi, std::vector<Pt>& xk, double ai,
                     double ak) {
  const double phi = std::atan2(ck.y - ci.y, ck.x - ci.x);
  const int m_ell = fp.a_ell * fp.n_ell;
  ring_points(ci, ai, (int)std::ceil(fp.a_f * fine_count(ai, fp) - 1e-12), xi);
  ring_points(ck, ak, (int)std::ceil(fp.a_f * fine_count(ak, fp) - 1e-12), xk);
  const double r = fp.mobius_r;
  for (int j = 0; j < m_ell; ++j) {
    double t = 2.0 * kPi * j / m_ell;
    std::complex<double> w(std::cos(t), std::sin(t));
    double tt = kPi + std::arg((w + r) / (1.0 + r * w));
    double angi = phi + tt - kPi, angk = phi + tt;
    xi.push_back({ci.x + ai * std::cos(angi), ci.y + ai * std::sin(angi)});
    xk.push_back({ck.x + ak * std::cos(angk), ck.y + ak * std::sin(angk)});
  }
}

void peanut(Pt ci, Pt ck, int m_p, std::vector<Pt>& z, double ai, double ak, double rho) {
  double ex = ck.x - ci.x, ey = ck.y - ci.y;
  const double d = std::sqrt(ex * ex + ey * ey);
  ex /= d;
  ey /= d;
  const double nx = -ey, ny = ex;  // n = e^perp
  // centre of the rolling circle: distance ai + rho from c_i and ak + rho from c_k
  const double s = ((ai + rho) * (ai + rho) - (ak + rho) * (ak + rho) + d * d) / (2.0 * d);
  const double h = std::sqrt((ai + rho) * (ai + rho) - s * s);
  const double psi_i = std::atan2(h, s), psi_k = std::atan2(h, d - s);
  const Pt m{ci.x + s * ex, ci.y + s * ey};
  struct Arc { Pt c; double r, a0, sweep; };
  const Arc arcs[5] = {
      {ci, ai, kPi, kPi - psi_i},                                                 // disk i, far point -> lower tangency
      {{m.x - h * nx, m.y - h * ny}, rho, kPi - psi_i, -(kPi - psi_i - psi_k)},   // lower concave arc
      {ck, ak, kPi + psi_k, 2 * kPi - 2 * psi_k},                                 // disk k, lower -> upper tangency
      {{m.x + h * nx, m.y + h * ny}, rho, -psi_k, -(kPi - psi_i - psi_k)},        // upper concave arc
      {ci, ai, psi_i, kPi - psi_i},                                               // disk i, upper tangency -> far point
  };
  double start[5], total = 0;
  for (int q = 0; q < 5; ++q) {
    start[q] = total;
    total += arcs[q].r * std::fabs(arcs[q].sweep);
  }
  z.resize(m_p);
  for (int p = 0; p < m_p; ++p) {
    double sp = p * total / m_p;
    int q = 4;
    while (q > 0 && sp < start[q]) --q;
    const Arc& A = arcs[q];
    double ang = A.a0 + std::copysign((sp - start[q]) / A.r, A.sweep);
    double ca = std::cos(ang), sa = std::sin(ang);
    z[p] = {A.c.x + A.r * (ca * ex + sa * nx), A.c.y + A.r * (ca * ey + sa * ny)};
  }
}

}  // namespace mfs
