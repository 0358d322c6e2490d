// Host-side point sets of the method: coarse rings, contact search, fine pair
// discretisation (Sec. 5) and peanut nodes (Sec. 3.3).  All FP64, absolute
// coordinates unless stated.
#pragma once

#include <cstdint>
#include <vector>

namespace mfs {

struct Pt { double x, y; };

// n points on the circle |p - c| = rad, first at angle 0.
void ring_points(Pt c, double rad, int n, std::vector<Pt>& out);

// 1 - ln(1/eps)/n (Sec. 6 ring rule).
double ring_rule(int n, double eps);

// Image accumulation radius R_acc(delta) = 1 + delta/2 - sqrt(delta + delta^2/4) (Sec. 5).
double accumulation_radius(double delta);

// Close pairs i < k with |c_i - c_k| <= a_i + a_k + delta_c, lexicographic order.
// Returns false (and the offending pair) if some gap is <= 0.
bool find_contacts(int P, const double* centers, const double* radii, double delta_c,
                   std::vector<int32_t>& pairs, int* bad_i, int* bad_k, double* bad_gap);

struct FineParams {
  int n_fp, n_ell, m_p, a_ell;
  double gamma, a_f, mobius_r, eps_ring;
};

// Fine source set of a unit-disk pair: proxies on radius R_f about each centre
// (global angles) and, when R_acc(delta) > R_f, shielding-ellipse sources
// c_i + e z_j and c_k - e z_j with |z_j| > R_f.  Order: [proxies_i, ellipse_i],
// [proxies_k, ellipse_k]; both lists have the same length.
void pair_fine_sources(Pt ci, Pt ck, const FineParams& fp, std::vector<Pt>& yi, std::vector<Pt>& yk);

// Number of kept ellipse nodes at gap delta (0 when R_acc(delta) <= R_f).
int ellipse_count(double delta, const FineParams& fp);

// Fine collocation nodes: ceil(a_f n_fp) equispaced (global angles) and
// a_ell n_ell Moebius-mapped nodes densest toward the neighbour, per disk.
void pair_fine_nodes(Pt ci, Pt ck, const FineParams& fp, std::vector<Pt>& xi, std::vector<Pt>& xk);

// m_p peanut nodes, uniform in arc length, counter-clockwise from the far point of disk i.
void peanut(Pt ci, Pt ck, int m_p, std::vector<Pt>& z);

}  // namespace mfs
