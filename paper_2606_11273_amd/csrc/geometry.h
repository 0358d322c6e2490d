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

// Limit point x_1 (distance from the centre of disk 1 toward disk 2) of two circles of radii
// a1, a2 at centre distance d: the common fixed point of the inversions in both circles
// (Sec. 5; unequal radii by the reading taken for unequal radii).  R_acc(d - 2) for unit disks.
double limit_point(double a1, double a2, double d);

// Fine proxy count of a disk: n_fp scaled with the radius (a reading of the paper).
int fine_count(double radius, const FineParams& fp);

// Fine source set of a pair (radii ai, ak): proxies on radius a R_f(N_fp(a)) about each
// centre (global angles) and, when the limit point lies beyond R_f, shielding-ellipse sources
// c_i + e z_j and c_k - e z'_j.  Order: [proxies_i, ellipse_i], [proxies_k, ellipse_k].
void pair_fine_sources(Pt ci, Pt ck, const FineParams& fp, std::vector<Pt>& yi, std::vector<Pt>& yk,
                       double ai = 1.0, double ak = 1.0);

// Number of kept ellipse nodes of a disk of radius a1 facing radius a2 at gap delta.
int ellipse_count(double delta, const FineParams& fp, double a1 = 1.0, double a2 = 1.0);

// Fine collocation nodes: ceil(a_f N_fp(a)) equispaced (global angles) and a_ell n_ell
// Moebius-mapped nodes densest toward the neighbour, per disk, on its boundary.
void pair_fine_nodes(Pt ci, Pt ck, const FineParams& fp, std::vector<Pt>& xi, std::vector<Pt>& xk,
                     double ai = 1.0, double ak = 1.0);

// m_p peanut nodes, uniform in arc length, counter-clockwise from the far point of disk i;
// the concave arcs belong to a circle of radius rho rolled around the pair.
void peanut(Pt ci, Pt ck, int m_p, std::vector<Pt>& z, double ai = 1.0, double ak = 1.0, double rho = 1.0);

}  // namespace mfs
