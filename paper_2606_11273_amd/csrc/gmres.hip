// mfs_gmres_solve: RHS -> GMRES on the Alg. 3 operator -> post-processing.
//
// GMRES is unrestarted, x0 = 0 unless given, with the Krylov basis resident in
// device memory.  Orthogonalisation is classical Gram-Schmidt applied twice
// (CGS2): two passes of h = V^T w, w -= V h per iteration, all FP64, with the dot
// products reduced in a fixed order.  The (k+1) x k Hessenberg least-squares
// problem is updated by Givens rotations on the host (a few doubles per
// iteration cross the bus).
//
// MFS_MIXED: FP64 iterative refinement around a GMRES whose operator applications
// switch from FP64 to the mixed operator (FP32 all-pairs sum, FP64 accumulation)
// once the Arnoldi residual estimate has dropped below tol_inner / delta, delta an
// upper estimate of the mixed operator's relative error: a per-problem floor, raised
// to the error measured on the basis vector at the first switch (one extra mixed
// application per solve), and raised again by f when a refinement step misses its
// target by a factor f > 10.  A mixed phase whose residual estimate stalls (less than
// 10% gained over 100 iterations) continues with the FP64 operator.  This is the relaxation
// of inexact Krylov methods (Simoncini & Szyld 2003; Bouras & Fraysse 2005): the
// operator error tolerated at step k grows like tol / |r_k|, so only the first
// iterations need FP64, and one Krylov space serves the whole solve instead of
// being rebuilt at every refinement step.  Each refinement step computes the
// true residual r = b - T_64 x in FP64 and stops when |r| <= tol |b|.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

using namespace mfs;

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) { return std::chrono::duration<double, std::milli>(clk::now() - t0).count(); }

Status ensure_krylov(mfs_ctx* c, int cap, int R) {
  Krylov& k = c->kr;
  const int64_t n = 2 * c->Nt;
  if (k.V && k.cap >= cap && k.rcap >= R && k.n == n) return Status{};
  for (double** p : {&k.V, &k.part, &k.hdev, &k.w, &k.x, &k.r, &k.b, &k.d, &k.tmp})
    if (*p) dev_free(c, *p);
  if (k.hhost) (void)hipHostFree(k.hhost);
  k.V = k.part = k.hdev = k.hhost = k.w = k.x = k.r = k.b = k.d = k.tmp = nullptr;
  k.cap = k.rcap = 0;
  for (double** p : {&k.w, &k.x, &k.r, &k.b, &k.d, &k.tmp}) MFS_HIP(dev_malloc(c, (void**)p, sizeof(double) * n * R));
  if (dev_malloc(c, (void**)&k.V, sizeof(double) * n * R * (cap + 1)) != hipSuccess) {
    (void)hipGetLastError();
    k.V = nullptr;
    return Status{MFS_ERR_OOM, "Krylov basis of " + std::to_string(cap + 1) + " x " + std::to_string(R) +
                                   " vectors does not fit"};
  }
  const int nblk = mdot_blocks(n);
  MFS_HIP(dev_malloc(c, (void**)&k.part, sizeof(double) * nblk * (cap + 2)));
  MFS_HIP(dev_malloc(c, (void**)&k.hdev, sizeof(double) * 3 * (cap + 2) * R));
  MFS_HIP(hipHostMalloc((void**)&k.hhost, sizeof(double) * 3 * (cap + 2) * R, hipHostMallocDefault));
  k.cap = cap;
  k.rcap = R;
  k.n = n;
  return Status{};
}

double dnorm(mfs_ctx* c, const double* v, Status* st) {
  Krylov& k = c->kr;
  const int64_t n = k.n;
  const int nblk = mdot_blocks(n);
  launch_mdot(c->stream, n, 1, v, n, v, k.part, k.hdev, nblk);
  double h = 0;
  if (hipMemcpyAsync(&k.hhost[0], k.hdev, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    *st = Status{MFS_ERR_DEVICE, "norm"};
    return 0;
  }
  h = k.hhost[0];
  return std::sqrt(h);
}

// Solve T d = r (starting from d = 0) to |r - T d| <= tol |r| (Givens estimate); d returned in k.d.
// Operator applications use the mixed kernel sum once the estimate is below switch_below.
// |a - b| / |b| for device vectors of length n; a is overwritten with a - b.
double rel_diff(mfs_ctx* c, int64_t n, double* a, const double* b, Status* st) {
  launch_axpby(c->stream, n, -1.0, b, 1.0, a);
  const double dn = dnorm(c, a, st);
  if (st->code) return 0.0;
  const double bn = dnorm(c, b, st);
  return bn > 0.0 ? dn / bn : 0.0;
}

// Switch point of the relaxed inner GMRES: the mixed operator is used once the residual
// estimate is below tol / max(delta, op_err), op_err the measured relative error of the
// mixed operator (negative while unknown).
double switch_point(bool mixed, double tol, double delta, double op_err) {
  return mixed ? std::min(1.0, tol / std::max(delta, op_err)) : 0.0;
}

// Stall test of the mixed phase: every kStallWindow / 2 mixed iterations, once there have
// been kStallWindow of them, the residual estimate is compared with its value
// kStallWindow iterations back; below a kStallDrop reduction the FP32 products have
// stopped the Krylov process from progressing (the noise of the FP32 sum, not a
// spectral plateau, which still gains ~40% per 100 iterations at P = 10^4), and the
// rest of the inner solve applies the FP64 operator, keeping the Krylov space.
constexpr int kStallWindow = 100;
constexpr double kStallDrop = 0.9;

bool stalled(const std::vector<double>& est, int first32, int j) {
  const int done = j + 1;
  return first32 >= 0 && done - first32 > kStallWindow && done % (kStallWindow / 2) == 0 &&
         est[j] > kStallDrop * est[j - kStallWindow];   // j - kStallWindow >= first32 >= 0
}

Status gmres_core(mfs_ctx* c, int prob, bool mixed, double delta, double& op_err, const double* r, double tol,
                  int maxit, int* iters, std::vector<double>& hist) {
  Krylov& k = c->kr;
  const int64_t n = k.n;
  const int nblk = mdot_blocks(n);
  Status st;
  double switch_below = switch_point(mixed, tol, delta, op_err);
  const double beta = dnorm(c, r, &st);
  if (st.code) return st;
  MFS_HIP(hipMemsetAsync(k.d, 0, sizeof(double) * n, c->stream));
  *iters = 0;
  if (!std::isfinite(beta)) return Status{MFS_ERR_NUMERIC, "non-finite residual"};
  if (beta == 0.0) return Status{};
  launch_scale_copy(c->stream, n, 1.0 / beta, r, k.V);
  std::vector<double> H((size_t)(maxit + 1) * maxit, 0.0), cs(maxit), sn(maxit), g(maxit + 1, 0.0);
  std::vector<double> est(maxit, 1.0);
  int first32 = -1;
  bool force64 = false;
  auto Hc = [&](int row, int col) -> double& { return H[(size_t)col * (maxit + 1) + row]; };
  g[0] = beta;
  int kdone = 0;
  const int cap = k.cap;
  const bool prof = std::getenv("MFS_PROFILE") != nullptr;
  auto t_start = clk::now();
  double rel_est = 1.0;
  for (int j = 0; j < maxit; ++j) {
    double* vj = k.V + (int64_t)j * n;
    bool use32 = mixed && !force64 && rel_est <= switch_below;
    if (use32 && op_err < 0.0) {
      // first switch: measure the mixed operator on this basis vector against the FP64
      // one (which this iteration keeps), then move the switch point if it is worse
      if ((st = apply_T(c, prob, false, vj, k.w)).code) return st;
      if ((st = apply_T(c, prob, true, vj, k.tmp)).code) return st;
      op_err = rel_diff(c, n, k.tmp, k.w, &st);
      if (st.code) return st;
      switch_below = switch_point(mixed, tol, delta, op_err);
      if (prof)
        std::fprintf(stderr, "[mfs gmres] mixed operator relative error %.2e: switch below %.2e\n", op_err,
                     switch_below);
      use32 = false;
    } else if ((st = apply_T(c, prob, use32, vj, k.w)).code) {
      return st;
    }
    if (use32 && first32 < 0) first32 = j;
    // CGS2
    launch_mdot(c->stream, n, j + 1, k.V, n, k.w, k.part, k.hdev, nblk);
    launch_maxpy(c->stream, n, j + 1, k.V, n, k.hdev, k.w);
    launch_mdot(c->stream, n, j + 1, k.V, n, k.w, k.part, k.hdev + (cap + 2), nblk);
    launch_maxpy(c->stream, n, j + 1, k.V, n, k.hdev + (cap + 2), k.w);
    launch_mdot(c->stream, n, 1, k.w, n, k.w, k.part, k.hdev + 2 * (cap + 2), nblk);
    MFS_HIP(hipMemcpyAsync(k.hhost, k.hdev, sizeof(double) * 3 * (cap + 2), hipMemcpyDeviceToHost, c->stream));
    MFS_HIP(hipStreamSynchronize(c->stream));
    for (int i = 0; i <= j; ++i) Hc(i, j) = k.hhost[i] + k.hhost[(cap + 2) + i];
    const double hn = std::sqrt(std::max(0.0, k.hhost[2 * (cap + 2)]));
    Hc(j + 1, j) = hn;
    for (int i = 0; i <= j + 1; ++i)
      if (!std::isfinite(Hc(i, j))) return Status{MFS_ERR_NUMERIC, "non-finite value in the Arnoldi process"};
    if (hn > 0.0) launch_scale_copy(c->stream, n, 1.0 / hn, k.w, k.V + (int64_t)(j + 1) * n);
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * Hc(i, j) + sn[i] * Hc(i + 1, j);
      Hc(i + 1, j) = -sn[i] * Hc(i, j) + cs[i] * Hc(i + 1, j);
      Hc(i, j) = t;
    }
    const double den = std::hypot(Hc(j, j), Hc(j + 1, j));
    cs[j] = Hc(j, j) / den;
    sn[j] = Hc(j + 1, j) / den;
    Hc(j, j) = den;
    Hc(j + 1, j) = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    kdone = j + 1;
    hist.push_back(std::fabs(g[j + 1]) / beta);
    rel_est = hist.back();
    if (prof && (kdone % 10 == 0))
      std::fprintf(stderr, "[mfs gmres] %s it %d resid %.3e  %.1f s\n", use32 ? "fp32-sum" : "fp64", kdone,
                   hist.back(), ms_since(t_start) * 1e-3);
    if (std::fabs(g[j + 1]) <= tol * beta || hn == 0.0) break;
    est[j] = rel_est;
    if (!force64 && stalled(est, first32, j)) {
      force64 = true;
      if (prof) std::fprintf(stderr, "[mfs gmres] mixed phase stalled at it %d: FP64 from here\n", kdone);
    }
  }
  std::vector<double> y(kdone);
  for (int i = kdone - 1; i >= 0; --i) {
    double s = g[i];
    for (int q = i + 1; q < kdone; ++q) s -= Hc(i, q) * y[q];
    y[i] = s / Hc(i, i);
  }
  MFS_HIP(hipMemcpyAsync(k.hdev, y.data(), sizeof(double) * kdone, hipMemcpyHostToDevice, c->stream));
  launch_gemv_n(c->stream, n, kdone, k.V, n, k.hdev, k.d);
  MFS_HIP(hipStreamSynchronize(c->stream));
  *iters = kdone;
  return Status{};
}

// Lockstep GMRES for R right-hand sides (the stacked form of gmres_core): every right-hand
// side keeps its own Krylov basis, Hessenberg matrix and Givens rotations; each step
// applies the operator to the R newest basis vectors at once (apply_T_rhs), so the
// all-pairs sum and the pair matrices are read once for all of them.  A right-hand side
// whose estimate reaches its tolerance is frozen (its slot is fed zeros).  The mixed
// kernel sum is used once every active right-hand side is below its switch point.
// r, d: R x n; tol, switch_below: R; iters: R.
Status gmres_core_rhs(mfs_ctx* c, int prob, bool mixed, int R, double delta, double& op_err, const double* r,
                      const double* tol, const bool* active_in, int maxit, int* iters,
                      std::vector<std::vector<double>>& hist) {
  Krylov& k = c->kr;
  const int64_t n = k.n;
  const int64_t ldv = (int64_t)R * n;
  const int nblk = mdot_blocks(n);
  const int cap = k.cap;
  const int64_t hstride = 3 * (int64_t)(cap + 2);
  Status st;
  std::vector<double> beta(R, 0.0), rel(R, 1.0), switch_below(R);
  for (int q = 0; q < R; ++q) switch_below[q] = switch_point(mixed, tol[q], delta, op_err);
  std::vector<char> active(R, 0);
  std::vector<int> kdone(R, 0);
  std::vector<std::vector<double>> H(R), cs(R), sn(R), g(R);
  std::vector<double> est(maxit, 1.0);   // worst active estimate
  int first32 = -1;
  bool force64 = false;
  MFS_HIP(hipMemsetAsync(k.d, 0, sizeof(double) * n * R, c->stream));
  MFS_HIP(hipMemsetAsync(k.V, 0, sizeof(double) * ldv, c->stream));
  for (int q = 0; q < R; ++q) {
    iters[q] = 0;
    if (!active_in[q]) continue;
    beta[q] = dnorm(c, r + q * n, &st);
    if (st.code) return st;
    if (!std::isfinite(beta[q])) return Status{MFS_ERR_NUMERIC, "non-finite residual"};
    if (beta[q] == 0.0) continue;
    active[q] = 1;
    launch_scale_copy(c->stream, n, 1.0 / beta[q], r + q * n, k.V + q * n);
    H[q].assign((size_t)(maxit + 1) * maxit, 0.0);
    cs[q].assign(maxit, 0.0);
    sn[q].assign(maxit, 0.0);
    g[q].assign(maxit + 1, 0.0);
    g[q][0] = beta[q];
  }
  const bool prof = std::getenv("MFS_PROFILE") != nullptr;
  auto t_start = clk::now();
  for (int j = 0; j < maxit; ++j) {
    bool any = false, all_low = true;
    for (int q = 0; q < R; ++q)
      if (active[q]) {
        any = true;
        if (rel[q] > switch_below[q]) all_low = false;
      }
    if (!any) break;
    bool use32 = mixed && all_low && !force64;
    double* vj = k.V + (int64_t)j * ldv;
    if (use32 && op_err < 0.0) {
      // first switch: measure the mixed operator on the active basis vectors (see gmres_core)
      if ((st = apply_T_rhs(c, prob, false, R, vj, k.w)).code) return st;
      if ((st = apply_T_rhs(c, prob, true, R, vj, k.tmp)).code) return st;
      double e = 0.0;
      for (int q = 0; q < R; ++q) {
        if (!active[q]) continue;
        e = std::max(e, rel_diff(c, n, k.tmp + q * n, k.w + q * n, &st));
        if (st.code) return st;
      }
      op_err = e;
      for (int q = 0; q < R; ++q) switch_below[q] = switch_point(mixed, tol[q], delta, op_err);
      if (prof) std::fprintf(stderr, "[mfs gmres x%d] mixed operator relative error %.2e\n", R, op_err);
      use32 = false;
    } else if ((st = apply_T_rhs(c, prob, use32, R, vj, k.w)).code) {
      return st;
    }
    if (use32 && first32 < 0) first32 = j;
    for (int q = 0; q < R; ++q) {
      if (!active[q]) continue;
      const double* Vq = k.V + q * n;
      double* wq = k.w + q * n;
      double* hq = k.hdev + q * hstride;
      launch_mdot(c->stream, n, j + 1, Vq, ldv, wq, k.part, hq, nblk);
      launch_maxpy(c->stream, n, j + 1, Vq, ldv, hq, wq);
      launch_mdot(c->stream, n, j + 1, Vq, ldv, wq, k.part, hq + (cap + 2), nblk);
      launch_maxpy(c->stream, n, j + 1, Vq, ldv, hq + (cap + 2), wq);
      launch_mdot(c->stream, n, 1, wq, n, wq, k.part, hq + 2 * (cap + 2), nblk);
    }
    MFS_HIP(hipMemcpyAsync(k.hhost, k.hdev, sizeof(double) * hstride * R, hipMemcpyDeviceToHost, c->stream));
    MFS_HIP(hipStreamSynchronize(c->stream));
    double* vn = k.V + (int64_t)(j + 1) * ldv;
    for (int q = 0; q < R; ++q) {
      if (!active[q]) {
        MFS_HIP(hipMemsetAsync(vn + q * n, 0, sizeof(double) * n, c->stream));
        continue;
      }
      const double* hh = k.hhost + q * hstride;
      auto Hc = [&](int row, int col) -> double& { return H[q][(size_t)col * (maxit + 1) + row]; };
      for (int i = 0; i <= j; ++i) Hc(i, j) = hh[i] + hh[(cap + 2) + i];
      const double hn = std::sqrt(std::max(0.0, hh[2 * (cap + 2)]));
      Hc(j + 1, j) = hn;
      for (int i = 0; i <= j + 1; ++i)
        if (!std::isfinite(Hc(i, j))) return Status{MFS_ERR_NUMERIC, "non-finite value in the Arnoldi process"};
      if (hn > 0.0)
        launch_scale_copy(c->stream, n, 1.0 / hn, k.w + q * n, vn + q * n);
      else
        MFS_HIP(hipMemsetAsync(vn + q * n, 0, sizeof(double) * n, c->stream));
      for (int i = 0; i < j; ++i) {
        const double t = cs[q][i] * Hc(i, j) + sn[q][i] * Hc(i + 1, j);
        Hc(i + 1, j) = -sn[q][i] * Hc(i, j) + cs[q][i] * Hc(i + 1, j);
        Hc(i, j) = t;
      }
      const double den = std::hypot(Hc(j, j), Hc(j + 1, j));
      cs[q][j] = Hc(j, j) / den;
      sn[q][j] = Hc(j + 1, j) / den;
      Hc(j, j) = den;
      Hc(j + 1, j) = 0.0;
      g[q][j + 1] = -sn[q][j] * g[q][j];
      g[q][j] = cs[q][j] * g[q][j];
      kdone[q] = j + 1;
      rel[q] = std::fabs(g[q][j + 1]) / beta[q];
      hist[q].push_back(rel[q]);
      if (std::fabs(g[q][j + 1]) <= tol[q] * beta[q] || hn == 0.0) active[q] = 0;
    }
    {
      double worst = 0.0;
      for (int q = 0; q < R; ++q)
        if (active[q]) worst = std::max(worst, rel[q]);
      est[j] = worst;
      if (!force64 && worst > 0.0 && stalled(est, first32, j)) {
        force64 = true;
        if (prof) std::fprintf(stderr, "[mfs gmres x%d] mixed phase stalled at it %d: FP64 from here\n", R, j + 1);
      }
    }
    if (prof && ((j + 1) % 10 == 0)) {
      double worst = 0;
      for (int q = 0; q < R; ++q) worst = std::max(worst, active[q] ? rel[q] : 0.0);
      std::fprintf(stderr, "[mfs gmres x%d] %s it %d worst active resid %.3e  %.1f s\n", R,
                   use32 ? "fp32-sum" : "fp64", j + 1, worst, ms_since(t_start) * 1e-3);
    }
  }
  for (int q = 0; q < R; ++q) {
    iters[q] = kdone[q];
    if (kdone[q] == 0) continue;
    auto Hc = [&](int row, int col) -> double& { return H[q][(size_t)col * (maxit + 1) + row]; };
    std::vector<double> y(kdone[q]);
    for (int i = kdone[q] - 1; i >= 0; --i) {
      double sum = g[q][i];
      for (int p = i + 1; p < kdone[q]; ++p) sum -= Hc(i, p) * y[p];
      y[i] = sum / Hc(i, i);
    }
    double* hq = k.hdev + q * hstride;
    MFS_HIP(hipMemcpyAsync(hq, y.data(), sizeof(double) * kdone[q], hipMemcpyHostToDevice, c->stream));
    launch_gemv_n(c->stream, n, kdone[q], k.V + q * n, ldv, hq, k.d + q * n);
    MFS_HIP(hipStreamSynchronize(c->stream));   // y is released at the end of this scope
  }
  return Status{};
}

// Relaxation parameter delta of the inner GMRES: operator applications switch from
// the FP64 to the mixed kernel sum once the residual estimate is below tol_inner /
// delta.  In the inexact-Krylov bound (Simoncini & Szyld 2003) delta stands for the
// mixed operator's relative error over the smallest singular value of the Hessenberg
// matrix, so it depends on the problem.  Mobility: the FP32 sum with FP64 disk
// moments is accurate to a few 1e-6 on smooth data; at P = 10^4 (area fraction 0.65,
// tol 5e-9) delta = 1e-6 needed 5 FP64 applications of 323 and 2 refinement steps;
// 1e-4 needed 17, 1e-2 needed 203.  Resistance: the compressed strengths of
// lubricated pairs are up to ~10^3 times the density, and the FP32 operator error
// reaches 5e-3 relative at gap 1e-3; delta = 1e-6 (mixed from the first step) left a
// 3-vector lockstep solve at 7e-6 after 300 iterations where 1e-4 converges, so
// resistance uses 1e-3.  MFS_MIXED_DELTA overrides both.  These are floors: the
// operator error measured at the first switch raises delta where the geometry makes
// the FP32 sum less accurate (closer gaps, larger compressed strengths), and a refinement
// step that misses its target raises it further (escalate).
// After a refinement step whose true residual missed the target by a factor f, the
// mixed operator's errors were amplified that much more than delta allowed for (the
// smallest singular values of the packed system); later steps switch that much later.
// delta reaches 1 at most (then the mixed operator serves only below the inner target).
double escalate(double delta, double op_err, double f) {
  if (!(f > 10.0)) return delta;
  const double d = std::min(1.0, std::max(delta, op_err) * f);
  if (std::getenv("MFS_PROFILE")) std::fprintf(stderr, "[mfs gmres] missed by %.2e: delta -> %.2e\n", f, d);
  return d;
}

double mixed_delta(int prob) {
  const double dflt = prob == MFS_MOBILITY ? 1e-6 : 1e-3;
  const char* e = std::getenv("MFS_MIXED_DELTA");
  const double d = e ? std::atof(e) : dflt;
  return d > 0 ? d : dflt;
}

}  // namespace

namespace {

struct SolveTotals {
  int iters = 0, outer = 0, hist_len = 0;
  double rel = 0, t_rhs = 0, t_it = 0, t_post = 0;
  bool noconv = false;
};

// One right-hand side: FP64 refinement around gmres_core (see the file comment).
Status solve_one(mfs_ctx* c, int prob, bool mixed, const double* given, double* out, const double* x0, double tol,
                 int max_iter, mfs_solve_info* info, SolveTotals& tot) {
  Krylov& k = c->kr;
  const int64_t n = k.n;
  Status st;
  auto t0 = clk::now();
  mfs_status s = mfs_rhs(c, (mfs_problem)prob, given, k.b);
  if (s != MFS_OK) return c->last;
  tot.t_rhs += ms_since(t0);
  t0 = clk::now();
  const double bn = dnorm(c, k.b, &st);
  if (st.code) return st;
  if (x0)
    MFS_HIP(hipMemcpyAsync(k.x, x0, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  else
    MFS_HIP(hipMemsetAsync(k.x, 0, sizeof(double) * n, c->stream));
  std::vector<double> hist;
  const int max_outer = mixed ? 10 : 3;
  int used = 0;
  double rel = 1.0;
  double delta = mixed_delta(prob);
  double op_err = -1.0;   // measured at the first switch to the mixed operator
  for (int o = 0; o < max_outer; ++o) {
    // r = b - T64 x
    if (o == 0 && !x0) {
      MFS_HIP(hipMemcpyAsync(k.r, k.b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    } else {
      if ((st = apply_T(c, prob, false, k.x, k.tmp)).code) return st;
      MFS_HIP(hipMemcpyAsync(k.r, k.b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
      launch_axpby(c->stream, n, -1.0, k.tmp, 1.0, k.r);
    }
    const double rn = dnorm(c, k.r, &st);
    if (st.code) return st;
    if (!std::isfinite(rn)) return Status{MFS_ERR_NUMERIC, "non-finite residual"};
    rel = bn > 0 ? rn / bn : 0.0;
    if (rel <= tol || used >= max_iter) break;
    if (mixed && o > 0) delta = escalate(delta, op_err, rel / tol);
    tot.outer = std::max(tot.outer, o + 1);
    // reach the target in one pass if the operator allows it
    const double tin = tol * bn / rn;
    if (std::getenv("MFS_PROFILE"))
      std::fprintf(stderr, "[mfs gmres] refinement %d: |r|/|b| = %.3e, inner tol %.3e, mixed below %.3e\n", o, rel,
                   tin, switch_point(mixed, tin, delta, op_err));
    int it = 0;
    if ((st = gmres_core(c, prob, mixed, delta, op_err, k.r, tin, max_iter - used, &it, hist)).code) return st;
    used += it;
    launch_axpby(c->stream, n, 1.0, k.d, 1.0, k.x);
    if (it == 0) break;
  }
  tot.iters += used;
  tot.t_it += ms_since(t0);
  t0 = clk::now();
  s = mfs_post(c, (mfs_problem)prob, k.x, out);
  if (s != MFS_OK) return c->last;
  tot.t_post += ms_since(t0);
  if (info && info->resid_hist && info->hist_cap > 0)
    for (double h : hist)
      if (tot.hist_len < info->hist_cap) info->resid_hist[tot.hist_len++] = h;
  tot.rel = std::max(tot.rel, rel);
  if (rel > tol) tot.noconv = true;
  return Status{};
}

// R right-hand sides in lockstep (2 <= R <= Krylov rcap): the refinement of solve_one
// with stacked residuals and gmres_core_rhs; each right-hand side stops on its own.
Status solve_stacked(mfs_ctx* c, int prob, bool mixed, int R, const double* given, double* out, const double* x0,
                     double tol, int max_iter, mfs_solve_info* info, SolveTotals& tot) {
  Krylov& k = c->kr;
  const int64_t n = k.n;
  Status st;
  auto t0 = clk::now();
  for (int q = 0; q < R; ++q)
    if (mfs_rhs(c, (mfs_problem)prob, given + 3 * (size_t)c->P * q, k.b + q * n) != MFS_OK) return c->last;
  tot.t_rhs += ms_since(t0);
  t0 = clk::now();
  std::vector<double> bn(R), rel(R, 1.0), tin(R);
  double delta = mixed_delta(prob);
  double op_err = -1.0;   // measured at the first switch to the mixed operator
  for (int q = 0; q < R; ++q) {
    bn[q] = dnorm(c, k.b + q * n, &st);
    if (st.code) return st;
  }
  if (x0)
    MFS_HIP(hipMemcpyAsync(k.x, x0, sizeof(double) * n * R, hipMemcpyDeviceToDevice, c->stream));
  else
    MFS_HIP(hipMemsetAsync(k.x, 0, sizeof(double) * n * R, c->stream));
  std::vector<std::vector<double>> hist(R);
  std::vector<int> used(R, 0), it(R, 0);
  std::unique_ptr<bool[]> act(new bool[R]);
  const int max_outer = mixed ? 10 : 3;
  for (int o = 0; o < max_outer; ++o) {
    if (o == 0 && !x0) {
      MFS_HIP(hipMemcpyAsync(k.r, k.b, sizeof(double) * n * R, hipMemcpyDeviceToDevice, c->stream));
    } else {
      if ((st = apply_T_rhs(c, prob, false, R, k.x, k.tmp)).code) return st;
      MFS_HIP(hipMemcpyAsync(k.r, k.b, sizeof(double) * n * R, hipMemcpyDeviceToDevice, c->stream));
      launch_axpby(c->stream, n * R, -1.0, k.tmp, 1.0, k.r);
    }
    bool any = false;
    for (int q = 0; q < R; ++q) {
      const double rn = dnorm(c, k.r + q * n, &st);
      if (st.code) return st;
      if (!std::isfinite(rn)) return Status{MFS_ERR_NUMERIC, "non-finite residual"};
      rel[q] = bn[q] > 0 ? rn / bn[q] : 0.0;
      act[q] = rel[q] > tol && used[q] < max_iter;
      if (act[q]) {
        any = true;
        tin[q] = tol * bn[q] / rn;
      } else {
        tin[q] = 1.0;
      }
    }
    if (!any) break;
    if (mixed && o > 0) {
      double f = 0.0;
      for (int q = 0; q < R; ++q)
        if (act[q]) f = std::max(f, rel[q] / tol);
      delta = escalate(delta, op_err, f);
    }
    tot.outer = std::max(tot.outer, o + 1);
    if (std::getenv("MFS_PROFILE")) {
      double worst = 0;
      for (int q = 0; q < R; ++q) worst = std::max(worst, rel[q]);
      std::fprintf(stderr, "[mfs gmres x%d] refinement %d: worst |r|/|b| = %.3e\n", R, o, worst);
    }
    int room = max_iter;
    for (int q = 0; q < R; ++q)
      if (act[q]) room = std::min(room, max_iter - used[q]);
    if ((st = gmres_core_rhs(c, prob, mixed, R, delta, op_err, k.r, tin.data(), act.get(), room, it.data(), hist))
            .code)
      return st;
    int most = 0;
    for (int q = 0; q < R; ++q) {
      used[q] += it[q];
      most = std::max(most, it[q]);
    }
    launch_axpby(c->stream, n * R, 1.0, k.d, 1.0, k.x);
    if (most == 0) break;
  }
  for (int q = 0; q < R; ++q) tot.iters += used[q];
  tot.t_it += ms_since(t0);
  t0 = clk::now();
  for (int q = 0; q < R; ++q)
    if (mfs_post(c, (mfs_problem)prob, k.x + q * n, out + 3 * (size_t)c->P * q) != MFS_OK) return c->last;
  tot.t_post += ms_since(t0);
  for (int q = 0; q < R; ++q) {
    if (info && info->resid_hist && info->hist_cap > 0)
      for (double h : hist[q])
        if (tot.hist_len < info->hist_cap) info->resid_hist[tot.hist_len++] = h;
    tot.rel = std::max(tot.rel, rel[q]);
    if (rel[q] > tol) tot.noconv = true;
  }
  return Status{};
}

}  // namespace

extern "C" mfs_status mfs_gmres_solve(mfs_ctx* c, mfs_problem prob, mfs_precision prec, int32_t n_rhs,
                                      const double* rhs, double* out, const double* x0, double tol,
                                      int32_t max_iter, mfs_solve_info* info) {
  if (!c) return MFS_ERR_ARG;
  auto failc = [&](Status st) {
    c->last = st;
    return st.code;
  };
  if ((prob != MFS_RESISTANCE && prob != MFS_MOBILITY) || (prec != MFS_FP64 && prec != MFS_MIXED) || n_rhs < 1 ||
      !rhs || !out || !(tol > 0) || max_iter < 1 || max_iter > 1000)
    return failc(Status{MFS_ERR_ARG, "bad argument (1 <= max_iter <= 1000, tol > 0)"});
  if (!c->ps[prob].ready && !c->pairs.empty())
    return failc(Status{MFS_ERR_STATE, "mfs_precompute_pairs has not run for this problem"});
  // right-hand sides run in lockstep groups of up to kLockstep
  constexpr int kLockstep = 8;
  const int R = std::min<int>(n_rhs, kLockstep);
  Status st = ensure_krylov(c, max_iter, R);
  if (st.code) return failc(st);
  const int64_t n = c->kr.n;
  const bool mixed = prec == MFS_MIXED;
  c->cnt_pair_evals = 0;
  c->cnt_mv64 = c->cnt_mv32 = 0;
  launch_zero_work(c);
  SolveTotals tot;
  // the densities are kept for mfs_get_density / flow evaluation
  c->mu_count = 0;
  if (c->mu_cap < n * n_rhs) {
    if (c->d_mu_last) dev_free(c, c->d_mu_last);
    c->d_mu_last = nullptr;
    c->mu_cap = 0;
    if (dev_malloc(c, &c->d_mu_last, sizeof(double) * n * n_rhs) != hipSuccess) {
      (void)hipGetLastError();
      return failc(Status{MFS_ERR_OOM, "device allocation of the solution densities failed"});
    }
    c->mu_cap = n * n_rhs;
  }
  for (int r0 = 0; r0 < n_rhs; r0 += R) {
    const int Rc = std::min(R, n_rhs - r0);
    const double* g = rhs + 3 * (size_t)c->P * r0;
    double* o = out + 3 * (size_t)c->P * r0;
    const double* x = x0 ? x0 + n * r0 : nullptr;
    st = Rc == 1 ? solve_one(c, prob, mixed, g, o, x, tol, max_iter, info, tot)
                 : solve_stacked(c, prob, mixed, Rc, g, o, x, tol, max_iter, info, tot);
    if (st.code) return failc(st);
    if (hipMemcpyAsync(c->d_mu_last + n * r0, c->kr.x, sizeof(double) * n * Rc, hipMemcpyDeviceToDevice,
                       c->stream) != hipSuccess)
      return failc(Status{MFS_ERR_DEVICE, "copy of the solution densities failed"});
  }
  c->mu_count = n_rhs;
  c->mu_prob = prob;
  if (info) {
    info->iters_total = tot.iters;
    info->outer_steps = tot.outer;
    info->rel_resid = tot.rel;
    info->hist_len = tot.hist_len;
    info->ms_rhs = tot.t_rhs;
    info->ms_iterate = tot.t_it;
    info->ms_post = tot.t_post;
    info->n_pairs = (int64_t)(c->pairs.size() / 2);
    info->matvecs_fp64 = c->cnt_mv64;
    info->matvecs_mixed = c->cnt_mv32;
    info->dense_pairs = c->cnt_pair_evals;
    int64_t w[3] = {0, 0, 0};
    if (mfs_kernel_sum_work(c, w, 0) != MFS_OK) return MFS_ERR_DEVICE;
    info->direct_pairs = w[0];
    info->disk_expansions = w[1];
    info->cluster_expansions = w[2];
  }
  if (tot.noconv) {
    char buf[64];
    std::snprintf(buf, sizeof(buf), "%.3e", tot.rel);
    c->last = Status{MFS_ERR_NOCONV, std::string("GMRES stopped above tolerance (relative residual ") + buf + ")"};
    return MFS_ERR_NOCONV;
  }
  c->last = Status{};
  return MFS_OK;
}
