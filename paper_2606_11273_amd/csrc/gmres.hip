// mfs_gmres_solve: RHS -> GMRES on the Alg. 3 operator -> post-processing.
//
// GMRES is unrestarted, x0 = 0 unless given, with the Krylov basis resident in
// device memory.  Orthogonalisation is classical Gram-Schmidt applied twice
// (CGS2): two passes of h = V^T w, w -= V h per iteration, all FP64, with the dot
// products reduced in a fixed order.  The (k+1) x k Hessenberg least-squares
// problem stays on the device: one wave per right-hand side applies the Givens
// rotations in FP64 (k_givens), scales the next basis vector and records the
// residual estimate.  The host does not wait for an iteration before launching the
// next one: it reads iteration j's estimate while iteration j + 1 runs, so it
// learns of convergence one iteration late and one extra iteration is launched
// and discarded (the device leaves a finished right-hand side's state alone).
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
  for (double** p : {&k.V, &k.part, &k.hdev, &k.w, &k.x, &k.r, &k.b, &k.d, &k.tmp, &k.H, &k.cs, &k.sn, &k.g, &k.y,
                     &k.ctl, &k.rec})
    if (*p) dev_free(c, *p);
  if (k.hhost) (void)hipHostFree(k.hhost);
  if (k.hrec) (void)hipHostFree(k.hrec);
  k.V = k.part = k.hdev = k.hhost = k.w = k.x = k.r = k.b = k.d = k.tmp = nullptr;
  k.H = k.cs = k.sn = k.g = k.y = k.ctl = k.rec = k.hrec = nullptr;
  k.cap = k.rcap = 0;
  for (hipEvent_t& e : k.ev)
    if (!e) MFS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
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
  const size_t cR = (size_t)R;
  MFS_HIP(dev_malloc(c, (void**)&k.H, sizeof(double) * cR * (cap + 1) * cap));
  MFS_HIP(dev_malloc(c, (void**)&k.cs, sizeof(double) * cR * cap));
  MFS_HIP(dev_malloc(c, (void**)&k.sn, sizeof(double) * cR * cap));
  MFS_HIP(dev_malloc(c, (void**)&k.g, sizeof(double) * cR * (cap + 1)));
  MFS_HIP(dev_malloc(c, (void**)&k.y, sizeof(double) * cR * (cap + 1)));
  MFS_HIP(dev_malloc(c, (void**)&k.ctl, sizeof(double) * cR * kGmCtl));
  MFS_HIP(dev_malloc(c, (void**)&k.rec, sizeof(double) * cR * 4 * (cap + 1)));
  MFS_HIP(hipHostMalloc((void**)&k.hrec, sizeof(double) * cR * 4 * (cap + 1), hipHostMallocDefault));
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
// mixed operator (negative while unknown).  A mixed operator whose measured error exceeds
// kMixedMaxErr is not used at all: its FP32 errors, amplified by the small singular values
// of the packed system, stall the Krylov process (measured: 1e-4 plateaus with 60-source
// rings on the ring-rule radius and on the bidisperse packing, where the FP64 solve needs a
// fraction of the iterations), so the solve stays FP64 after the one measurement.  This
// holds for mobility; resistance, whose compressed lubrication strengths make its mixed
// operator error 1e-4 .. 5e-3 even on small grids, relies on its larger delta instead.
constexpr double kMixedMaxErr = 1e-5;

double switch_point(bool mixed, double tol, double delta, double op_err, double max_err) {
  if (!mixed || op_err > max_err) return 0.0;
  return std::min(1.0, tol / std::max(delta, op_err));
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

// GMRES for R right-hand sides in lockstep (R = 1: a single solve): every right-hand side
// keeps its own Krylov basis, Hessenberg matrix and Givens rotations (on the device); each
// step applies the operator to the R newest basis vectors at once (apply_T_rhs), so the
// all-pairs sum and the pair matrices are read once for all of them.  A right-hand side
// whose estimate reaches its tolerance is frozen (the device feeds it zeros from then on).
// The mixed kernel sum is used once every active right-hand side is below its switch
// point.  Decisions (operator precision, stall, stop) use the estimates the host has read,
// which lag one iteration.  r, d: R x n; tol: R; iters: R.
Status gmres_core_rhs(mfs_ctx* c, int prob, bool mixed, int R, double delta, double& op_err, const double* r,
                      const double* tol, const bool* active_in, int maxit, int* iters,
                      std::vector<std::vector<double>>& hist) {
  Krylov& k = c->kr;
  const int64_t n = k.n;
  const int64_t ldv = (int64_t)R * n;
  const int nblk = mdot_blocks(n);
  const int cap = k.cap;
  const int64_t hstride = 3 * (int64_t)(cap + 2);
  hipStream_t s = c->stream;
  Status st;
  const double max_err = prob == MFS_MOBILITY ? kMixedMaxErr : INFINITY;
  std::vector<double> beta(R, 0.0), rel(R, 1.0), switch_below(R);
  for (int q = 0; q < R; ++q) switch_below[q] = switch_point(mixed, tol[q], delta, op_err, max_err);
  std::vector<char> active(R, 0);   // as far as the host knows
  std::vector<double> est(maxit, 1.0);   // worst active estimate per iteration
  int first32 = -1;
  bool force64 = false;
  MFS_HIP(hipMemsetAsync(k.d, 0, sizeof(double) * n * R, s));
  MFS_HIP(hipMemsetAsync(k.V, 0, sizeof(double) * ldv, s));
  std::vector<double> ctl((size_t)R * kGmCtl, 0.0), g0((size_t)R * (cap + 1), 0.0);
  for (int q = 0; q < R; ++q) {
    iters[q] = 0;
    double* cq = ctl.data() + (size_t)q * kGmCtl;
    cq[kGmDone] = 1.0;
    cq[kGmEst] = 1.0;
    if (!active_in[q]) continue;
    beta[q] = dnorm(c, r + q * n, &st);
    if (st.code) return st;
    if (!std::isfinite(beta[q])) return Status{MFS_ERR_NUMERIC, "non-finite residual"};
    if (beta[q] == 0.0) continue;
    active[q] = 1;
    cq[kGmBeta] = beta[q];
    cq[kGmTol] = tol[q] * beta[q];
    cq[kGmDone] = 0.0;
    g0[(size_t)q * (cap + 1)] = beta[q];
    launch_scale_copy(s, n, 1.0 / beta[q], r + q * n, k.V + q * n);
  }
  MFS_HIP(hipMemcpyAsync(k.ctl, ctl.data(), sizeof(double) * ctl.size(), hipMemcpyHostToDevice, s));
  MFS_HIP(hipMemcpyAsync(k.g, g0.data(), sizeof(double) * g0.size(), hipMemcpyHostToDevice, s));
  const bool prof = std::getenv("MFS_PROFILE") != nullptr;
  auto t_start = clk::now();
  bool use32_last = false;
  // read iteration jj's records (the host waits for that iteration's event first)
  auto absorb = [&](int jj) -> Status {
    MFS_HIP(hipEventSynchronize(k.ev[jj & 1]));
    double worst = 0.0;
    for (int q = 0; q < R; ++q) {
      const double* o = k.hrec + ((int64_t)jj * R + q) * 4;
      if (o[3] != 0.0) return Status{MFS_ERR_NUMERIC, "non-finite value in the Arnoldi process"};
      if (!active[q]) continue;
      if ((int)o[2] == jj + 1) {   // this iteration advanced right-hand side q
        rel[q] = o[0];
        hist[q].push_back(o[0]);
      }
      if (o[1] != 0.0) active[q] = 0;
      else worst = std::max(worst, rel[q]);
    }
    est[jj] = worst;
    if (!force64 && worst > 0.0 && stalled(est, first32, jj)) {
      force64 = true;
      if (prof) std::fprintf(stderr, "[mfs gmres x%d] mixed phase stalled at it %d: FP64 from here\n", R, jj + 1);
    }
    if (prof && ((jj + 1) % 10 == 0))
      std::fprintf(stderr, "[mfs gmres x%d] %s it %d worst active resid %.3e  %.1f s\n", R,
                   use32_last ? "fp32-sum" : "fp64", jj + 1, worst, ms_since(t_start) * 1e-3);
    return Status{};
  };
  int launched = 0, absorbed = 0;
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
      // first switch: measure the mixed operator on the active basis vectors against the FP64
      // one (which this iteration keeps), then move the switch points
      if ((st = apply_T_rhs(c, prob, false, R, vj, k.w)).code) return st;
      if ((st = apply_T_rhs(c, prob, true, R, vj, k.tmp)).code) return st;
      double e = 0.0;
      for (int q = 0; q < R; ++q) {
        if (!active[q]) continue;
        e = std::max(e, rel_diff(c, n, k.tmp + q * n, k.w + q * n, &st));
        if (st.code) return st;
      }
      op_err = e;
      for (int q = 0; q < R; ++q) switch_below[q] = switch_point(mixed, tol[q], delta, op_err, max_err);
      if (prof) std::fprintf(stderr, "[mfs gmres x%d] mixed operator relative error %.2e\n", R, op_err);
      use32 = false;
    } else if ((st = apply_T_rhs(c, prob, use32, R, vj, k.w)).code) {
      return st;
    }
    if (use32 && first32 < 0) first32 = j;
    use32_last = use32;
    for (int q = 0; q < R; ++q) {
      if (!active[q]) continue;   // the device zero-feeds it
      const double* Vq = k.V + q * n;
      double* wq = k.w + q * n;
      double* hq = k.hdev + q * hstride;
      launch_mdot(s, n, j + 1, Vq, ldv, wq, k.part, hq, nblk);
      launch_maxpy(s, n, j + 1, Vq, ldv, hq, wq);
      launch_mdot(s, n, j + 1, Vq, ldv, wq, k.part, hq + (cap + 2), nblk);
      launch_maxpy(s, n, j + 1, Vq, ldv, hq + (cap + 2), wq);
      launch_mdot(s, n, 1, wq, n, wq, k.part, hq + 2 * (cap + 2), nblk);
    }
    launch_givens(s, j, cap, R, k.hdev, hstride, k.H, k.cs, k.sn, k.g, k.ctl, k.rec);
    launch_scale_ctl(s, n, R, k.ctl, k.w, k.V + (int64_t)(j + 1) * ldv);
    MFS_HIP(hipMemcpyAsync(k.hrec + (int64_t)j * R * 4, k.rec + (int64_t)j * R * 4, sizeof(double) * 4 * R,
                           hipMemcpyDeviceToHost, s));
    MFS_HIP(hipGetLastError());
    MFS_HIP(hipEventRecord(k.ev[j & 1], s));
    launched = j + 1;
    // iteration j runs while the host reads iteration j - 1
    if (j >= 1) {
      if ((st = absorb(j - 1)).code) return st;
      absorbed = j;
    }
  }
  MFS_HIP(hipStreamSynchronize(s));
  for (int jj = absorbed; jj < launched; ++jj)
    if ((st = absorb(jj)).code) return st;
  MFS_HIP(hipMemcpyAsync(ctl.data(), k.ctl, sizeof(double) * ctl.size(), hipMemcpyDeviceToHost, s));
  MFS_HIP(hipStreamSynchronize(s));
  launch_backsolve(s, cap, R, k.H, k.g, k.ctl, k.y);
  for (int q = 0; q < R; ++q) {
    iters[q] = (int)ctl[(size_t)q * kGmCtl + kGmK];
    if (iters[q] > 0) launch_gemv_n(s, n, iters[q], k.V + q * n, ldv, k.y + (int64_t)q * (cap + 1), k.d + q * n);
  }
  MFS_HIP(hipGetLastError());
  MFS_HIP(hipStreamSynchronize(s));
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

// R right-hand sides in lockstep (1 <= R <= Krylov rcap): FP64 refinement on the true
// residual around gmres_core_rhs (see the file comment); each right-hand side stops on its own.
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
    st = solve_stacked(c, prob, mixed, Rc, g, o, x, tol, max_iter, info, tot);
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
    int64_t w[5] = {0, 0, 0, 0, 0};
    if (mfs_kernel_sum_work(c, w, 0) != MFS_OK) return MFS_ERR_DEVICE;
    info->direct_pairs = w[0];
    info->ring_expansions = w[1];
    info->expansion_terms = w[2];
    info->local_translations = w[3];
    info->local_evaluations = w[4];
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
