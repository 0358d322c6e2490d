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
// upper estimate of the mixed operator's relative error.  This is the relaxation
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

#include "internal.h"

using namespace mfs;

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t0) { return std::chrono::duration<double, std::milli>(clk::now() - t0).count(); }

Status ensure_krylov(mfs_ctx* c, int cap) {
  Krylov& k = c->kr;
  const int64_t n = 2 * c->Nt;
  if (k.V && k.cap >= cap && k.n == n) return Status{};
  if (k.V) (void)hipFree(k.V);
  if (k.part) (void)hipFree(k.part);
  if (k.hdev) (void)hipFree(k.hdev);
  if (k.hhost) (void)hipHostFree(k.hhost);
  k.V = k.part = k.hdev = k.hhost = nullptr;
  for (double** p : {&k.w, &k.x, &k.r, &k.b, &k.d, &k.tmp})
    if (!*p) MFS_HIP(hipMalloc((void**)p, sizeof(double) * n));
  if (hipMalloc((void**)&k.V, sizeof(double) * n * (cap + 1)) != hipSuccess) {
    (void)hipGetLastError();
    k.V = nullptr;
    return Status{MFS_ERR_OOM, "Krylov basis of " + std::to_string(cap + 1) + " vectors does not fit"};
  }
  const int nblk = mdot_blocks(n);
  MFS_HIP(hipMalloc((void**)&k.part, sizeof(double) * nblk * (cap + 2)));
  MFS_HIP(hipMalloc((void**)&k.hdev, sizeof(double) * 3 * (cap + 2)));
  MFS_HIP(hipHostMalloc((void**)&k.hhost, sizeof(double) * 3 * (cap + 2), hipHostMallocDefault));
  k.cap = cap;
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
Status gmres_core(mfs_ctx* c, int prob, bool mixed, double switch_below, const double* r, double tol, int maxit,
                  int* iters, std::vector<double>& hist) {
  Krylov& k = c->kr;
  const int64_t n = k.n;
  const int nblk = mdot_blocks(n);
  Status st;
  const double beta = dnorm(c, r, &st);
  if (st.code) return st;
  MFS_HIP(hipMemsetAsync(k.d, 0, sizeof(double) * n, c->stream));
  *iters = 0;
  if (!std::isfinite(beta)) return Status{MFS_ERR_NUMERIC, "non-finite residual"};
  if (beta == 0.0) return Status{};
  launch_scale_copy(c->stream, n, 1.0 / beta, r, k.V);
  std::vector<double> H((size_t)(maxit + 1) * maxit, 0.0), cs(maxit), sn(maxit), g(maxit + 1, 0.0);
  auto Hc = [&](int row, int col) -> double& { return H[(size_t)col * (maxit + 1) + row]; };
  g[0] = beta;
  int kdone = 0;
  const int cap = k.cap;
  const bool prof = std::getenv("MFS_PROFILE") != nullptr;
  auto t_start = clk::now();
  double rel_est = 1.0;
  for (int j = 0; j < maxit; ++j) {
    double* vj = k.V + (int64_t)j * n;
    const bool use32 = mixed && rel_est <= switch_below;
    if ((st = apply_T(c, prob, use32, vj, k.w)).code) return st;
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

// Relaxation parameter delta of the inner GMRES: operator applications switch from
// the FP64 to the mixed kernel sum once the residual estimate is below tol_inner /
// delta.  In the inexact-Krylov bound (Simoncini & Szyld 2003) delta stands for the
// mixed operator's relative error over the smallest singular value of the Hessenberg
// matrix.  The FP32 sum with FP64 disk moments is accurate to a few 1e-6 on smooth
// data; at P = 10^4 (area fraction 0.65) delta = 1e-4 reached tol 5e-9 in 3
// refinement steps with 17 of 325 applications in FP64 (1e-3: 32 FP64, 1e-2: 203).
// MFS_MIXED_DELTA overrides it.
double mixed_delta() {
  const char* e = std::getenv("MFS_MIXED_DELTA");
  const double d = e ? std::atof(e) : 1e-4;
  return d > 0 ? d : 1e-4;
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
#define MFS_HIP_CALL_OR(call)                                                        \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess) return failc(Status{MFS_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}); \
  } while (0)
  if ((prob != MFS_RESISTANCE && prob != MFS_MOBILITY) || (prec != MFS_FP64 && prec != MFS_MIXED) || n_rhs < 1 ||
      !rhs || !out || !(tol > 0) || max_iter < 1 || max_iter > 1000)
    return failc(Status{MFS_ERR_ARG, "bad argument (1 <= max_iter <= 1000, tol > 0)"});
  if (!c->ps[prob].ready && !c->pairs.empty())
    return failc(Status{MFS_ERR_STATE, "mfs_precompute_pairs has not run for this problem"});
  Status st = ensure_krylov(c, max_iter);
  if (st.code) return failc(st);
  Krylov& k = c->kr;
  const int64_t n = k.n;
  mfs_status result = MFS_OK;
  double t_rhs = 0, t_it = 0, t_post = 0;
  int iters_total = 0, outer = 0, hist_len = 0;
  double rel = 0;
  c->cnt_pair_evals = 0;
  c->cnt_mv64 = c->cnt_mv32 = 0;
  for (int rr = 0; rr < n_rhs; ++rr) {
    auto t0 = clk::now();
    mfs_status s = mfs_rhs(c, prob, rhs + 3 * (size_t)c->P * rr, k.b);
    if (s != MFS_OK) return s;
    t_rhs += ms_since(t0);
    t0 = clk::now();
    const double bn = dnorm(c, k.b, &st);
    if (st.code) return failc(st);
    if (x0)
      MFS_HIP_CALL_OR(hipMemcpyAsync(k.x, x0 + n * rr, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    else
      MFS_HIP_CALL_OR(hipMemsetAsync(k.x, 0, sizeof(double) * n, c->stream));
    std::vector<double> hist;
    const bool mixed = prec == MFS_MIXED;
    // outer refinement (a single pass for FP64 with x0 = 0)
    const int max_outer = mixed ? 10 : 3;
    int used = 0;
    rel = 1.0;
    for (int o = 0; o < max_outer; ++o) {
      // r = b - T64 x
      if (o == 0 && !x0) {
        MFS_HIP_CALL_OR(hipMemcpyAsync(k.r, k.b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
      } else {
        if ((st = apply_T(c, prob, false, k.x, k.tmp)).code) return failc(st);
        MFS_HIP_CALL_OR(hipMemcpyAsync(k.r, k.b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
        launch_axpby(c->stream, n, -1.0, k.tmp, 1.0, k.r);
      }
      const double rn = dnorm(c, k.r, &st);
      if (st.code) return failc(st);
      if (!std::isfinite(rn)) return failc(Status{MFS_ERR_NUMERIC, "non-finite residual"});
      rel = bn > 0 ? rn / bn : 0.0;
      if (rel <= tol || used >= max_iter) break;
      ++outer;
      // reach the target in one pass if the operator allows it
      const double tin = tol * bn / rn;
      const double switch_below = mixed ? std::min(1.0, tin / mixed_delta()) : 0.0;
      if (std::getenv("MFS_PROFILE"))
        std::fprintf(stderr, "[mfs gmres] refinement %d: |r|/|b| = %.3e, inner tol %.3e, mixed below %.3e\n", o, rel,
                     tin, switch_below);
      int it = 0;
      if ((st = gmres_core(c, prob, mixed, switch_below, k.r, tin, max_iter - used, &it, hist)).code)
        return failc(st);
      used += it;
      launch_axpby(c->stream, n, 1.0, k.d, 1.0, k.x);
      if (it == 0) break;
    }
    iters_total += used;
    t_it += ms_since(t0);
    t0 = clk::now();
    s = mfs_post(c, prob, k.x, out + 3 * (size_t)c->P * rr);
    if (s != MFS_OK) return s;
    t_post += ms_since(t0);
    if (info && info->resid_hist && info->hist_cap > 0) {
      for (double h : hist)
        if (hist_len < info->hist_cap) info->resid_hist[hist_len++] = h;
    }
    if (rel > tol) result = MFS_ERR_NOCONV;
  }
  if (info) {
    info->iters_total = iters_total;
    info->outer_steps = outer;
    info->rel_resid = rel;
    info->hist_len = hist_len;
    info->ms_rhs = t_rhs;
    info->ms_iterate = t_it;
    info->ms_post = t_post;
    info->n_pairs = (int64_t)(c->pairs.size() / 2);
    info->matvecs_fp64 = c->cnt_mv64;
    info->matvecs_mixed = c->cnt_mv32;
    info->pair_evals = c->cnt_pair_evals;
  }
  if (result != MFS_OK) {
    char buf[64];
    std::snprintf(buf, sizeof(buf), "%.3e", rel);
    c->last = Status{result, std::string("GMRES stopped above tolerance (relative residual ") + buf + ")"};
    return result;
  }
  c->last = Status{};
  return MFS_OK;
}
