// Flow evaluation and boundary residual (C ABI part of include/mfs.h).
//
// After a solve, the velocity at any point outside the bodies follows from the density mu
// through the two-body representation (Sec. 3.3, eq. chi; the flowEval output of Alg. 2):
// the coarse strengths of every disk (one-body plus the compressed pair corrections) give
// the field everywhere except near a close pair, where the pair's fine sources replace its
// compressed strengths.  The fine sources need each pair's fine map G, which the pair
// precompute keeps when mfs_keep_fine_factors has been called.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "internal.h"

using namespace mfs;

namespace {

mfs_status failc(mfs_ctx* c, Status st) {
  c->last = st;
  return st.code;
}

template <class T>
Status grow(mfs_ctx* c, T** p, int64_t* cap, int64_t need) {
  if (*cap >= need && *p) return Status{};
  dev_free(c, *p);
  *p = nullptr;
  *cap = 0;
  if (dev_malloc(c, p, sizeof(T) * std::max<int64_t>(need, 1)) != hipSuccess)
    return Status{MFS_ERR_OOM, "device allocation for flow evaluation failed"};
  *cap = need;
  return Status{};
}

// flag[0] = 1 if some body index is outside [-1, P) (plain stores of the same value).
__global__ void k_check_body(int64_t n_pts, const int32_t* __restrict__ body, int P, int* __restrict__ flag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_pts && (body[t] < -1 || body[t] >= P)) flag[0] = 1;
}

struct Scratch {   // per-call device buffers of the context, freed on every exit path
  mfs_ctx* c;
  void* p = nullptr;
  explicit Scratch(mfs_ctx* ctx) : c(ctx) {}
  hipError_t alloc(size_t bytes) { return dev_malloc(c, &p, bytes); }
  ~Scratch() { dev_free(c, p); }
};

// u at n_pts points (device), see mfs_flow_eval.
Status flow_eval(mfs_ctx* c, int prob, const double* mu, const double* given, int64_t n_pts, const double* pts,
                 const int32_t* body, double* u) {
  const int C = (int)(c->pairs.size() / 2);
  const PairSet& ps = c->ps[prob];
  if (C > 0 && !ps.ready) return Status{MFS_ERR_STATE, "mfs_precompute_pairs has not run for this problem"};
  if (C > 0 && !ps.fine)
    return Status{MFS_ERR_STATE, "no fine factors: call mfs_keep_fine_factors before mfs_precompute_pairs"};
  if (n_pts == 0) return Status{};
  {
    Scratch flag(c);
    int h = 0;
    MFS_HIP(flag.alloc(sizeof(int)));
    MFS_HIP(hipMemcpyAsync(flag.p, &h, sizeof(int), hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_check_body, dim3((unsigned)((n_pts + 255) / 256)), dim3(256), 0, c->stream, n_pts, body,
                       c->P, (int*)flag.p);
    MFS_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    MFS_HIP(hipStreamSynchronize(c->stream));
    if (h) return Status{MFS_ERR_ARG, "body index outside [-1, P)"};
  }
  Status st;
  int64_t fsrc_cap = c->d_fsrc ? c->Ns : 0;
  if ((st = grow(c, &c->d_fsrc, &fsrc_cap, c->Ns)).code) return st;
  int64_t fmp_cap = c->d_fmp64 ? mp64_record(c) : 0;
  if ((st = grow(c, &c->d_fmp64, &fmp_cap, mp64_record(c))).code) return st;
  if (C > 0) {
    int64_t ptil_cap = c->d_ptil ? c->xoff[C] : 0;
    if ((st = grow(c, &c->d_ptil, &ptil_cap, c->xoff[C])).code) return st;
    if ((st = grow(c, &c->d_sigf, &c->sigf_cap, ps.yoff[C])).code) return st;
  }
  // step 1 of Alg. 3: lambda_bar and the pairs' lambda_tilde; total strengths with positions
  launch_onebody_apply(c, prob, mu, c->d_lam_bar);
  launch_pair_A(c, prob, c->d_lam_bar, c->d_ltil);
  launch_gather_project_to(c, prob, c->d_lam_bar, c->d_ltil, true, c->d_fsrc);
  if (prob == MFS_MOBILITY) {
    MFS_HIP(hipMemcpyAsync(c->d_given, given, sizeof(double) * 3 * c->P, hipMemcpyHostToDevice, c->stream));
    launch_add_rhs_sources(c, c->d_given, c->d_fsrc);
  }
  launch_moments64(c, c->d_fsrc, c->d_fmp64);
  if (!launch_kernel_sum_points(c, c->d_fsrc, c->d_fmp64, n_pts, pts, body, u))
    return Status{MFS_ERR_OOM, "device allocation of the kernel-sum partials failed"};
  if (C > 0) {
    launch_fine_strengths(c, prob, c->d_lam_bar, c->d_ltil, c->d_ptil, c->d_sigf);
    launch_flow_near(c, prob, n_pts, pts, body, c->d_ptil, c->d_sigf, u);
  }
  MFS_HIP(hipGetLastError());
  MFS_HIP(hipStreamSynchronize(c->stream));   // given is a host buffer of the caller
  return Status{};
}

}  // namespace

extern "C" {

mfs_status mfs_keep_fine_factors(mfs_ctx* c, int32_t keep) {
  if (!c) return MFS_ERR_ARG;
  c->keep_fine = keep != 0;
  c->last = Status{};
  return MFS_OK;
}

mfs_status mfs_get_density(const mfs_ctx* cc, int32_t rhs, double* mu) {
  mfs_ctx* c = const_cast<mfs_ctx*>(cc);
  if (!c) return MFS_ERR_ARG;
  if (!mu) return failc(c, Status{MFS_ERR_ARG, "mu is NULL"});
  if (c->mu_count == 0) return failc(c, Status{MFS_ERR_STATE, "no solve has run on this context"});
  if (rhs < 0 || rhs >= c->mu_count)
    return failc(c, Status{MFS_ERR_ARG, "right-hand side index out of range of the latest solve"});
  const int64_t n = 2 * c->Nt;
  if (hipMemcpyAsync(mu, c->d_mu_last + n * rhs, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream) !=
          hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipGetLastError();
    return failc(c, Status{MFS_ERR_DEVICE, "copy of the density failed"});
  }
  c->last = Status{};
  return MFS_OK;
}

mfs_status mfs_flow_eval(mfs_ctx* c, mfs_problem prob, const double* mu, const double* given, int64_t n_pts,
                         const double* pts, const int32_t* body, double* u) {
  if (!c) return MFS_ERR_ARG;
  if (prob != MFS_RESISTANCE && prob != MFS_MOBILITY) return failc(c, Status{MFS_ERR_ARG, "unknown problem"});
  if (n_pts < 0 || !mu || (n_pts > 0 && (!pts || !body || !u)) || (prob == MFS_MOBILITY && !given))
    return failc(c, Status{MFS_ERR_ARG, "bad argument (mobility needs the forces and torques)"});
  if (prob == MFS_MOBILITY)
    for (int q = 0; q < 3 * c->P; ++q)
      if (!std::isfinite(given[q])) return failc(c, Status{MFS_ERR_NUMERIC, "non-finite force or torque"});
  Status st = flow_eval(c, prob, mu, given, n_pts, pts, body, u);
  if (st.code) return failc(c, st);
  c->last = Status{};
  return MFS_OK;
}

mfs_status mfs_boundary_residual(mfs_ctx* c, mfs_problem prob, const double* mu, const double* given,
                                 const double* rigid, int32_t n_per_body, double* eps, double* eps_max) {
  if (!c) return MFS_ERR_ARG;
  if (prob != MFS_RESISTANCE && prob != MFS_MOBILITY) return failc(c, Status{MFS_ERR_ARG, "unknown problem"});
  if (!mu || !rigid || !eps_max || n_per_body < 1 || n_per_body > 1 << 20 || (prob == MFS_MOBILITY && !given))
    return failc(c, Status{MFS_ERR_ARG, "bad argument (1 <= n_per_body <= 2^20; mobility needs given)"});
  for (int q = 0; q < 3 * c->P; ++q)
    if (!std::isfinite(rigid[q])) return failc(c, Status{MFS_ERR_NUMERIC, "non-finite rigid motion"});
  const int64_t n_pts = (int64_t)c->P * n_per_body;
  const int64_t nblk = (n_pts + 255) / 256;
  Scratch s_pts(c), s_body(c), s_u(c), s_rig(c), s_max(c);
  if (s_pts.alloc(sizeof(double) * 2 * n_pts) != hipSuccess || s_body.alloc(sizeof(int32_t) * n_pts) != hipSuccess ||
      s_u.alloc(sizeof(double) * 2 * n_pts) != hipSuccess || s_rig.alloc(sizeof(double) * 3 * c->P) != hipSuccess ||
      s_max.alloc(sizeof(double) * 2 * (nblk + 1)) != hipSuccess)
    return failc(c, Status{MFS_ERR_OOM, "device allocation for the boundary residual failed"});
  double* pts = (double*)s_pts.p;
  int32_t* body = (int32_t*)s_body.p;
  double* u = (double*)s_u.p;
  launch_boundary_nodes(c, n_per_body, pts, body);
  Status st = flow_eval(c, prob, mu, given, n_pts, pts, body, u);
  if (st.code) return failc(c, st);
  double mx[2] = {0.0, 0.0};
  if (hipMemcpyAsync(s_rig.p, rigid, sizeof(double) * 3 * c->P, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return failc(c, Status{MFS_ERR_DEVICE, "copy of the rigid motions failed"});
  launch_boundary_residual(c, n_pts, pts, body, u, (const double*)s_rig.p, eps, (double*)s_max.p);
  if (hipMemcpyAsync(mx, s_max.p, sizeof(mx), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    (void)hipGetLastError();
    return failc(c, Status{MFS_ERR_DEVICE, "boundary residual kernels failed"});
  }
  *eps_max = mx[1] > 0.0 ? mx[0] / mx[1] : mx[0];
  c->last = Status{};
  return MFS_OK;
}

}  // extern "C"
