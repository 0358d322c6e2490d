// C ABI of the library (include/mfs.h): setup, precompute, matvec, solve.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <algorithm>
#include <new>

#include "internal.h"

using namespace mfs;

namespace mfs {

hipError_t dev_malloc(mfs_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (c && c->alloc.alloc) {
    *p = c->alloc.alloc(bytes ? bytes : 1, c->alloc.user);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  const hipError_t e = hipMalloc(p, bytes ? bytes : 1);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
  }
  return e;
}

void dev_free(mfs_ctx* c, void* p) {
  if (!p) return;
  if (c && c->alloc.alloc)
    c->alloc.free(p, c->alloc.user);
  else
    (void)hipFree(p);
}

}  // namespace mfs

namespace {

thread_local std::string g_setup_err;

mfs_status fail(mfs_ctx* c, Status st) {
  if (c)
    c->last = st;
  else
    g_setup_err = st.msg;
  return st.code;
}

mfs_status ok(mfs_ctx* c) {
  if (c) c->last = Status{};
  return MFS_OK;
}

template <class T>
Status dalloc(mfs_ctx* c, T** p, size_t n) {
  *p = nullptr;
  if (dev_malloc(c, (void**)p, sizeof(T) * (n ? n : 1)) != hipSuccess) {
    (void)hipGetLastError();
    return Status{MFS_ERR_OOM, "device allocation of " + std::to_string(sizeof(T) * n) + " bytes failed"};
  }
  return Status{};
}

template <class T>
Status upload(mfs_ctx* c, T** p, const std::vector<T>& h, hipStream_t s) {
  Status st = dalloc(c, p, h.size());
  if (st.code) return st;
  if (!h.empty()) MFS_HIP(hipMemcpyAsync(*p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s));
  return Status{};
}

void free_all(mfs_ctx* c) {
  void* ptrs[] = {c->d_nbr_off,  c->d_nbr_list, c->d_src_off,  c->d_col_off,  c->d_cls,       c->d_tgt_body,
                  c->d_pairs,    c->d_bp_off,   c->d_bp_list,  c->d_xoff,     c->d_aoff,      c->d_coff,
                  c->d_centers,  c->d_Y,        c->d_X,        c->d_lam_bar,  c->d_ltil,      c->d_u,
                  c->d_corr,     c->d_upart,    c->d_epair,    c->d_out3,     c->d_given,     c->d_src64,
                  c->ps[0].A,    c->ps[0].E,    c->ps[1].A,    c->ps[1].E,    c->kr.V,        c->kr.w,
                  c->kr.part,    c->kr.hdev,    c->kr.x,       c->kr.r,       c->kr.b,        c->kr.d,
                  c->kr.tmp,     c->d_lam_bar_m, c->d_ltil_m,  c->d_u_m,      c->d_corr_m,    c->d_src64m,
                  c->d_mu_last,  c->d_fsrc,     c->d_ptil,     c->d_sigf,     c->d_fmp64,     c->d_slot_of,
                  c->d_slot_body, c->d_ssrc_off, c->d_nbr_slot, c->d_cl_start, c->d_ccent,    c->d_crad64,
                  c->d_tperm,    c->d_work};
  for (void* p : ptrs)
    if (p) dev_free(c, p);
  for (void* p : {(void*)c->d_cell_child_off, (void*)c->d_cell_child, (void*)c->d_cell_by_height, (void*)c->d_cell_c,
                  (void*)c->d_wcent, (void*)c->d_wstart, (void*)c->d_cellraw, (void*)c->d_cellrec, (void*)c->d_ring64, (void*)c->d_ring32})
    if (p) dev_free(c, p);
  for (const FmmLists& L : c->fl)
    for (void* p : {(void*)L.d_m2l_off, (void*)L.d_m2l, (void*)L.d_near_off, (void*)L.d_near})
      if (p) dev_free(c, p);
  for (const PairSet& ps : c->ps)
    for (void* p : {(void*)ps.G, (void*)ps.Yf, (void*)ps.KKf, (void*)ps.pgeo, (void*)ps.nf, (void*)ps.d_goff,
                    (void*)ps.d_yoff})
      if (p) dev_free(c, p);
  for (void* p : {(void*)c->kr.H, (void*)c->kr.cs, (void*)c->kr.sn, (void*)c->kr.g, (void*)c->kr.y, (void*)c->kr.ctl,
                  (void*)c->kr.rec})
    if (p) dev_free(c, p);
  if (c->kr.hhost) (void)hipHostFree(c->kr.hhost);
  if (c->kr.hrec) (void)hipHostFree(c->kr.hrec);
  for (hipEvent_t e : c->kr.ev)
    if (e) (void)hipEventDestroy(e);
  for (void* p : c->class_bufs)
    if (p) dev_free(c, p);
  if (c->blas) rocblas_destroy_handle(c->blas);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// Host-only checks and contact search (no HIP call, so argument and geometry errors
// are reported without touching the device).
Status validate_host(mfs_ctx* c, const double* centers, const double* radii, const int32_t* n_src,
                     const int32_t* n_col, const double* r_src) {
  const int P = c->P;
  c->centers.assign(centers, centers + 2 * P);
  c->radii.assign(radii, radii + P);
  c->n_src.assign(n_src, n_src + P);
  c->n_col.assign(n_col, n_col + P);
  c->r_src.resize(P);
  for (int i = 0; i < P; ++i) {
    if (!(radii[i] > 0.0) || !std::isfinite(radii[i]) || !std::isfinite(centers[2 * i]) ||
        !std::isfinite(centers[2 * i + 1]))
      return Status{MFS_ERR_ARG, "body " + std::to_string(i) + ": invalid centre or radius"};
    if (n_src[i] < 1 || n_col[i] <= n_src[i] || n_col[i] > kMaxCol)
      return Status{MFS_ERR_ARG, "body " + std::to_string(i) + ": need 1 <= n_src < n_col <= 512"};
    double rs = r_src[i] > 0.0 ? r_src[i] : ring_rule(n_src[i], c->prm.eps_ring);
    if (!(rs > 0.0 && rs < 1.0)) return Status{MFS_ERR_ARG, "body " + std::to_string(i) + ": source ring radius not in (0, 1)"};
    c->r_src[i] = rs;
  }
  int bi = -1, bk = -1;
  double bg = 0;
  if (!find_contacts(P, centers, radii, c->prm.delta_c, c->pairs, &bi, &bk, &bg))
    return Status{MFS_ERR_GEOMETRY, "disks " + std::to_string(bi) + " and " + std::to_string(bk) +
                                        " overlap or touch (gap " + std::to_string(bg) + ")"};
  return Status{};
}

// Order of the disks for the kernel sums ("slots") and the clusters of the two-level FP64 sum
// at arbitrary points (flow evaluation).  Disks are sorted along a
// Morton curve over their centres (16 bits per axis, ties by index); the curve is cut into
// quadtree cells holding about 16..64 disks, and each cell into runs of at most
// kClMaxBodies disks and kClMaxSources sources: these runs are the clusters.  A cluster's
// centre is the mean of its disks' centres.  Its radius R, the one the far test uses (far:
// beyond 4 R), is the largest distance from there to a source ring (|c_b - C| + rho_b), raised
// where needed to (D + R) / 4 with D = 3 max(a) + delta_c: a node x of disk i lies within D of
// every contact partner k of i (|x - c_k| <= a_i + a_i + a_k + delta_c), so a cluster holding
// i or one of its partners is never far from x, whatever the cluster's size.
void build_clusters(mfs_ctx* c) {
  const int P = c->P;
  double x0 = c->centers[0], x1 = x0, y0 = c->centers[1], y1 = y0;
  for (int i = 1; i < P; ++i) {
    x0 = std::min(x0, c->centers[2 * i]);
    x1 = std::max(x1, c->centers[2 * i]);
    y0 = std::min(y0, c->centers[2 * i + 1]);
    y1 = std::max(y1, c->centers[2 * i + 1]);
  }
  const double span = std::max(std::max(x1 - x0, y1 - y0), 1e-300);
  auto spread = [](uint32_t v) {   // bit k of v -> bit 2k
    uint64_t x = v & 0xffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
  };
  std::vector<uint64_t> code(P);
  for (int i = 0; i < P; ++i) {
    const uint32_t qx = (uint32_t)std::min(65535.0, std::floor((c->centers[2 * i] - x0) / span * 65535.0));
    const uint32_t qy = (uint32_t)std::min(65535.0, std::floor((c->centers[2 * i + 1] - y0) / span * 65535.0));
    code[i] = spread(qx) | (spread(qy) << 1);
  }
  c->slot_body.resize(P);
  for (int i = 0; i < P; ++i) c->slot_body[i] = i;
  std::stable_sort(c->slot_body.begin(), c->slot_body.end(), [&](int a, int b) { return code[a] < code[b]; });
  c->slot_of.assign(P, 0);
  for (int s = 0; s < P; ++s) c->slot_of[c->slot_body[s]] = s;
  // quadtree level whose cells hold at least 16 disks on average: 4^(16 - L) cells <= P / 16
  int depth = 0;
  while (depth < 16 && (int64_t)1 << (2 * (depth + 1)) <= std::max(1, P / 16)) ++depth;
  const int shift = 2 * (16 - depth);
  c->cl_start.assign(1, 0);
  int nb = 0, ns = 0;
  for (int s = 0; s < P; ++s) {
    const int b = c->slot_body[s];
    const bool new_cell = s > 0 && (code[b] >> shift) != (code[c->slot_body[s - 1]] >> shift);
    if (s > 0 && (new_cell || nb == kClMaxBodies || ns + c->n_src[b] > kClMaxSources)) {
      c->cl_start.push_back(s);
      nb = ns = 0;
    }
    ++nb;
    ns += c->n_src[b];
  }
  c->cl_start.push_back(P);
  c->ncl = (int)c->cl_start.size() - 1;
  double amax = 0;
  for (int i = 0; i < P; ++i) amax = std::max(amax, c->radii[i]);
  const double reach = 3.0 * amax + c->prm.delta_c;
  c->cl_centre.assign(2 * c->ncl, 0.0);
  c->cl_radius.assign(c->ncl, 0.0);
  for (int q = 0; q < c->ncl; ++q) {
    double cx = 0, cy = 0;
    for (int s = c->cl_start[q]; s < c->cl_start[q + 1]; ++s) {
      cx += c->centers[2 * c->slot_body[s]];
      cy += c->centers[2 * c->slot_body[s] + 1];
    }
    const int m = c->cl_start[q + 1] - c->cl_start[q];
    cx /= m;
    cy /= m;
    double r = 0;
    for (int s = c->cl_start[q]; s < c->cl_start[q + 1]; ++s) {
      const int b = c->slot_body[s];
      const double* yr = c->h_Yr[c->cls[b]].data();
      r = std::max(r, std::hypot(c->centers[2 * b] - cx, c->centers[2 * b + 1] - cy) + std::hypot(yr[0], yr[1]));
    }
    c->cl_centre[2 * q] = cx;
    c->cl_centre[2 * q + 1] = cy;
    c->cl_radius[q] = std::max(r, (reach + r) / 4.0);
  }
}

Status build(mfs_ctx* c, const double* centers, const double* radii, const int32_t* n_src, const int32_t* n_col,
             const double* r_src) {
  (void)radii;
  (void)r_src;
  const int P = c->P;
  c->src_off.assign(P + 1, 0);
  c->col_off.assign(P + 1, 0);
  for (int i = 0; i < P; ++i) {
    c->src_off[i + 1] = c->src_off[i] + n_src[i];
    c->col_off[i + 1] = c->col_off[i] + n_col[i];
  }
  c->Ns = c->src_off[P];
  c->Nt = c->col_off[P];
  const int C = (int)(c->pairs.size() / 2);
  c->xoff.assign(C + 1, 0);
  c->aoff.assign(C + 1, 0);
  c->coff.assign(C + 1, 0);
  std::vector<std::vector<int32_t>> bl(P);
  for (int p = 0; p < C; ++p) {
    const int i = c->pairs[2 * p], k = c->pairs[2 * p + 1];
    const int64_t nx = 2 * (int64_t)(n_src[i] + n_src[k]);
    c->xoff[p + 1] = c->xoff[p] + nx;
    c->aoff[p + 1] = c->aoff[p] + nx * nx;
    c->coff[p + 1] = c->coff[p] + 2 * (int64_t)(n_col[i] + n_col[k]);
    bl[i].push_back(2 * p);
    bl[k].push_back(2 * p + 1);
  }
  c->bp_off.assign(P + 1, 0);
  c->bp_list.clear();
  c->nbr_off.assign(P + 1, 0);
  c->nbr_list.clear();
  for (int i = 0; i < P; ++i) {
    c->bp_list.insert(c->bp_list.end(), bl[i].begin(), bl[i].end());
    c->bp_off[i + 1] = (int32_t)c->bp_list.size();
    std::vector<int32_t> nb;
    for (int32_t e : bl[i]) nb.push_back(c->pairs[2 * (e >> 1) + 1 - (e & 1)]);
    std::sort(nb.begin(), nb.end());
    c->nbr_list.insert(c->nbr_list.end(), nb.begin(), nb.end());
    c->nbr_off[i + 1] = (int32_t)c->nbr_list.size();
  }
  Status st = onebody_factors(c);
  if (st.code) return st;
  build_clusters(c);
  // slot-ordered source offsets and partner lists (kernel sums)
  std::vector<int32_t> ssrc_off(P + 1, 0), nbr_slot(c->nbr_list.size());
  for (int s = 0; s < P; ++s) ssrc_off[s + 1] = ssrc_off[s] + n_src[c->slot_body[s]];
  for (int i = 0; i < P; ++i) {
    for (int e = c->nbr_off[i]; e < c->nbr_off[i + 1]; ++e) nbr_slot[e] = c->slot_of[c->nbr_list[e]];
    std::sort(nbr_slot.begin() + c->nbr_off[i], nbr_slot.begin() + c->nbr_off[i + 1]);
  }
  // exact evaluation counts of one kernel sum: all sources, and without own disk and partners
  c->evals_all = c->Ns * c->Nt;
  c->evals_skip = 0;
  for (int i = 0; i < P; ++i) {
    int64_t skipped = n_src[i];
    for (int e = c->nbr_off[i]; e < c->nbr_off[i + 1]; ++e) skipped += n_src[c->nbr_list[e]];
    c->evals_skip += (int64_t)n_col[i] * (c->Ns - skipped);
  }
  // absolute coordinates
  std::vector<double> Y(2 * c->Ns), X(2 * c->Nt);
  std::vector<int32_t> tb(c->Nt);
  for (int i = 0; i < P; ++i) {
    const int k = c->cls[i];
    const std::vector<double>& yr = c->h_Yr[k];
    const std::vector<double>& xr = c->h_Xr[k];
    for (int j = 0; j < n_src[i]; ++j) {
      Y[2 * (c->src_off[i] + j)] = centers[2 * i] + yr[2 * j];
      Y[2 * (c->src_off[i] + j) + 1] = centers[2 * i + 1] + yr[2 * j + 1];
    }
    for (int q = 0; q < n_col[i]; ++q) {
      const int64_t t = c->col_off[i] + q;
      X[2 * t] = centers[2 * i] + xr[2 * q];
      X[2 * t + 1] = centers[2 * i + 1] + xr[2 * q + 1];
      tb[t] = i;
    }
  }
  hipStream_t s = c->stream;
  if ((st = upload(c, &c->d_src_off, c->src_off, s)).code) return st;
  if ((st = upload(c, &c->d_col_off, c->col_off, s)).code) return st;
  if ((st = upload(c, &c->d_cls, c->cls, s)).code) return st;
  if ((st = upload(c, &c->d_tgt_body, tb, s)).code) return st;
  if ((st = upload(c, &c->d_pairs, c->pairs, s)).code) return st;
  if ((st = upload(c, &c->d_bp_off, c->bp_off, s)).code) return st;
  if ((st = upload(c, &c->d_bp_list, c->bp_list, s)).code) return st;
  if ((st = upload(c, &c->d_nbr_off, c->nbr_off, s)).code) return st;
  if ((st = upload(c, &c->d_nbr_list, c->nbr_list, s)).code) return st;
  if ((st = upload(c, &c->d_xoff, c->xoff, s)).code) return st;
  if ((st = upload(c, &c->d_aoff, c->aoff, s)).code) return st;
  if ((st = upload(c, &c->d_coff, c->coff, s)).code) return st;
  if ((st = upload(c, &c->d_centers, c->centers, s)).code) return st;
  if ((st = upload(c, &c->d_Y, Y, s)).code) return st;
  if ((st = upload(c, &c->d_X, X, s)).code) return st;
  if ((st = upload(c, &c->d_slot_of, c->slot_of, s)).code) return st;
  if ((st = upload(c, &c->d_slot_body, c->slot_body, s)).code) return st;
  if ((st = upload(c, &c->d_ssrc_off, ssrc_off, s)).code) return st;
  if ((st = upload(c, &c->d_nbr_slot, nbr_slot, s)).code) return st;
  if ((st = upload(c, &c->d_cl_start, c->cl_start, s)).code) return st;
  if ((st = upload(c, &c->d_ccent, c->cl_centre, s)).code) return st;
  if ((st = upload(c, &c->d_crad64, c->cl_radius, s)).code) return st;
  {
    // the kernel sums visit the targets disk by disk in slot order, so that a workgroup's
    // targets (and a wave's) lie close together and far clusters are far for all of them
    std::vector<int32_t> tperm;
    tperm.reserve(c->Nt);
    for (int sl = 0; sl < P; ++sl) {
      const int b = c->slot_body[sl];
      for (int q = c->col_off[b]; q < c->col_off[b + 1]; ++q) tperm.push_back(q);
    }
    if ((st = upload(c, &c->d_tperm, tperm, s)).code) return st;
  }
  if ((st = build_fmm(c)).code) return st;
  if ((st = dalloc(c, &c->d_work, 8)).code) return st;
  launch_zero_work(c);
  if ((st = dalloc(c, &c->d_lam_bar, 2 * c->Ns)).code) return st;
  if ((st = dalloc(c, &c->d_ltil, c->xoff[C])).code) return st;
  if ((st = dalloc(c, &c->d_u, 2 * c->Nt)).code) return st;
  if ((st = dalloc(c, &c->d_corr, c->coff[C])).code) return st;
  if ((st = dalloc(c, &c->d_epair, 6 * (size_t)C)).code) return st;
  if ((st = dalloc(c, &c->d_out3, 3 * (size_t)P)).code) return st;
  if ((st = dalloc(c, &c->d_given, 3 * (size_t)P)).code) return st;
  if ((st = dalloc(c, &c->d_src64, c->Ns)).code) return st;
  MFS_HIP(hipStreamSynchronize(s));
  return Status{};
}

Status check_kernel_sum(mfs_ctx* c, bool launched) {
  if (!launched) return Status{MFS_ERR_OOM, "kernel-sum split buffer does not fit"};
  MFS_HIP(hipGetLastError());
  return Status{};
}

}  // namespace

namespace mfs {

Status apply_T(mfs_ctx* c, int prob, bool mixed, const double* mu, double* u, const SplitBuf* sb) {
  const bool wp = c->pairs.size() > 0;
  launch_onebody_apply(c, prob, mu, c->d_lam_bar);
  if (wp) launch_pair_A(c, prob, c->d_lam_bar, c->d_ltil);
  FmmRec fr = fmm_records(c, 0);
  if (sb && !fmm_records_in(c, sb, &fr)) return Status{MFS_ERR_ARG, "the caller's buffer is too small"};
  launch_gather_project(c, prob, c->d_lam_bar, c->d_ltil, wp, mixed, !mixed, &fr);
  const bool ks = launch_kernel_sum(c, mixed, 2, c->d_u, 1.0 / (4.0 * kPiD * c->prm.mu), &fr);
  c->cnt_pair_evals += c->evals_skip;
  if (mixed)
    ++c->cnt_mv32;
  else
    ++c->cnt_mv64;
  if (wp) launch_pair_field(c, prob, c->d_ltil, c->d_corr);
  launch_finish(c, c->d_u, mu, c->d_corr, u, wp);
  return check_kernel_sum(c, ks);
}

// Stacked buffers for R right-hand sides.
Status ensure_stacked(mfs_ctx* c, int R) {
  if (c->rhs_cap >= R) return Status{};
  for (void* p : {(void*)c->d_lam_bar_m, (void*)c->d_ltil_m, (void*)c->d_u_m, (void*)c->d_corr_m, (void*)c->d_src64m})
    if (p) dev_free(c, p);
  c->d_lam_bar_m = c->d_ltil_m = c->d_u_m = c->d_corr_m = nullptr;
  c->d_src64m = nullptr;
  c->rhs_cap = 0;
  const int C = (int)(c->pairs.size() / 2);
  Status st;
  if ((st = dalloc(c, &c->d_lam_bar_m, (size_t)R * 2 * c->Ns)).code) return st;
  if ((st = dalloc(c, &c->d_ltil_m, (size_t)R * c->xoff[C])).code) return st;
  if ((st = dalloc(c, &c->d_u_m, (size_t)R * 2 * c->Nt)).code) return st;
  if ((st = dalloc(c, &c->d_corr_m, (size_t)R * c->coff[C])).code) return st;
  if ((st = dalloc(c, &c->d_src64m, (size_t)R * c->Ns)).code) return st;
  c->rhs_cap = R;
  return Status{};
}

Status apply_T_rhs(mfs_ctx* c, int prob, bool mixed, int R, const double* mu, double* u) {
  const int64_t n = 2 * c->Nt;
  int max_src = 0;
  for (int i = 0; i < c->P; ++i) max_src = std::max(max_src, c->n_src[i]);
  // stacked kernels take 8, 4 or 2 vectors; a remainder of one goes through apply_T
  int r0 = 0;
  while (r0 < R) {
    const int left = R - r0;
    const int Rc = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    if (Rc == 1 || max_src > 256) {
      Status st = apply_T(c, prob, mixed, mu + r0 * n, u + r0 * n);
      if (st.code) return st;
      r0 += 1;
      continue;
    }
    Status st = ensure_stacked(c, 8);
    if (st.code) return st;
    if ((st = ensure_fmm_records(c, 8)).code) return st;
    const bool wp = c->pairs.size() > 0;
    const int C = (int)(c->pairs.size() / 2);
    const int64_t ns2 = 2 * c->Ns, nx = c->xoff[C], nc = c->coff[C];
    for (int r = 0; r < Rc; ++r) launch_onebody_apply(c, prob, mu + (r0 + r) * n, c->d_lam_bar_m + r * ns2);
    if (wp && !launch_pair_A_rhs(c, prob, Rc, c->d_lam_bar_m, ns2, c->d_ltil_m, nx))
      for (int r = 0; r < Rc; ++r) launch_pair_A(c, prob, c->d_lam_bar_m + r * ns2, c->d_ltil_m + r * nx);
    for (int r = 0; r < Rc; ++r)
      launch_gather_project_to(c, prob, c->d_lam_bar_m + r * ns2, c->d_ltil_m + r * nx, wp, c->d_src64m + r * c->Ns);
    for (int r = 0; r < Rc; ++r) launch_fmm_records(c, prob, c->d_src64m + r * c->Ns, fmm_records(c, r), mixed);
    const bool ks = launch_kernel_sum_rhs(c, mixed, 2, Rc, c->d_u_m, 1.0 / (4.0 * kPiD * c->prm.mu));
    if ((st = check_kernel_sum(c, ks)).code) return st;
    c->cnt_pair_evals += (int64_t)Rc * c->evals_skip;
    if (mixed)
      c->cnt_mv32 += Rc;
    else
      c->cnt_mv64 += Rc;
    for (int r = 0; r < Rc; ++r) {
      if (wp) launch_pair_field(c, prob, c->d_ltil_m + r * nx, c->d_corr_m + r * nc);
      launch_finish(c, c->d_u_m + r * n, mu + (r0 + r) * n, c->d_corr_m + r * nc, u + (r0 + r) * n, wp);
    }
    MFS_HIP(hipGetLastError());
    r0 += Rc;
  }
  return Status{};
}

}  // namespace mfs

// ---------------------------------------------------------------------------
extern "C" {

void mfs_default_params(mfs_params* p) {
  if (!p) return;
  p->mu = 1.0;
  p->delta_c = 0.2;
  p->eps_trunc = 1e-14;
  p->eps_trunc_fine = 1e-11;
  p->eps_ring = 1e-12;
  p->n_fp = 150;
  p->n_ell = 80;
  p->m_p = 200;
  p->a_ell = 5;
  p->gamma = 0.3;
  p->a_f = 1.2;
  p->mobius_r = 0.6;
}

mfs_status mfs_setup(mfs_ctx** out, int32_t P, const double* centers, const double* radii, const int32_t* n_src,
                     const int32_t* n_col, const double* r_src, const mfs_params* prm, void* stream) {
  return mfs_setup_ex(out, P, centers, radii, n_src, n_col, r_src, prm, stream, nullptr);
}

mfs_status mfs_setup_ex(mfs_ctx** out, int32_t P, const double* centers, const double* radii,
                        const int32_t* n_src, const int32_t* n_col, const double* r_src, const mfs_params* prm,
                        void* stream, const mfs_allocator* allocator) {
  if (!out) return fail(nullptr, Status{MFS_ERR_ARG, "ctx pointer is NULL"});
  *out = nullptr;
  if (P < 1 || !centers || !radii || !n_src || !n_col || !r_src)
    return fail(nullptr, Status{MFS_ERR_ARG, "P < 1 or NULL geometry array"});
  if (allocator && (!allocator->alloc || !allocator->free))
    return fail(nullptr, Status{MFS_ERR_ARG, "allocator without alloc or free callback"});
  mfs_params p;
  if (prm)
    p = *prm;
  else
    mfs_default_params(&p);
  if (!(p.mu > 0) || !(p.delta_c >= 0) || !(p.eps_trunc > 0 && p.eps_trunc < 1) ||
      !(p.eps_trunc_fine > 0 && p.eps_trunc_fine < 1) || !(p.eps_ring > 0 && p.eps_ring < 1) || p.n_fp < 4 ||
      p.n_ell < 1 || p.m_p < 8 || p.a_ell < 1 || !(p.gamma > 0 && p.gamma < 1) || !(p.a_f >= 1) ||
      !(p.mobius_r >= 0 && p.mobius_r < 1) || !(p.delta_c < 2 * (std::sqrt(3.0) - 1.0)) ||
      ring_rule(p.n_fp, p.eps_ring) <= 0)
    return fail(nullptr, Status{MFS_ERR_ARG, "invalid method parameters"});
  mfs_ctx* c = new (std::nothrow) mfs_ctx();
  if (!c) return fail(nullptr, Status{MFS_ERR_OOM, "host allocation failed"});
  c->P = P;
  c->prm = p;
  if (allocator) c->alloc = *allocator;
  {
    Status st = validate_host(c, centers, radii, n_src, n_col, r_src);
    if (st.code) {
      delete c;
      return fail(nullptr, st);
    }
  }
  c->stream = (hipStream_t)stream;   // NULL: the null (default) stream
  c->own_stream = false;
  if (rocblas_create_handle(&c->blas) != rocblas_status_success ||
      rocblas_set_stream(c->blas, c->stream) != rocblas_status_success) {
    free_all(c);
    delete c;
    return fail(nullptr, Status{MFS_ERR_DEVICE, "rocBLAS handle creation failed"});
  }
  Status st = build(c, centers, radii, n_src, n_col, r_src);
  if (!st.code) st = scratch_for_current_device(&c->scratch);
  if (st.code) {
    free_all(c);
    delete c;
    return fail(nullptr, st);
  }
  *out = c;
  return MFS_OK;
}

mfs_status mfs_precompute_pairs(mfs_ctx* c, mfs_problem prob, int64_t* n_pairs_out) {
  if (!c) return fail(nullptr, Status{MFS_ERR_ARG, "ctx is NULL"});
  if (prob != MFS_RESISTANCE && prob != MFS_MOBILITY) return fail(c, Status{MFS_ERR_ARG, "unknown problem"});
  Status st = precompute_pairs(c, prob);
  if (st.code) return fail(c, st);
  if (n_pairs_out) *n_pairs_out = (int64_t)(c->pairs.size() / 2);
  return ok(c);
}

mfs_status mfs_get_pairs(const mfs_ctx* c, int64_t* n_pairs, int32_t* pairs) {
  if (!c || !n_pairs) return MFS_ERR_ARG;
  *n_pairs = (int64_t)(c->pairs.size() / 2);
  if (pairs) std::memcpy(pairs, c->pairs.data(), sizeof(int32_t) * c->pairs.size());
  return MFS_OK;
}

mfs_status mfs_get_clusters(const mfs_ctx* c, int32_t* n_clusters, int32_t* slot_body, int32_t* cl_start,
                            double* centre, double* radius) {
  if (!c || !n_clusters) return MFS_ERR_ARG;
  *n_clusters = c->ncl;
  if (slot_body) std::memcpy(slot_body, c->slot_body.data(), sizeof(int32_t) * c->slot_body.size());
  if (cl_start) std::memcpy(cl_start, c->cl_start.data(), sizeof(int32_t) * c->cl_start.size());
  if (centre) std::memcpy(centre, c->cl_centre.data(), sizeof(double) * c->cl_centre.size());
  if (radius) std::memcpy(radius, c->cl_radius.data(), sizeof(double) * c->cl_radius.size());
  return MFS_OK;
}

mfs_status mfs_get_fmm(const mfs_ctx* c, mfs_problem prob, mfs_precision prec, int64_t* sizes, int32_t* cell_lo,
                       int32_t* cell_hi, double* cell_c, double* cell_r, int32_t* wave_start, double* wave_c,
                       int32_t* m2l_off, int32_t* m2l, int32_t* near_off, int32_t* near, double* tier_d2) {
  if (!c || !sizes || (prob != MFS_RESISTANCE && prob != MFS_MOBILITY) || (prec != MFS_FP64 && prec != MFS_MIXED))
    return MFS_ERR_ARG;
  const FmmLists& L = c->fl[prec == MFS_MIXED ? 1 : 0];
  sizes[0] = c->ncell;
  sizes[1] = c->nwave;
  sizes[2] = (int64_t)L.m2l.size();
  sizes[3] = (int64_t)L.near.size();
  auto cp = [](void* dst, const void* src, size_t bytes) {
    if (dst && bytes) std::memcpy(dst, src, bytes);
  };
  cp(cell_lo, c->cell_lo.data(), sizeof(int32_t) * c->cell_lo.size());
  cp(cell_hi, c->cell_hi.data(), sizeof(int32_t) * c->cell_hi.size());
  cp(cell_c, c->cell_c.data(), sizeof(double) * c->cell_c.size());
  cp(cell_r, c->cell_r.data(), sizeof(double) * c->cell_r.size());
  cp(wave_start, c->h_wstart.data(), sizeof(int32_t) * c->h_wstart.size());
  cp(wave_c, c->h_wcent.data(), sizeof(double) * c->h_wcent.size());
  cp(m2l_off, L.m2l_off.data(), sizeof(int32_t) * L.m2l_off.size());
  cp(m2l, L.m2l.data(), sizeof(int32_t) * L.m2l.size());
  cp(near_off, L.near_off.data(), sizeof(int32_t) * L.near_off.size());
  cp(near, L.near.data(), sizeof(int32_t) * L.near.size());
  if (tier_d2) {
    const ClassTab& ct = c->ct[prob];
    for (int s = 0; s < c->P; ++s) {
      const int k = c->cls[c->slot_body[s]];
      for (int t = 0; t < kRingTiers; ++t)
        tier_d2[kRingTiers * s + t] = prec == MFS_MIXED ? ct.tier32[k][t] : ct.tier64[k][t];
    }
  }
  return MFS_OK;
}

mfs_status mfs_set_pair_matrices(mfs_ctx* c, mfs_problem prob, const double* A, const double* E) {
  if (!c) return fail(nullptr, Status{MFS_ERR_ARG, "ctx is NULL"});
  if ((prob != MFS_RESISTANCE && prob != MFS_MOBILITY) || !A || !E)
    return fail(c, Status{MFS_ERR_ARG, "unknown problem or NULL matrix"});
  const int C = (int)(c->pairs.size() / 2);
  PairSet& ps = c->ps[prob];
  if (!ps.A) {
    Status st = dalloc(c, &ps.A, c->aoff[C]);
    if (!st.code) st = dalloc(c, &ps.E, 6 * c->xoff[C]);
    if (st.code) return fail(c, st);
  }
  std::vector<double> Ac(c->aoff[C]), Ec(6 * c->xoff[C]);
  for (int p = 0; p < C; ++p) {
    const int64_t n = c->xoff[p + 1] - c->xoff[p];
    const double* a = A + c->aoff[p];
    double* ac = Ac.data() + c->aoff[p];
    for (int64_t r = 0; r < n; ++r)
      for (int64_t q = 0; q < n; ++q) ac[q * n + r] = a[r * n + q];
    const double* e = E + 6 * c->xoff[p];
    double* ec = Ec.data() + 6 * c->xoff[p];
    for (int r = 0; r < 6; ++r)
      for (int64_t q = 0; q < n; ++q) ec[q * 6 + r] = e[r * n + q];
  }
  if (!finite_all(Ac.data(), Ac.size()) || !finite_all(Ec.data(), Ec.size()))
    return fail(c, Status{MFS_ERR_NUMERIC, "non-finite pair matrix"});
  if (hipMemcpy(ps.A, Ac.data(), sizeof(double) * Ac.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(ps.E, Ec.data(), sizeof(double) * Ec.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail(c, Status{MFS_ERR_DEVICE, "hipMemcpy of pair matrices failed"});
  ps.ready = true;
  ps.fine = false;   // imported matrices come without fine factors
  return ok(c);
}

mfs_status mfs_get_pair_matrices(const mfs_ctx* cc, mfs_problem prob, double* A, double* E) {
  mfs_ctx* c = const_cast<mfs_ctx*>(cc);
  if (!c) return MFS_ERR_ARG;
  if ((prob != MFS_RESISTANCE && prob != MFS_MOBILITY) || !A || !E) return fail(c, Status{MFS_ERR_ARG, "bad argument"});
  const PairSet& ps = c->ps[prob];
  if (!ps.ready) return fail(c, Status{MFS_ERR_STATE, "pair matrices not computed for this problem"});
  const int C = (int)(c->pairs.size() / 2);
  std::vector<double> Ac(c->aoff[C]), Ec(6 * c->xoff[C]);
  if (hipStreamSynchronize(c->stream) != hipSuccess ||
      hipMemcpy(Ac.data(), ps.A, sizeof(double) * Ac.size(), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(Ec.data(), ps.E, sizeof(double) * Ec.size(), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, Status{MFS_ERR_DEVICE, "hipMemcpy of pair matrices failed"});
  for (int p = 0; p < C; ++p) {
    const int64_t n = c->xoff[p + 1] - c->xoff[p];
    const double* ac = Ac.data() + c->aoff[p];
    double* a = A + c->aoff[p];
    for (int64_t r = 0; r < n; ++r)
      for (int64_t q = 0; q < n; ++q) a[r * n + q] = ac[q * n + r];
    const double* ec = Ec.data() + 6 * c->xoff[p];
    double* e = E + 6 * c->xoff[p];
    for (int r = 0; r < 6; ++r)
      for (int64_t q = 0; q < n; ++q) e[r * n + q] = ec[q * 6 + r];
  }
  return ok(c);
}

mfs_status mfs_apply(mfs_ctx* c, mfs_problem prob, mfs_precision prec, int32_t n_rhs, const double* mu_in,
                     double* u_out) {
  if (!c) return fail(nullptr, Status{MFS_ERR_ARG, "ctx is NULL"});
  if ((prob != MFS_RESISTANCE && prob != MFS_MOBILITY) || (prec != MFS_FP64 && prec != MFS_MIXED) || n_rhs < 1 ||
      !mu_in || !u_out)
    return fail(c, Status{MFS_ERR_ARG, "bad argument"});
  if (!c->ps[prob].ready && !c->pairs.empty())
    return fail(c, Status{MFS_ERR_STATE, "mfs_precompute_pairs has not run for this problem"});
  Status st = apply_T_rhs(c, prob, prec == MFS_MIXED, n_rhs, mu_in, u_out);
  if (st.code) return fail(c, st);
  return ok(c);
}

mfs_status mfs_apply_noalloc(mfs_ctx* c, mfs_problem prob, mfs_precision prec, const double* mu_in,
                             double* u_out) {
  if (!c) return fail(nullptr, Status{MFS_ERR_ARG, "ctx is NULL"});
  if ((prob != MFS_RESISTANCE && prob != MFS_MOBILITY) || (prec != MFS_FP64 && prec != MFS_MIXED) || !mu_in ||
      !u_out)
    return fail(c, Status{MFS_ERR_ARG, "bad argument"});
  if (!c->ps[prob].ready && !c->pairs.empty())
    return fail(c, Status{MFS_ERR_STATE, "mfs_precompute_pairs has not run for this problem"});
  if (!c->scratch) return fail(c, Status{MFS_ERR_STATE, "no scratch array resolved for this context's device"});
  const bool mixed = prec == MFS_MIXED;
  const int64_t need = fmm_record_doubles(c);
  if (need > kScratchDoubles)
    return fail(c, Status{MFS_ERR_ARG, "the kernel sum's expansion records (" + std::to_string(need * 8) +
                                           " bytes) exceed the no-allocation scratch array (" +
                                           std::to_string(kScratchDoubles * 8) + " bytes)"});
  const SplitBuf sb{c->scratch, kScratchDoubles};
  Status st = apply_T(c, prob, mixed, mu_in, u_out, &sb);
  if (st.code) return fail(c, st);
  return ok(c);
}

mfs_status mfs_kernel_sum_work(mfs_ctx* c, int64_t* work, int32_t reset) {
  if (!c) return fail(nullptr, Status{MFS_ERR_ARG, "ctx is NULL"});
  if (!work) return fail(c, Status{MFS_ERR_ARG, "work is NULL"});
  unsigned long long h[5] = {0, 0, 0, 0, 0};
  if (hipMemcpyAsync(h, c->d_work, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(c, Status{MFS_ERR_DEVICE, "reading the work counters failed"});
  for (int e = 0; e < 5; ++e) work[e] = (int64_t)h[e];
  if (reset) launch_zero_work(c);
  return ok(c);
}

mfs_status mfs_kernel_sum(mfs_ctx* c, mfs_precision prec, const double* sigma, double* u, int32_t skip) {
  if (!c) return fail(nullptr, Status{MFS_ERR_ARG, "ctx is NULL"});
  if ((prec != MFS_FP64 && prec != MFS_MIXED) || !sigma || !u || skip < 0 || skip > 2)
    return fail(c, Status{MFS_ERR_ARG, "bad argument"});
  const bool mixed = prec == MFS_MIXED;
  launch_gather_project(c, MFS_RESISTANCE, sigma, nullptr, false, mixed, !mixed);
  const bool ks = launch_kernel_sum(c, mixed, skip, u, 1.0 / (4.0 * kPiD * c->prm.mu));
  Status st = check_kernel_sum(c, ks);
  if (st.code) return fail(c, st);
  return ok(c);
}

mfs_status mfs_time_kernel_sum(mfs_ctx* c, mfs_precision prec, const double* sigma, double* u, int32_t skip,
                               int32_t reps, double* ms_records, double* ms_sum) {
  if (!c) return fail(nullptr, Status{MFS_ERR_ARG, "ctx is NULL"});
  if ((prec != MFS_FP64 && prec != MFS_MIXED) || !sigma || !u || skip < 0 || skip > 2 || reps < 1 || !ms_records ||
      !ms_sum)
    return fail(c, Status{MFS_ERR_ARG, "bad argument"});
  const bool mixed = prec == MFS_MIXED;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  for (hipEvent_t& e : ev)
    if (hipEventCreate(&e) != hipSuccess) return fail(c, Status{MFS_ERR_DEVICE, "hipEventCreate"});
  const FmmRec fr = fmm_records(c, 0);
  (void)hipEventRecord(ev[0], c->stream);
  launch_gather_project(c, MFS_RESISTANCE, sigma, nullptr, false, mixed, !mixed, &fr);
  (void)hipEventRecord(ev[1], c->stream);
  for (int r = 0; r < reps; ++r) launch_ksum_fmm(c, mixed, skip, c->d_src64, fr, u, 1.0 / (4.0 * kPiD * c->prm.mu));
  (void)hipEventRecord(ev[2], c->stream);
  Status st;
  if (hipGetLastError() != hipSuccess || hipEventSynchronize(ev[2]) != hipSuccess)
    st = Status{MFS_ERR_DEVICE, "kernel-sum launch failed"};
  float a = 0.f, b = 0.f;
  if (!st.code && (hipEventElapsedTime(&a, ev[0], ev[1]) != hipSuccess || hipEventElapsedTime(&b, ev[1], ev[2]) != hipSuccess))
    st = Status{MFS_ERR_DEVICE, "hipEventElapsedTime"};
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  if (st.code) return fail(c, st);
  *ms_records = a;
  *ms_sum = b / reps;
  return ok(c);
}

mfs_status mfs_rhs(mfs_ctx* c, mfs_problem prob, const double* given, double* b) {
  if (!c) return fail(nullptr, Status{MFS_ERR_ARG, "ctx is NULL"});
  if ((prob != MFS_RESISTANCE && prob != MFS_MOBILITY) || !given || !b) return fail(c, Status{MFS_ERR_ARG, "bad argument"});
  if (!finite_all(given, 3 * (size_t)c->P)) return fail(c, Status{MFS_ERR_NUMERIC, "non-finite right-hand side"});
  if (hipMemcpyAsync(c->d_given, given, sizeof(double) * 3 * c->P, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return fail(c, Status{MFS_ERR_DEVICE, "hipMemcpy"});
  bool ks = true;
  if (prob == MFS_MOBILITY) {
    launch_rhs_mobility_sources(c, c->d_given);
    ks = launch_kernel_sum(c, false, 0, b, -1.0 / (4.0 * kPiD * c->prm.mu));
    c->cnt_pair_evals += c->evals_all;
  } else {
    launch_rhs_resistance(c, c->d_given, b);
  }
  Status st = check_kernel_sum(c, ks);
  if (!st.code && hipStreamSynchronize(c->stream) != hipSuccess) st = Status{MFS_ERR_DEVICE, "stream error"};
  if (st.code) return fail(c, st);
  return ok(c);
}

mfs_status mfs_post(mfs_ctx* c, mfs_problem prob, const double* mu, double* out) {
  if (!c) return fail(nullptr, Status{MFS_ERR_ARG, "ctx is NULL"});
  if ((prob != MFS_RESISTANCE && prob != MFS_MOBILITY) || !mu || !out) return fail(c, Status{MFS_ERR_ARG, "bad argument"});
  if (!c->ps[prob].ready && !c->pairs.empty())
    return fail(c, Status{MFS_ERR_STATE, "mfs_precompute_pairs has not run for this problem"});
  launch_onebody_apply(c, prob, mu, c->d_lam_bar);
  launch_post(c, prob, c->d_lam_bar, c->d_out3);
  if (hipMemcpyAsync(out, c->d_out3, sizeof(double) * 3 * c->P, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(c, Status{MFS_ERR_DEVICE, "post-processing failed"});
  return ok(c);
}

mfs_status mfs_get_sizes(const mfs_ctx* c, int32_t* P, int64_t* ns, int64_t* nt, int64_t* np) {
  if (!c) return MFS_ERR_ARG;
  if (P) *P = c->P;
  if (ns) *ns = c->Ns;
  if (nt) *nt = c->Nt;
  if (np) *np = (int64_t)(c->pairs.size() / 2);
  return MFS_OK;
}

mfs_status mfs_destroy(mfs_ctx* c) {
  if (!c) return MFS_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
  return MFS_OK;
}

const char* mfs_last_error(const mfs_ctx* c) {
  if (!c) return g_setup_err.c_str();
  return c->last.msg.c_str();
}

}  // extern "C"
