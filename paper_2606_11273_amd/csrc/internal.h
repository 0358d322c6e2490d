// Internal state and kernel entry points of the MFS library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mfs.h"
#include "geometry.h"

namespace mfs {

constexpr int kMaxClasses = 4;     // distinct (radius, n_src, n_col, r_src) disk classes
constexpr int kMaxCol = 512;       // n_col limit per disk
constexpr int kMp64Order = 18;     // order of the FP64 kernel sum's far-field expansion
constexpr int kMp64CoefPerDisk = 3 * kMp64Order + 3;   // FP64 complex coefficients per disk (last: rho^2)
// Two-level FP64 sum at arbitrary points (flow evaluation): disks in a space-filling-curve
// order ("slots"), grouped into clusters of at most kClMaxBodies consecutive slots; a cluster
// far from a target is summed through one expansion of order kCl64Order about its centre.  The
// hierarchical kernel sum's cells carry records of the same layout.
constexpr int kClMaxBodies = 16;
constexpr int kClMaxSources = 1024;                   // sources per cluster (one LDS tile)
constexpr int kCl64Order = 31;
// Local expansions (M2L / L2P) of the kernel sums: a cluster farther than kLocSep32 (R + r_b)
// (FP32 sum) or kLocSep64 (R + r_b) (FP64 sum), and than 4 R + r_b, from the centre of a
// workgroup's targets (r_b their radius) is translated into the workgroup's local expansion,
// order kLoc32 / kLoc64 in both source and target orders (theta <= 1/2 and 1/3: truncation
// below 5e-10 and 1e-15 of sum |sigma|)
constexpr int kLoc32 = 31;
constexpr int kLoc64 = 31;
constexpr double kLocSep32 = 2.0;
constexpr double kLocSep64 = 3.0;
static_assert(kLoc32 <= kCl64Order && kLoc64 <= kCl64Order && kLoc64 < 32, "local orders");
constexpr int kCl64CoefPerCluster = 4 * kCl64Order + 2;   // FP64 complex coefficients per cluster
// Hierarchical far field of the kernel sums over the context's own targets: a quadtree of
// cells over the disks in slot order (leaf c < P = the disk in slot c); per wave of kFmmT x 64
// consecutive targets of the visiting order, a list of cells translated into the wave's local
// expansion (M2L, a cell beyond kFmmSep (R + r_w) of the wave's centre, r_w the wave's radius,
// holding no target's disk or contact partner) and a list of near disks, each summed at the
// wave's targets from the disk's own ring expansion, at the lowest order of kTierOrder whose
// distance threshold every target meets, else directly.  Cell records: kCl64Order.
constexpr int kFmmT = 2;
constexpr int kRing64Order = 56;   // ring expansion orders of the near disks (FP64, FP32 sums)
constexpr int kRing32Order = 44;
constexpr int kRingTiers = 3;
// per disk: A_k/(2k), B_k/(2k) (k = 1..p), conj(A_k) (k = 0..p), conj(B_1), (rho^2, d3^2), (d1^2, d2^2),
// d_i the distances beyond which the tier-i order meets the truncation target, then the disk's
// FP64 centre and body index: (c_x, c_y), (body, 0) in the FP64 record; c_x, c_y and body as
// the bits of FP64 values in one float2 each in the FP32 record (padded to 16-byte units)
constexpr int kRing64Coef = 3 * kRing64Order + 6;
constexpr int kRing32Coef = 3 * kRing32Order + 8;
static_assert(kRing32Coef % 2 == 0, "FP32 ring records are staged in 16-byte units");
// raw moments of a cell about its centre for the upward pass: A_k, B_k, D_k (k = 0..kCl64Order)
constexpr int kCellRaw = 3 * (kCl64Order + 1);
// a cell's record for the translations: k_cluster_moments64's layout, then (c_x, c_y), pad
constexpr int kCellRec = kCl64CoefPerCluster + 2;
constexpr double kPiD = 3.14159265358979323846;

struct Status {
  mfs_status code = MFS_OK;
  std::string msg;
};

// A caller-provided buffer for the kernel sum's split partials (cap doubles): the
// kernel sum then allocates nothing.
struct SplitBuf {
  double* p = nullptr;
  int64_t cap = 0;
};

// Shared one-body factors of a disk class, passed to kernels by value.
struct ClassTab {
  int n = 0;
  int nc[kMaxClasses], mc[kMaxClasses], rank[kMaxClasses];
  const double* U[kMaxClasses];     // (2 mc x rank) row-major: left singular vectors
  const double* sinv[kMaxClasses];  // rank: truncated 1/sigma
  const double* Vt[kMaxClasses];    // (rank x 2 nc) row-major: right singular vectors transposed
  const double* Yr[kMaxClasses];    // nc x 2: sources relative to the centre
  const double* Xr[kMaxClasses];    // mc x 2: nodes relative to the centre
  double KtKi[kMaxClasses][9];      // (K^T K)^{-1}, row-major, of the coarse source ring
  double radius[kMaxClasses];
  // squared distances from a disk's centre beyond which its ring expansion at the tier orders
  // (FP64 sum: 27, 40, kRing64Order; FP32 sum: 14, 24, kRing32Order) meets the truncation target
  double tier64[kMaxClasses][kRingTiers], tier32[kMaxClasses][kRingTiers];
};

// Where one vector's records of the hierarchical kernel sum go: the context's buffers (vector
// r, fmm_records) or a caller's buffer
struct FmmRec {
  double2* raw = nullptr;   // ncell x kCellRaw
  double2* rec = nullptr;   // ncell x kCellRec
  double2* r64 = nullptr;   // P x kRing64Coef
  float2* r32 = nullptr;    // P x kRing32Coef
};

// Per-wave interaction lists of the hierarchical kernel sum for one separation factor
struct FmmLists {
  double sep = 0.0;
  std::vector<int32_t> m2l_off, m2l, near_off, near;   // CSR per wave; near: slots, increasing
  int32_t *d_m2l_off = nullptr, *d_m2l = nullptr, *d_near_off = nullptr, *d_near = nullptr;
};

struct PairSet {
  bool ready = false;
  double* A = nullptr;   // per pair column-major (n x n), n = n_i + n_k, offset aoff[c]
  double* E = nullptr;   // per pair column-major (6 x n), offset 6 * xoff[c]
  // fine factors for flow evaluation (kept by the precompute on request)
  bool fine = false;
  double* G = nullptr;        // per pair column-major (nf x n) fine map, nf = 2 (nf_i + nf_k), offset goff[c]
  double* Yf = nullptr;       // per pair nf_i + nf_k fine source points (x, y), offset yoff[c]
  double* KKf = nullptr;      // per pair 2 x 9: (K_f^T K_f)^{-1} of disk i's and disk k's fine sources
  double* pgeo = nullptr;     // per pair 12: c_i, c_k, a_i, a_k, lower and upper rolling-circle centres
  int32_t* nf = nullptr;      // per pair 2: fine source counts of disk i and disk k
  int64_t *d_goff = nullptr, *d_yoff = nullptr;
  std::vector<int64_t> goff, yoff;   // C + 1 (yoff counts doubles: 2 per fine point)
};

// GMRES work space, sized on first use, for up to rcap right-hand sides in lockstep.
struct Krylov {
  int64_t n = 0;
  int cap = 0;           // basis vectors allocated per right-hand side
  int rcap = 0;          // right-hand sides
  double* V = nullptr;   // n x rcap x (cap + 1): vector j of right-hand side r at V + (j rcap + r) n
  double* w = nullptr;
  double* part = nullptr;    // partial dot products
  double* hdev = nullptr;    // reduced dots
  double* hhost = nullptr;   // pinned host mirror
  double* x = nullptr;    // the vectors below hold rcap x n doubles
  double* r = nullptr;
  double* b = nullptr;
  double* d = nullptr;
  double* tmp = nullptr;
  // device least squares (k_givens): per right-hand side H ((cap + 1) x cap), cs, sn (cap),
  // g (cap + 1), y (cap + 1), ctl (kGmCtl); per iteration and right-hand side 4 record values,
  // mirrored in pinned host memory
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr, *ctl = nullptr, *rec = nullptr;
  double* hrec = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
};

}  // namespace mfs

struct mfs_ctx {
  int P = 0;
  mfs_params prm{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  rocblas_handle blas = nullptr;
  mfs::Status last;
  int pre_batch = 0;   // pairs per precompute batch; 0: sized from free device memory
  bool keep_fine = false;  // the precompute keeps each pair's fine map and points (flow evaluation)
  mfs_allocator alloc{nullptr, nullptr, nullptr};   // caller's device allocator (alloc NULL: hipMalloc)

  // host geometry
  std::vector<double> centers, radii, r_src;
  std::vector<int32_t> n_src, n_col, cls;  // per body
  std::vector<int32_t> src_off, col_off;   // P + 1
  std::vector<int32_t> pairs;              // 2 C
  std::vector<int64_t> xoff, aoff, coff;   // C + 1: pair source-vector, matrix and node-vector offsets
  std::vector<int32_t> bp_off, bp_list;    // body -> (pair, side) CSR
  std::vector<int32_t> nbr_off, nbr_list;  // body -> sorted contact partners
  // FP32 kernel-sum order: slot_body[s] = body in slot s, slot_of[b] = its inverse;
  // cluster q holds slots cl_start[q] .. cl_start[q + 1] - 1
  std::vector<int32_t> slot_body, slot_of, cl_start;
  std::vector<double> cl_centre, cl_radius;   // 2 ncl, ncl: centre and the radius holding its sources
  int ncl = 0;
  int64_t Ns = 0, Nt = 0;

  // class data
  mfs::ClassTab ct[2];                     // [problem]
  std::vector<void*> class_bufs;
  std::vector<double> h_Yr[mfs::kMaxClasses], h_Xr[mfs::kMaxClasses];   // host copies (relative rings)

  // device geometry
  int32_t *d_src_off = nullptr, *d_col_off = nullptr, *d_cls = nullptr, *d_tgt_body = nullptr;
  int32_t *d_pairs = nullptr, *d_bp_off = nullptr, *d_bp_list = nullptr, *d_nbr_off = nullptr, *d_nbr_list = nullptr;
  int64_t *d_xoff = nullptr, *d_aoff = nullptr, *d_coff = nullptr;
  double* d_centers = nullptr;   // P x 2
  double* d_Y = nullptr;         // Ns x 2 absolute sources
  double* d_X = nullptr;         // Nt x 2 absolute nodes
  // disks in slot order (a space-filling curve): the kernel sums' visiting order
  int32_t *d_slot_of = nullptr, *d_slot_body = nullptr, *d_ssrc_off = nullptr, *d_nbr_slot = nullptr;
  int32_t* d_cl_start = nullptr;
  double* d_ccent = nullptr;     // ncl x 2 cluster centres
  double* d_crad64 = nullptr;    // ncl cluster radii (FP64 sum)
  int32_t* d_tperm = nullptr;    // Nt: the kernel sums visit targets in slot order (disk by disk)
  // hierarchical kernel sum: cells (leaves 0..P-1 = slots), children CSR, heights, wave centres
  int ncell = 0, nwave = 0, cell_height = 0;
  std::vector<int32_t> cell_lo, cell_hi, cell_child_off, cell_child, cell_by_height, height_off;
  std::vector<double> cell_c, cell_r;   // 2 ncell centres, ncell source radii
  int32_t *d_cell_child_off = nullptr, *d_cell_child = nullptr, *d_cell_by_height = nullptr;
  double *d_cell_c = nullptr, *d_wcent = nullptr;
  int32_t* d_wstart = nullptr;   // nwave + 1: each wave's first position in the visiting order
  std::vector<int32_t> h_wstart;   // host copies of the wave starts and centres
  std::vector<double> h_wcent;
  mfs::FmmLists fl[2];           // [0] FP64 sum, [1] mixed sum
  double2* d_cellraw = nullptr;  // ncell x kCellRaw (per stacked vector: rhs_cap of them)
  double2* d_cellrec = nullptr;  // ncell x kCl64CoefPerCluster
  double2* d_ring64 = nullptr;   // P x kRing64Coef (slot order)
  float2* d_ring32 = nullptr;    // P x kRing32Coef (slot order)
  int fmm_rcap = 0;              // vectors the record buffers above hold
  unsigned long long* d_work = nullptr;   // kernel-sum work counters: direct pairs, disk and cluster expansions
  double* scratch = nullptr;     // the device's static scratch array (mfs_apply_noalloc), resolved at setup

  // work vectors
  double *d_lam_bar = nullptr, *d_ltil = nullptr, *d_u = nullptr, *d_corr = nullptr;
  double *d_upart = nullptr, *d_epair = nullptr, *d_out3 = nullptr, *d_given = nullptr;
  double4* d_src64 = nullptr;    // per source: (y_x, y_y, sigma_x, sigma_y)
  int64_t upart_cap = 0;

  // stacked right-hand sides of the matvec (allocated on first use for rhs_cap vectors)
  int rhs_cap = 0;
  double *d_lam_bar_m = nullptr, *d_ltil_m = nullptr, *d_u_m = nullptr, *d_corr_m = nullptr;
  double4* d_src64m = nullptr;   // rhs_cap arrays of Ns records

  mfs::PairSet ps[2];
  mfs::Krylov kr;

  // densities of the latest mfs_gmres_solve (n x mu_count) and flow-evaluation work space
  double* d_mu_last = nullptr;
  int64_t mu_cap = 0;
  int mu_count = 0, mu_prob = -1;
  double4* d_fsrc = nullptr;           // Ns records: sources with the total strengths
  double *d_ptil = nullptr, *d_sigf = nullptr;   // projected lambda_tilde (xoff[C]); fine strengths (max yoff)
  double2* d_fmp64 = nullptr;          // far-field coefficients of d_fsrc
  int64_t sigf_cap = 0;

  // work counters (host side, reset by mfs_gmres_solve)
  int64_t evals_all = 0, evals_skip = 0;     // pair evaluations of one kernel sum per skip mode
  int64_t cnt_pair_evals = 0;
  int32_t cnt_mv64 = 0, cnt_mv32 = 0;
};

namespace mfs {

// Length (double2) of one FP64 far-field record: kMp64CoefPerDisk per disk, then
// kCl64CoefPerCluster per cluster
inline int64_t mp64_record(const mfs_ctx* c) {
  return (int64_t)c->P * kMp64CoefPerDisk + (int64_t)c->ncl * kCl64CoefPerCluster;
}

// Device memory of a context: the caller's allocator when mfs_setup_ex gave one, else
// hipMalloc / hipFree (capi.hip).
hipError_t dev_malloc(mfs_ctx* c, void** p, size_t bytes);
void dev_free(mfs_ctx* c, void* p);
template <class T>
hipError_t dev_malloc(mfs_ctx* c, T** p, size_t bytes) {
  return dev_malloc(c, (void**)p, bytes);
}

// ---- kernel launchers (kernels.hip) ----
void launch_onebody_apply(mfs_ctx* c, int prob, const double* mu, double* lam_bar);
void launch_pair_A(mfs_ctx* c, int prob, const double* lam_bar, double* ltil);
// strengths packed into c->d_src64 and the hierarchical kernel sum's records of them (fr; NULL:
// the context's), with the FP32 ring records when pack32
void launch_gather_project(mfs_ctx* c, int prob, const double* lam_bar, const double* ltil, bool with_pairs,
                           bool pack32, bool pack64, const FmmRec* fr = nullptr);
// the same into an explicit packed array (caller's disk order)
void launch_gather_project_to(mfs_ctx* c, int prob, const double* lam_bar, const double* ltil, bool with_pairs,
                              double4* src64);
// stacked forms for R = 2, 4 or 8 vectors (false: unsupported size or out of memory)
bool launch_pair_A_rhs(mfs_ctx* c, int prob, int R, const double* lam_bar, int64_t lam_stride, double* ltil,
                       int64_t ltil_stride);
bool launch_kernel_sum_rhs(mfs_ctx* c, bool mixed, int mode, int R, double* u, double scale);
// mode 0: all sources; 1: skip the target's own disk; 2: also skip its contact partners.  Sums
// c->d_src64 with the records fr (NULL: the context's).  false: out of memory
bool launch_kernel_sum(mfs_ctx* c, bool mixed, int mode, double* u, double scale, const FmmRec* fr = nullptr);
// hierarchical kernel sum (fmm.hip): host tree and lists at setup; records of packed FP64
// sources (src64) for R stacked vectors; the sum itself at the context's targets
Status build_fmm(mfs_ctx* c);
Status ensure_fmm_records(mfs_ctx* c, int R);
FmmRec fmm_records(mfs_ctx* c, int r);
int64_t fmm_record_doubles(const mfs_ctx* c);
bool fmm_records_in(const mfs_ctx* c, const SplitBuf* sb, FmmRec* out);   // false: sb too small
void launch_fmm_records(mfs_ctx* c, int prob, const double4* src64, const FmmRec& fr, bool ring32);
void launch_ksum_fmm(mfs_ctx* c, bool mixed, int mode, const double4* src64, const FmmRec& fr, double* u,
                     double scale);
// zero the kernel-sum work counters (a kernel, so that the call may sit in a captured graph)
void launch_zero_work(mfs_ctx* c);
// the device's static scratch array for mfs_apply_noalloc (kernels.hip), resolved once per device
constexpr int64_t kScratchDoubles = (int64_t)16 << 20;   // 128 MiB
Status scratch_for_current_device(double** ptr);
void launch_pair_field(mfs_ctx* c, int prob, const double* ltil, double* corr);
void launch_finish(mfs_ctx* c, const double* u_sum, const double* mu, const double* corr, double* u_out,
                   bool with_pairs);
void launch_rhs_mobility_sources(mfs_ctx* c, const double* given);
void launch_rhs_resistance(mfs_ctx* c, const double* given, double* b);
void launch_post(mfs_ctx* c, int prob, const double* lam_bar, double* out3);
// flow evaluation (kernels.hip)
void launch_add_rhs_sources(mfs_ctx* c, const double* given, double4* src64);
bool launch_kernel_sum_points(mfs_ctx* c, const double4* src, const double2* mp64, int64_t n_pts,
                              const double* pts, const int32_t* body, double* u);
// FP64 far-field coefficients of a packed FP64 source array: per disk, then per cluster
// (one mp64_record)
void launch_moments64(mfs_ctx* c, const double4* src64, double2* mp64);
void launch_fine_strengths(mfs_ctx* c, int prob, const double* lam_bar, const double* ltil, double* ptil,
                           double* sigf);
void launch_flow_near(mfs_ctx* c, int prob, int64_t n_pts, const double* pts, const int32_t* body,
                      const double* ptil, const double* sigf, double* u);
void launch_boundary_nodes(mfs_ctx* c, int n_per_body, double* pts, int32_t* body);
void launch_boundary_residual(mfs_ctx* c, int64_t n_pts, const double* pts, const int32_t* body, const double* u,
                              const double* rigid, double* eps, double* maxima);
// GMRES helpers
void launch_mdot(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* w, double* part,
                 double* out, int nblk);
void launch_maxpy(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* h, double* w);
void launch_scale_copy(hipStream_t s, int64_t n, double a, const double* x, double* y);
void launch_axpby(hipStream_t s, int64_t n, double a, const double* x, double b, double* y);
void launch_gemv_n(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* y, double* x);
// GMRES least squares on the device: control record per right-hand side
constexpr int kGmBeta = 0, kGmTol = 1, kGmInv = 2, kGmK = 3, kGmDone = 4, kGmBad = 5, kGmEst = 6, kGmCtl = 8;
void launch_givens(hipStream_t s, int j, int cap, int R, const double* hdev, int64_t hstride, double* H, double* cs,
                   double* sn, double* g, double* ctl, double* rec);
void launch_scale_ctl(hipStream_t s, int64_t n, int R, const double* ctl, const double* x, double* y);
void launch_backsolve(hipStream_t s, int cap, int R, const double* H, const double* g, const double* ctl, double* y);
int mdot_blocks(int64_t n);

// ---- precompute (precompute.hip) ----
Status onebody_factors(mfs_ctx* c);
Status precompute_pairs(mfs_ctx* c, int prob);

// ---- matvec pieces (capi.hip) ----
// sb: a caller's buffer for the kernel sum's records (mfs_apply_noalloc); NULL: the context's
Status apply_T(mfs_ctx* c, int prob, bool mixed, const double* mu, double* u, const SplitBuf* sb = nullptr);
// T applied to R vectors (mu, u: R x n, vector r at offset r n); stacked kernels for R in {2, 4, 8}
Status apply_T_rhs(mfs_ctx* c, int prob, bool mixed, int R, const double* mu, double* u);

}  // namespace mfs

#define MFS_HIP(call)                                                                             \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess)                                                                         \
      return ::mfs::Status{MFS_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)
