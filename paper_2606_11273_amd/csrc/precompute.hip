// Device precompute: one-body factors (Sec. 3.1, Sec. 4.1) and per-pair compressed
// corrections (Sec. 3.2-3.4, Sec. 4.3-4.4, Sec. 5), FP64 throughout.
//
// Per pair (i, k), with fine sources Yf, fine nodes Xf, peanut nodes z, coarse
// sources Yc = Y^(i) u Y^(k) and Pi = I - L (mobility) or I (resistance):
//   F  = S(Xf, Yf) Pi_f [+ blockdiag(Bf_i Kf_i^T, Bf_k Kf_k^T) for mobility]
//   X  = [[0, S(Xf_i, Y^(k)) Pi], [S(Xf_k, Y^(i)) Pi, 0]]
//   C  = S(z, Yc) Pi,   D = S(z, Yf) Pi_f
//   G  = F^+ X  (truncated SVD, 1e-11 relative), applied as V (Sigma^+ (U^T X))
//   A  = -C^+ (D G)  (truncated SVD, 1e-14 relative)
//   E  = +-blockdiag(Kf_i^T, Kf_k^T) G   (+ mobility velocities, - resistance forces)
// Matrices are filled by a kernel of this file, factorised by rocSOLVER's batched
// SVD and multiplied with rocBLAS GEMMs; pairs are processed in batches of one class
// combination (class of disk i, class of disk k) whose fine source lists are zero-padded
// per disk to a common length (zero columns do not change the truncated pseudoinverse).
// The paper's fine sets are for unit disks; a disk of radius a gets fine counts scaled by a,
// the limit point of its two circles and a rolling unit circle for the peanut.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <array>
#include <cstring>
#include <string>

#include "internal.h"

namespace mfs {

// The SVD and QR entry points.  A host process may already hold another rocSOLVER under the same soname
// (PyTorch's wheel bundles its own ROCm libraries and loads them first; the library's
// dependencies then bind to those, which keeps one HIP runtime per process).  The batched SVD of
// the rocSOLVER in the ROCm installation this library is built against (MFS_ROCM_LIB) is several
// times faster at these sizes than older ones, so its entry points are taken from there,
// loaded by path; it binds to the process's rocBLAS and HIP runtime like the library itself
// (same soname majors).  If that file cannot be loaded, or MFS_ROCSOLVER_LINKED=1, the linked
// rocSOLVER is used.
#ifndef MFS_ROCM_LIB
#define MFS_ROCM_LIB "/opt/rocm/lib"
#endif
struct SvdEntry {
  decltype(&rocsolver_dgesvd) gesvd = &rocsolver_dgesvd;
  decltype(&rocsolver_dgesvd_strided_batched) gesvd_sb = &rocsolver_dgesvd_strided_batched;
  decltype(&rocsolver_dgeqrf_strided_batched) geqrf_sb = &rocsolver_dgeqrf_strided_batched;
  const char* origin = "linked";
};
static const SvdEntry& svd_entry() {
  static const SvdEntry e = [] {
    SvdEntry r;
    const char* lk = std::getenv("MFS_ROCSOLVER_LINKED");
    if (lk && std::atoi(lk) != 0) return r;
    void* h = dlopen(MFS_ROCM_LIB "/librocsolver.so.0", RTLD_NOW | RTLD_LOCAL);
    if (!h) return r;
    auto a = (decltype(&rocsolver_dgesvd))dlsym(h, "rocsolver_dgesvd");
    auto b = (decltype(&rocsolver_dgesvd_strided_batched))dlsym(h, "rocsolver_dgesvd_strided_batched");
    auto q = (decltype(&rocsolver_dgeqrf_strided_batched))dlsym(h, "rocsolver_dgeqrf_strided_batched");
    if (a && b && q) {
      r.gesvd = a;
      r.gesvd_sb = b;
      r.geqrf_sb = q;
      r.origin = MFS_ROCM_LIB "/librocsolver.so.0";
    }
    return r;
  }();
  return e;
}

#define MFS_RB(call)                                                                          \
  do {                                                                                        \
    rocblas_status s_ = (call);                                                               \
    if (s_ != rocblas_status_success)                                                         \
      return Status{MFS_ERR_DEVICE, std::string(#call) + ": rocBLAS status " + std::to_string((int)s_)}; \
  } while (0)

namespace {

// Stokeslet block at d = x - y, scaled by 1/(4 pi mu): s00, s01(=s10), s11.
__device__ __forceinline__ void stokeslet(double dx, double dy, double k, double& s00, double& s01, double& s11) {
  const double r2 = dx * dx + dy * dy;
  const double lg = 0.5 * log(r2);
  const double ir2 = 1.0 / r2;
  s00 = k * (dx * dx * ir2 - lg);
  s11 = k * (dy * dy * ir2 - lg);
  s01 = k * (dx * dy * ir2);
}

// One column block of a projected Stokeslet matrix: the sources of one body.
struct SrcBlock {
  const double* y;   // n x 2 absolute positions
  int n;             // actual count
  int col0;          // first point column of this block in the matrix
  double cx, cy;     // body centre
  const double* KKi; // (K^T K)^{-1} of this block's sources (row-major 3x3)
};

// Fill rows 2t, 2t+1 of a column-major matrix for target point x on body rb
// (0 or 1), with source blocks b0, b1:
//   value = S(x, y_s) - (S K)(x) (K^T K)^{-1} K_s^T   [if project]
//         + B_x K_s^T                                  [if rigid and block == rb]
// Blocks with index == rb are left zero when cross_only.
__device__ void fill_row(double* M, int64_t ld, int64_t row2, double x, double y, int rb, const SrcBlock* blk,
                         bool project, bool rigid, bool cross_only, double kscale) {
  for (int b = 0; b < 2; ++b) {
    const SrcBlock& B = blk[b];
    if (cross_only && b == rb) continue;
    double sk[2][3] = {{0, 0, 0}, {0, 0, 0}};
    if (project) {
      for (int s = 0; s < B.n; ++s) {
        double s00, s01, s11;
        stokeslet(x - B.y[2 * s], y - B.y[2 * s + 1], kscale, s00, s01, s11);
        const double rx = B.y[2 * s] - B.cx, ry = B.y[2 * s + 1] - B.cy;
        // S K_s with K_s = [1 0 -ry; 0 1 rx]
        sk[0][0] += s00;
        sk[0][1] += s01;
        sk[0][2] += -s00 * ry + s01 * rx;
        sk[1][0] += s01;
        sk[1][1] += s11;
        sk[1][2] += -s01 * ry + s11 * rx;
      }
    }
    // SK (K^T K)^{-1}
    double q[2][3] = {{0, 0, 0}, {0, 0, 0}};
    if (project)
      for (int a = 0; a < 2; ++a)
        for (int m = 0; m < 3; ++m) q[a][m] = sk[a][0] * B.KKi[0 * 3 + m] + sk[a][1] * B.KKi[1 * 3 + m] + sk[a][2] * B.KKi[2 * 3 + m];
    const bool add_rigid = rigid && b == rb;
    const double bx = x - B.cx, by = y - B.cy;  // B_x = [1 0 -by; 0 1 bx]
    for (int s = 0; s < B.n; ++s) {
      double s00, s01, s11;
      stokeslet(x - B.y[2 * s], y - B.y[2 * s + 1], kscale, s00, s01, s11);
      const double rx = B.y[2 * s] - B.cx, ry = B.y[2 * s + 1] - B.cy;
      // K_s^T = [1 0; 0 1; -ry rx]
      double v00 = s00, v01 = s01, v10 = s01, v11 = s11;
      if (project) {
        v00 -= q[0][0] - q[0][2] * ry;
        v01 -= q[0][1] + q[0][2] * rx;
        v10 -= q[1][0] - q[1][2] * ry;
        v11 -= q[1][1] + q[1][2] * rx;
      }
      if (add_rigid) {  // B_x K_s^T
        v00 += 1.0 + by * ry;
        v01 += -by * rx;
        v10 += -bx * ry;
        v11 += 1.0 + bx * rx;
      }
      const int64_t col2 = 2 * (int64_t)(B.col0 + s);
      M[col2 * ld + row2] = v00;
      M[col2 * ld + row2 + 1] = v10;
      M[(col2 + 1) * ld + row2] = v01;
      M[(col2 + 1) * ld + row2 + 1] = v11;
    }
  }
}

struct PairGeo {
  // per pair in a batch (device pointers into one staging buffer)
  const double* yf[2];   // fine sources of i and k
  const double* yc[2];   // coarse sources of i and k
  const double* xf;      // 2 mf fine nodes (i then k)
  const double* z;       // mp peanut nodes
  int nf[2];
  double c[2][2];
  double KKf[2][9];      // fine (K^T K)^{-1} per body
  double KKc[2][9];      // coarse (K^T K)^{-1} per body (its class)
};

// Sizes of one batch (all its pairs have the same disk classes on each side).
struct BatchDims {
  int mf[2];     // fine nodes of disk i, disk k
  int nfpad[2];  // padded fine sources of disk i, disk k
  int nc[2];     // coarse sources of disk i, disk k
  int mp;        // peanut nodes
  int64_t ldF, ldD;  // = 2 (mf0 + mf1), 2 mp
  int64_t sF, sX, sD, sC;  // batch strides
};

// One thread per target point of one matrix; blockIdx.y = pair in batch, blockIdx.z = matrix (0 F, 1 X, 2 D, 3 C).
__global__ __launch_bounds__(64) void k_fill(const PairGeo* __restrict__ geo, BatchDims d, int mobility, double kscale,
                                             double* F, double* X, double* D, double* Cm) {
  const int p = blockIdx.y;
  const int which = blockIdx.z;
  const PairGeo& g = geo[p];
  const int npts = (which <= 1) ? d.mf[0] + d.mf[1] : d.mp;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npts) return;
  SrcBlock blk[2];
  const bool fine_cols = (which == 0 || which == 2);
  for (int b = 0; b < 2; ++b) {
    blk[b].y = fine_cols ? g.yf[b] : g.yc[b];
    blk[b].n = fine_cols ? g.nf[b] : d.nc[b];
    blk[b].col0 = b == 0 ? 0 : (fine_cols ? d.nfpad[0] : d.nc[0]);
    blk[b].cx = g.c[b][0];
    blk[b].cy = g.c[b][1];
    blk[b].KKi = fine_cols ? g.KKf[b] : g.KKc[b];
  }
  double x, y;
  int rb = -1;
  if (which <= 1) {
    x = g.xf[2 * t];
    y = g.xf[2 * t + 1];
    rb = t < d.mf[0] ? 0 : 1;
  } else {
    x = g.z[2 * t];
    y = g.z[2 * t + 1];
  }
  const bool proj = mobility != 0;
  switch (which) {
    case 0: fill_row(F + p * d.sF, d.ldF, 2 * (int64_t)t, x, y, rb, blk, proj, proj, false, kscale); break;
    case 1: fill_row(X + p * d.sX, d.ldF, 2 * (int64_t)t, x, y, rb, blk, proj, false, true, kscale); break;
    case 2: fill_row(D + p * d.sD, d.ldD, 2 * (int64_t)t, x, y, -1, blk, proj, false, false, kscale); break;
    default: fill_row(Cm + p * d.sC, d.ldD, 2 * (int64_t)t, x, y, -1, blk, proj, false, false, kscale); break;
  }
}

// sinv_j = 1/s_j if s_j > eps s_0 else 0, then scale row j of T (column-major, ld, ncol columns).
// s_0 is the largest singular value of the group of `group` consecutive matrices that p belongs
// to (the two symmetry blocks of one pair share the threshold of the whole matrix).
__global__ __launch_bounds__(256) void k_trunc_scale(int nsv, const double* __restrict__ S, int64_t sS, double eps,
                                                     double* T, int64_t ld, int ncol, int64_t sT, int group) {
  const int p = blockIdx.y;
  // sigma_1 as the largest entry (no reliance on the order the SVD returns)
  __shared__ double red[256];
  double m = 0.0;
  const int g0 = (p / group) * group;
  for (int j = threadIdx.x; j < nsv * group; j += 256) m = fmax(m, S[(g0 + j / nsv) * sS + j % nsv]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const double s0 = red[0];
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)nsv * ncol) return;
  const int j = (int)(idx % nsv);
  const int col = (int)(idx / nsv);
  const double sj = S[p * sS + j];
  const double f = (sj > eps * s0) ? 1.0 / sj : 0.0;
  T[p * sT + (int64_t)col * ld + j] *= f;
}

// Pairs of equal disks.  The point reflection through the pair's midpoint maps each of the
// pair's point sets onto itself, disk i's points onto disk k's (a ring of an even count from
// angle 0: point j to point j + n/2; the ellipse sources and Moebius nodes, built in the pair's
// frame: point j to point j; the peanut: point p to point p + M_p/2), and flips every vector.
// The Stokeslet is even in x - y, so F, C, D and X commute with it, and in the orthonormal
// bases Q_e = [I; e Sigma] / sqrt 2 (e = +1, -1; Sigma the map from disk i's points to disk
// k's with the sign flip) each splits into two blocks of half the size:
//   F_e = F_ii + e F_ik Sigma_s,  X_e = (X_i + e Sigma_n^T X_k) / sqrt 2,
// F^+ X = sum_e Q_e F_e^+ X_e, the singular values of F being those of F_+ and F_- (one
// truncation threshold for both).  The peanut's two halves (points p < M_p/2 and their images)
// play the parts of disk i's and disk k's nodes for C and D G.
__device__ __forceinline__ int sym_map(int j, int nring) { return j < nring ? (j + nring / 2) % nring : j; }

// [F_e X_e] (mh x (nh + nx), leading dimension mh) of every pair of a batch: matrix 2q + (e < 0)
// of FXs.  One block per (column, matrix); column c < nh of F_e, else column c - nh of X_e.
__global__ __launch_bounds__(256) void k_sym_split_F(const double* __restrict__ F, int64_t ldF, int64_t sF,
                                                     const double* __restrict__ X, int64_t sX, int mh, int nh, int nx,
                                                     int nring_src, int nring_node, double* __restrict__ FXs) {
  const int col = blockIdx.x, mat = blockIdx.y, q = mat >> 1;
  const double e = (mat & 1) ? 1.0 : -1.0;   // + block: F_ii - F_ik[mapped]; the minus sign is Sigma's flip
  double* o = FXs + (int64_t)mat * mh * (nh + nx) + (int64_t)col * mh;
  if (col < nh) {
    const int colk = nh + 2 * sym_map(col >> 1, nring_src) + (col & 1);
    const double* a = F + q * sF + (int64_t)col * ldF;
    const double* b = F + q * sF + (int64_t)colk * ldF;
    for (int r = threadIdx.x; r < mh; r += 256) o[r] = a[r] + e * b[r];
  } else if (col < nh + nx) {
    const int xc = col - nh;
    const double* a = X + q * sX + (int64_t)xc * ldF;
    for (int r = threadIdx.x; r < mh; r += 256) {
      const int rk = mh + 2 * sym_map(r >> 1, nring_node) + (r & 1);
      o[r] = (a[r] + e * a[rk]) * 0.70710678118654752440;
    }
  }
}

// After the Householder QR of a tall [F X] (rows x (cols + nx), R in the upper triangle): the
// cols x cols factor R11 (zeros below the diagonal) and R12 = Q1^T X (cols x nx), both with
// leading dimension cols.  One block per (column, matrix).
__global__ __launch_bounds__(256) void k_split_qr(const double* __restrict__ A, int64_t rows, int64_t sA, int cols,
                                                  int nx, double* __restrict__ R, double* __restrict__ T0) {
  const int col = blockIdx.x, mat = blockIdx.y;
  const double* a = A + (int64_t)mat * sA + (int64_t)col * rows;
  if (col < cols) {
    double* o = R + (int64_t)mat * cols * cols + (int64_t)col * cols;
    for (int r = threadIdx.x; r < cols; r += 256) o[r] = r <= col ? a[r] : 0.0;
  } else if (col < cols + nx) {
    double* o = T0 + (int64_t)mat * cols * nx + (int64_t)(col - cols) * cols;
    for (int r = threadIdx.x; r < cols; r += 256) o[r] = a[r];
  }
}

// G (n x nx per pair, stride sG) from G_e (nh x nx, matrices 2q, 2q + 1):
// G_i = (G_+ + G_-) / sqrt 2, G_k = Sigma_s (G_+ - G_-) / sqrt 2.  One block per (column, pair).
__global__ __launch_bounds__(256) void k_sym_join_G(const double* __restrict__ Gs, int nh, int nx, int nring_src,
                                                    double* __restrict__ G, int64_t sG) {
  const int col = blockIdx.x, q = blockIdx.y;
  const double* gp = Gs + (int64_t)(2 * q) * nh * nx + (int64_t)col * nh;
  const double* gm = gp + (int64_t)nh * nx;
  double* o = G + q * sG + (int64_t)col * (2 * nh);
  for (int j = threadIdx.x; j < nh; j += 256) {
    const double p = gp[j], m = gm[j];
    o[j] = (p + m) * 0.70710678118654752440;
    o[nh + 2 * sym_map(j >> 1, nring_src) + (j & 1)] = -(p - m) * 0.70710678118654752440;
  }
}

// C_e (zh x nxh) and (D G)_e (zh x nx): rows of the peanut's first half (zh = M_p rows) and of
// its images (rows zh + r); columns of disk i's coarse sources and of disk k's (ring of ncc).
__global__ __launch_bounds__(256) void k_sym_split_C(const double* __restrict__ Cm, int64_t sC,
                                                     const double* __restrict__ DG, int64_t sDG, int zh, int nxh,
                                                     int nx, int ncc, double* __restrict__ Cs,
                                                     double* __restrict__ DGs) {
  const int col = blockIdx.x, mat = blockIdx.y, q = mat >> 1;
  const double e = (mat & 1) ? 1.0 : -1.0;
  const int64_t ld = 2 * (int64_t)zh;
  if (col < nxh) {
    const int colk = nxh + 2 * sym_map(col >> 1, ncc) + (col & 1);
    const double* a = Cm + q * sC + (int64_t)col * ld;
    const double* b = Cm + q * sC + (int64_t)colk * ld;
    double* o = Cs + (int64_t)mat * zh * nxh + (int64_t)col * zh;
    for (int r = threadIdx.x; r < zh; r += 256) o[r] = a[r] + e * b[r];
  } else if (col < nxh + nx) {
    const int xc = col - nxh;
    const double* a = DG + q * sDG + (int64_t)xc * ld;
    double* o = DGs + (int64_t)mat * zh * nx + (int64_t)xc * zh;
    for (int r = threadIdx.x; r < zh; r += 256) o[r] = (a[r] + e * a[zh + r]) * 0.70710678118654752440;
  }
}

// A (nx x nx, column-major, into A + aoff[q]) from A_e (nxh x nx): rows of disk i's coarse
// sources (A_+ + A_-) / sqrt 2, of disk k's Sigma_c (A_+ - A_-) / sqrt 2.
__global__ __launch_bounds__(256) void k_sym_join_A(const double* __restrict__ As, int nxh, int nx, int ncc,
                                                    double* __restrict__ A, const int64_t* __restrict__ aoff) {
  const int col = blockIdx.x, q = blockIdx.y;
  const double* ap = As + (int64_t)(2 * q) * nxh * nx + (int64_t)col * nxh;
  const double* am = ap + (int64_t)nxh * nx;
  double* o = A + aoff[q] + (int64_t)col * nx;
  for (int j = threadIdx.x; j < nxh; j += 256) {
    const double p = ap[j], m = am[j];
    o[j] = (p + m) * 0.70710678118654752440;
    o[nxh + 2 * sym_map(j >> 1, ncc) + (j & 1)] = -(p - m) * 0.70710678118654752440;
  }
}

// Keep G of each pair in compact form for flow evaluation: the rows of the padded
// per-batch G (disk i's fine sources at 0, disk k's at 2 nfpad0) go to rows 0..2 nf_i and
// 2 nf_i..2 (nf_i + nf_k) of a column-major (2 (nf_i + nf_k)) x ncols block at goff[q].
__global__ __launch_bounds__(256) void k_store_fine(int ncols, int nfpad0, const int32_t* __restrict__ nfq,
                                                    const double* __restrict__ G, int64_t sG, int64_t ldG,
                                                    double* __restrict__ Gout, const int64_t* __restrict__ goff) {
  const int col = blockIdx.x, q = blockIdx.y;
  if (col >= ncols) return;
  const int nf0 = nfq[2 * q], nf1 = nfq[2 * q + 1];
  const int nfr = 2 * (nf0 + nf1);
  const double* src = G + q * sG + (int64_t)col * ldG;
  double* dst = Gout + goff[q] + (int64_t)col * nfr;
  for (int rr = threadIdx.x; rr < nfr; rr += 256) dst[rr] = src[rr < 2 * nf0 ? rr : 2 * nfpad0 + (rr - 2 * nf0)];
}

// E = sgn blockdiag(Kf_i^T, Kf_k^T) G for each pair; G column-major (2 (nfpad0 + nfpad1)) x ncols.
__global__ void k_extract(const PairGeo* __restrict__ geo, BatchDims d, const double* __restrict__ G, int64_t sG,
                          double sgn, double* __restrict__ E, const int64_t* __restrict__ eoff) {
  const int p = blockIdx.y;
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int ncols = 2 * (d.nc[0] + d.nc[1]);
  if (col >= ncols) return;
  const PairGeo& g = geo[p];
  const double* Gc = G + p * sG + (int64_t)col * (2 * (d.nfpad[0] + d.nfpad[1]));
  for (int b = 0; b < 2; ++b) {
    double f0 = 0, f1 = 0, f2 = 0;
    for (int s = 0; s < g.nf[b]; ++s) {
      const int64_t r = 2 * (int64_t)((b == 0 ? 0 : d.nfpad[0]) + s);
      const double gx = Gc[r], gy = Gc[r + 1];
      const double rx = g.yf[b][2 * s] - g.c[b][0], ry = g.yf[b][2 * s + 1] - g.c[b][1];
      f0 += gx;
      f1 += gy;
      f2 += -ry * gx + rx * gy;
    }
    double* Ec = E + eoff[p] + (int64_t)col * 6;
    Ec[3 * b] = sgn * f0;
    Ec[3 * b + 1] = sgn * f1;
    Ec[3 * b + 2] = sgn * f2;
  }
}

void inv3(const double* M, double* R) {
  const double a = M[0], b = M[1], c = M[2], d = M[3], e = M[4], f = M[5], g = M[6], h = M[7], i = M[8];
  const double A = e * i - f * h, B = -(d * i - f * g), C = d * h - e * g;
  const double det = a * A + b * B + c * C;
  R[0] = A / det;
  R[1] = -(b * i - c * h) / det;
  R[2] = (b * f - c * e) / det;
  R[3] = B / det;
  R[4] = (a * i - c * g) / det;
  R[5] = -(a * f - c * d) / det;
  R[6] = C / det;
  R[7] = -(a * h - b * g) / det;
  R[8] = (a * e - b * d) / det;
}

// (K^T K)^{-1} for points relative to centre (rows [1 0 -ry; 0 1 rx]).
void ktk_inv(const std::vector<Pt>& pts, double cx, double cy, double* out) {
  double M[9] = {0};
  for (const Pt& p : pts) {
    const double rx = p.x - cx, ry = p.y - cy;
    M[0] += 1;
    M[4] += 1;
    M[2] += -ry;
    M[6] += -ry;
    M[5] += rx;
    M[7] += rx;
    M[8] += rx * rx + ry * ry;
  }
  inv3(M, out);
}

struct DevMem {   // a per-batch device buffer of the context, freed at the end of its scope
  mfs_ctx* c = nullptr;
  void* p = nullptr;
  hipError_t alloc(mfs_ctx* ctx, size_t bytes) {
    c = ctx;
    return dev_malloc(c, &p, bytes);
  }
  ~DevMem() { dev_free(c, p); }
};

}  // namespace

// Tier distances of a class's ring expansion (hierarchical kernel sum).  For strengths
// sigma = G mu of the one-body map (G = (I - L) S_L^+ for mobility, P^+ for resistance; n x m,
// column-major) and |mu| = 1, the moments A_k = sum sigma w^k and B_k = sum sigma conj(w)^k
// are bounded by the norms of their rows a_k, b_k, and truncating the ring expansion after
// order p leaves at distance R at most
//   tail(p, R) = sum_{k > p} (|a_k| / (2k) + |b_k| / (2k) + |a_k|) R^-k
// (the three series of the ring expansion; k up to kmax, beyond which the ring's aliasing
// repeats the moments scaled by rho^nc).  The ring rule's small singular values make the top
// modes of sigma large, so this bound, not (rho / R)^p, sets the order near a disk.  For any
// other strengths the bound is sum |sigma| (rho / R)^(p+1) / (1 - rho / R).  The tier distance
// is the larger of the distances where the two meet tol and tol_theta; its square is stored.
static void ring_tiers(int nc, int m, const std::vector<double>& Yr, const std::vector<double>& G, const int* orders,
                       int ntier, double tol, double tol_theta, double* thr2) {
  const int kmax = std::min(2 * nc + 8, 320);
  std::vector<double> na(kmax + 1, 0.0), nb(kmax + 1, 0.0);
  std::vector<double> ar((size_t)(kmax + 1) * m, 0.0), ai(ar.size(), 0.0), br(ar.size(), 0.0), bi(ar.size(), 0.0);
  for (int s2 = 0; s2 < nc; ++s2) {
    const double wx = Yr[2 * s2], wy = Yr[2 * s2 + 1];
    double pr = 1.0, pi = 0.0;   // w^k
    for (int k = 0; k <= kmax; ++k) {
      for (int q = 0; q < m; ++q) {
        const double gx = G[(size_t)q * 2 * nc + 2 * s2], gy = G[(size_t)q * 2 * nc + 2 * s2 + 1];
        // sigma w^k and sigma conj(w)^k with sigma = gx + i gy
        ar[(size_t)k * m + q] += gx * pr - gy * pi;
        ai[(size_t)k * m + q] += gx * pi + gy * pr;
        br[(size_t)k * m + q] += gx * pr + gy * pi;
        bi[(size_t)k * m + q] += gy * pr - gx * pi;
      }
      const double t = pr * wx - pi * wy;
      pi = pr * wy + pi * wx;
      pr = t;
    }
  }
  for (int k = 0; k <= kmax; ++k) {
    double sa = 0.0, sb = 0.0;
    for (int q = 0; q < m; ++q) {
      sa += ar[(size_t)k * m + q] * ar[(size_t)k * m + q] + ai[(size_t)k * m + q] * ai[(size_t)k * m + q];
      sb += br[(size_t)k * m + q] * br[(size_t)k * m + q] + bi[(size_t)k * m + q] * bi[(size_t)k * m + q];
    }
    na[k] = std::sqrt(sa);
    nb[k] = std::sqrt(sb);
  }
  const double rho = std::sqrt(Yr[0] * Yr[0] + Yr[1] * Yr[1]);
  for (int t = 0; t < ntier; ++t) {
    const int p = orders[t];
    auto tail = [&](double R) {
      double e = 0.0;
      for (int k = p + 1; k <= kmax; ++k) e += ((na[k] + nb[k]) / (2.0 * k) + na[k]) * std::pow(R, -(double)k);
      return e;
    };
    double lo = rho * (1.0 + 1e-9), hi = 1e3 * std::max(rho, 1.0), R;
    if (tail(hi) > tol) {
      R = 1e150;   // never: the tier is not used
    } else {
      for (int it = 0; it < 100; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (tail(mid) > tol) lo = mid; else hi = mid;
      }
      R = std::max(hi, rho * std::pow(tol_theta, -1.0 / (p + 1)));
    }
    thr2[t] = R * R;
  }
  for (int t = 1; t < ntier; ++t) thr2[t] = std::min(thr2[t], thr2[t - 1]);
}

// ---------------------------------------------------------------------------
Status onebody_factors(mfs_ctx* c) {
  // distinct classes
  std::vector<int> first_of_class;
  c->cls.assign(c->P, -1);
  std::vector<std::array<double, 4>> keys;
  for (int i = 0; i < c->P; ++i) {
    std::array<double, 4> key{c->radii[i], (double)c->n_src[i], (double)c->n_col[i], c->r_src[i]};
    int k = -1;
    for (size_t q = 0; q < keys.size(); ++q)
      if (keys[q] == key) k = (int)q;
    if (k < 0) {
      if ((int)keys.size() == kMaxClasses)
        return Status{MFS_ERR_ARG, "more than 4 distinct disk classes (radius, n_src, n_col, r_src)"};
      keys.push_back(key);
      k = (int)keys.size() - 1;
    }
    c->cls[i] = k;
  }
  const double kscale = 1.0 / (4.0 * kPiD * c->prm.mu);
  for (int prob = 0; prob < 2; ++prob) {
    ClassTab& ct = c->ct[prob];
    ct.n = (int)keys.size();
    for (int k = 0; k < ct.n; ++k) {
      const double a = keys[k][0], rs = keys[k][3];
      const int nc = (int)keys[k][1], mc = (int)keys[k][2];
      std::vector<Pt> Y, X;
      ring_points({0, 0}, rs * a, nc, Y);
      ring_points({0, 0}, a, mc, X);
      const int m = 2 * mc, n = 2 * nc;
      // P = S(X, Y), column-major m x n
      std::vector<double> M((size_t)m * n);
      for (int q = 0; q < mc; ++q)
        for (int j = 0; j < nc; ++j) {
          const double dx = X[q].x - Y[j].x, dy = X[q].y - Y[j].y;
          const double r2 = dx * dx + dy * dy, lg = 0.5 * std::log(r2);
          M[(size_t)(2 * j) * m + 2 * q] = kscale * (dx * dx / r2 - lg);
          M[(size_t)(2 * j) * m + 2 * q + 1] = kscale * (dx * dy / r2);
          M[(size_t)(2 * j + 1) * m + 2 * q] = kscale * (dx * dy / r2);
          M[(size_t)(2 * j + 1) * m + 2 * q + 1] = kscale * (dy * dy / r2 - lg);
        }
      double KKi[9];
      ktk_inv(Y, 0, 0, KKi);
      if (prob == MFS_MOBILITY) {
        // S_L = P (I - L) + B K^T, L = K (K^T K)^{-1} K^T  (eq. SL)
        std::vector<double> K((size_t)n * 3), B((size_t)m * 3);  // row-major
        for (int j = 0; j < nc; ++j) {
          K[(2 * j) * 3 + 0] = 1; K[(2 * j) * 3 + 1] = 0; K[(2 * j) * 3 + 2] = -Y[j].y;
          K[(2 * j + 1) * 3 + 0] = 0; K[(2 * j + 1) * 3 + 1] = 1; K[(2 * j + 1) * 3 + 2] = Y[j].x;
        }
        for (int q = 0; q < mc; ++q) {
          B[(2 * q) * 3 + 0] = 1; B[(2 * q) * 3 + 1] = 0; B[(2 * q) * 3 + 2] = -X[q].y;
          B[(2 * q + 1) * 3 + 0] = 0; B[(2 * q + 1) * 3 + 1] = 1; B[(2 * q + 1) * 3 + 2] = X[q].x;
        }
        // W = (K^T K)^{-1} K^T (3 x n); PK = P K (m x 3)
        std::vector<double> W((size_t)3 * n), PK((size_t)m * 3, 0.0);
        for (int r = 0; r < 3; ++r)
          for (int j = 0; j < n; ++j) W[r * n + j] = KKi[r * 3 + 0] * K[j * 3 + 0] + KKi[r * 3 + 1] * K[j * 3 + 1] + KKi[r * 3 + 2] * K[j * 3 + 2];
        for (int row = 0; row < m; ++row)
          for (int r = 0; r < 3; ++r) {
            double s = 0;
            for (int j = 0; j < n; ++j) s += M[(size_t)j * m + row] * K[j * 3 + r];
            PK[row * 3 + r] = s;
          }
        for (int row = 0; row < m; ++row)
          for (int j = 0; j < n; ++j) {
            double v = M[(size_t)j * m + row];
            for (int r = 0; r < 3; ++r) v += -PK[row * 3 + r] * W[r * n + j] + B[row * 3 + r] * K[j * 3 + r];
            M[(size_t)j * m + row] = v;
          }
      }
      // SVD on the device
      const int mn = std::min(m, n);
      DevMem dA, dS, dU, dV, dE, dInfo;
      MFS_HIP(dA.alloc(c, sizeof(double) * m * n));
      MFS_HIP(dS.alloc(c, sizeof(double) * mn));
      MFS_HIP(dU.alloc(c, sizeof(double) * m * mn));
      MFS_HIP(dV.alloc(c, sizeof(double) * mn * n));
      MFS_HIP(dE.alloc(c, sizeof(double) * mn));
      MFS_HIP(dInfo.alloc(c, sizeof(int)));
      MFS_HIP(hipMemcpyAsync(dA.p, M.data(), sizeof(double) * m * n, hipMemcpyHostToDevice, c->stream));
      MFS_RB(svd_entry().gesvd(c->blas, rocblas_svect_singular, rocblas_svect_singular, m, n, (double*)dA.p, m,
                              (double*)dS.p, (double*)dU.p, m, (double*)dV.p, mn, (double*)dE.p,
                              rocblas_outofplace, (int*)dInfo.p));
      std::vector<double> S(mn), U((size_t)m * mn), VT((size_t)mn * n);
      int info = 0;
      MFS_HIP(hipMemcpyAsync(S.data(), dS.p, sizeof(double) * mn, hipMemcpyDeviceToHost, c->stream));
      MFS_HIP(hipMemcpyAsync(U.data(), dU.p, sizeof(double) * m * mn, hipMemcpyDeviceToHost, c->stream));
      MFS_HIP(hipMemcpyAsync(VT.data(), dV.p, sizeof(double) * mn * n, hipMemcpyDeviceToHost, c->stream));
      MFS_HIP(hipMemcpyAsync(&info, dInfo.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      MFS_HIP(hipStreamSynchronize(c->stream));
      if (info != 0) return Status{MFS_ERR_NUMERIC, "one-body SVD did not converge"};
      int rank = 0;
      while (rank < mn && S[rank] > S[0] * c->prm.eps_trunc) ++rank;
      {
        // G = Pi S^+ (n x m, column-major): V Sigma^+ U^T, then (I - L) per column for mobility
        std::vector<double> Gm((size_t)n * m, 0.0);
        for (int q = 0; q < m; ++q)
          for (int j = 0; j < rank; ++j) {
            const double f = U[(size_t)j * m + q] / S[j];
            for (int i = 0; i < n; ++i) Gm[(size_t)q * n + i] += VT[(size_t)i * mn + j] * f;
          }
        if (prob == MFS_MOBILITY)
          for (int q = 0; q < m; ++q) {
            double* col = Gm.data() + (size_t)q * n;
            double kt[3] = {0, 0, 0};
            for (int j = 0; j < nc; ++j) {
              kt[0] += col[2 * j];
              kt[1] += col[2 * j + 1];
              kt[2] += -Y[j].y * col[2 * j] + Y[j].x * col[2 * j + 1];
            }
            double cf[3];
            for (int r = 0; r < 3; ++r) cf[r] = KKi[3 * r] * kt[0] + KKi[3 * r + 1] * kt[1] + KKi[3 * r + 2] * kt[2];
            for (int j = 0; j < nc; ++j) {
              col[2 * j] -= cf[0] - cf[2] * Y[j].y;
              col[2 * j + 1] -= cf[1] + cf[2] * Y[j].x;
            }
          }
        std::vector<double> Yv(2 * nc);
        for (int j = 0; j < nc; ++j) {
          Yv[2 * j] = Y[j].x;
          Yv[2 * j + 1] = Y[j].y;
        }
        const int o64[kRingTiers] = {27, 40, kRing64Order}, o32[kRingTiers] = {14, 24, kRing32Order};
        ring_tiers(nc, m, Yv, Gm, o64, kRingTiers, 1e-15, 1e-16, ct.tier64[k]);
        ring_tiers(nc, m, Yv, Gm, o32, kRingTiers, 1e-9, 1e-9, ct.tier32[k]);
      }
      std::vector<double> Urm((size_t)m * rank), Vtrm((size_t)rank * n), sinv(rank);
      for (int q = 0; q < m; ++q)
        for (int j = 0; j < rank; ++j) Urm[(size_t)q * rank + j] = U[(size_t)j * m + q];
      for (int j = 0; j < rank; ++j) {
        sinv[j] = 1.0 / S[j];
        for (int i = 0; i < n; ++i) Vtrm[(size_t)j * n + i] = VT[(size_t)i * mn + j];
      }
      std::vector<double>& Yr = c->h_Yr[k];
      std::vector<double>& Xr = c->h_Xr[k];
      Yr.assign(2 * nc, 0.0);
      Xr.assign(2 * mc, 0.0);
      for (int j = 0; j < nc; ++j) {
        Yr[2 * j] = Y[j].x;
        Yr[2 * j + 1] = Y[j].y;
      }
      for (int q = 0; q < mc; ++q) {
        Xr[2 * q] = X[q].x;
        Xr[2 * q + 1] = X[q].y;
      }
      auto upload = [&](const std::vector<double>& h, const double** dst) -> Status {
        void* p = nullptr;
        MFS_HIP(dev_malloc(c, &p, sizeof(double) * std::max<size_t>(1, h.size())));
        c->class_bufs.push_back(p);
        MFS_HIP(hipMemcpy(p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
        *dst = (const double*)p;
        return Status{};
      };
      Status st;
      if ((st = upload(Urm, &ct.U[k])).code) return st;
      if ((st = upload(sinv, &ct.sinv[k])).code) return st;
      if ((st = upload(Vtrm, &ct.Vt[k])).code) return st;
      if ((st = upload(Yr, &ct.Yr[k])).code) return st;
      if ((st = upload(Xr, &ct.Xr[k])).code) return st;
      ct.nc[k] = nc;
      ct.mc[k] = mc;
      ct.rank[k] = rank;
      ct.radius[k] = a;
      std::memcpy(ct.KtKi[k], KKi, sizeof(KKi));
    }
  }
  return Status{};
}

// ---------------------------------------------------------------------------
Status precompute_pairs(mfs_ctx* c, int prob) {
  const int C = (int)(c->pairs.size() / 2);
  PairSet& ps = c->ps[prob];
  const int64_t asz = c->aoff[C], esz = 6 * c->xoff[C];
  if (!ps.A) {
    MFS_HIP(dev_malloc(c, &ps.A, sizeof(double) * std::max<int64_t>(1, asz)));
    MFS_HIP(dev_malloc(c, &ps.E, sizeof(double) * std::max<int64_t>(1, esz)));
  }
  if (C == 0) {
    ps.ready = true;
    return Status{};
  }
  FineParams fp{c->prm.n_fp, c->prm.n_ell, c->prm.m_p, c->prm.a_ell, c->prm.gamma, c->prm.a_f, c->prm.mobius_r,
                c->prm.eps_ring};
  const int mp = fp.m_p;
  const double kscale = 1.0 / (4.0 * kPiD * c->prm.mu);
  const int mobility = prob == MFS_MOBILITY ? 1 : 0;
  const ClassTab& ct = c->ct[prob];
  auto fine_nodes_of = [&](double a) { return (int)std::ceil(fp.a_f * fine_count(a, fp) - 1e-12) + fp.a_ell * fp.n_ell; };

  // Order pairs by (class of disk i, class of disk k, fine-source count): a batch holds one
  // class combination (equal matrix shapes) and pads little.
  std::vector<int> order(C), nfe0(C), nfe1(C);
  for (int p = 0; p < C; ++p) {
    const int i = c->pairs[2 * p], k = c->pairs[2 * p + 1];
    const double dx = c->centers[2 * k] - c->centers[2 * i], dy = c->centers[2 * k + 1] - c->centers[2 * i + 1];
    const double ai = c->radii[i], ak = c->radii[k], gap = std::sqrt(dx * dx + dy * dy) - ai - ak;
    nfe0[p] = fine_count(ai, fp) + ellipse_count(gap, fp, ai, ak);
    nfe1[p] = fine_count(ak, fp) + ellipse_count(gap, fp, ak, ai);
    order[p] = p;
  }
  auto type_of = [&](int p) { return c->cls[c->pairs[2 * p]] * kMaxClasses + c->cls[c->pairs[2 * p + 1]]; };
  // pairs of equal disks whose point sets the reflection through the midpoint maps onto each
  // other with the index maps of k_sym_split_F (checked on the constructed points) take the
  // split form: two SVDs of half the size
  std::vector<char> symp(C, 0);
  for (int p = 0; p < C; ++p) {
    const int i = c->pairs[2 * p], k = c->pairs[2 * p + 1];
    if (c->cls[i] != c->cls[k] || std::getenv("MFS_PRECOMPUTE_NOSYM")) continue;
    const double a = c->radii[i];
    const int nring = fine_count(a, fp), nnode = (int)std::ceil(fp.a_f * nring - 1e-12);
    if (nring % 2 || nnode % 2 || mp % 2 || ct.nc[c->cls[i]] % 2) continue;
    const Pt ci{c->centers[2 * i], c->centers[2 * i + 1]}, ck{c->centers[2 * k], c->centers[2 * k + 1]};
    std::vector<Pt> yi, yk, xi, xk, z;
    pair_fine_sources(ci, ck, fp, yi, yk, a, a);
    pair_fine_nodes(ci, ck, fp, xi, xk, a, a);
    peanut(ci, ck, mp, z, a, a);
    if (yi.size() != yk.size() || xi.size() != xk.size() || (int)xi.size() < nnode) continue;
    const double sx = ci.x + ck.x, sy = ci.y + ck.y, tol = 1e-11 * (1.0 + std::fabs(sx) + std::fabs(sy));
    auto mirror = [&](Pt u, Pt v) { return std::fabs(u.x + v.x - sx) <= tol && std::fabs(u.y + v.y - sy) <= tol; };
    bool ok = true;
    for (size_t j = 0; ok && j < yi.size(); ++j)
      ok = mirror(yi[j], yk[(int)j < nring ? ((int)j + nring / 2) % nring : (int)j]);
    for (size_t j = 0; ok && j < xi.size(); ++j)
      ok = mirror(xi[j], xk[(int)j < nnode ? ((int)j + nnode / 2) % nnode : (int)j]);
    for (int j = 0; ok && j < mp / 2; ++j) ok = mirror(z[j], z[j + mp / 2]);
    symp[p] = ok ? 1 : 0;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    if (type_of(a) != type_of(b)) return type_of(a) < type_of(b);
    if (symp[a] != symp[b]) return symp[a] > symp[b];
    return std::max(nfe0[a], nfe1[a]) < std::max(nfe0[b], nfe1[b]);
  });
  double rmax = 0.0;
  for (int i = 0; i < c->P; ++i) rmax = std::max(rmax, c->radii[i]);
  const int mf = fine_nodes_of(rmax);

  // Fine factors for flow evaluation: each pair's G (compact rows), fine points, fine
  // (K^T K)^{-1} and peanut geometry, kept when the context asks for them.
  for (void** q : {(void**)&ps.G, (void**)&ps.Yf, (void**)&ps.KKf, (void**)&ps.pgeo, (void**)&ps.nf,
                   (void**)&ps.d_goff, (void**)&ps.d_yoff}) {
    if (*q) dev_free(c, *q);
    *q = nullptr;
  }
  ps.fine = false;
  const bool keep = c->keep_fine;
  std::vector<double> h_Yf, h_KKf, h_pgeo;
  std::vector<int32_t> h_nf;
  if (keep) {
    ps.goff.assign(C + 1, 0);
    ps.yoff.assign(C + 1, 0);
    for (int p = 0; p < C; ++p) {
      const int64_t nfr = 2 * (int64_t)(nfe0[p] + nfe1[p]);
      ps.goff[p + 1] = ps.goff[p] + nfr * (c->xoff[p + 1] - c->xoff[p]);
      ps.yoff[p + 1] = ps.yoff[p] + nfr;
    }
    MFS_HIP(dev_malloc(c, &ps.G, sizeof(double) * std::max<int64_t>(1, ps.goff[C])));
    h_Yf.assign(ps.yoff[C], 0.0);
    h_KKf.assign(18 * (size_t)C, 0.0);
    h_pgeo.assign(12 * (size_t)C, 0.0);
    h_nf.assign(2 * (size_t)C, 0);
  }

  const bool prof = std::getenv("MFS_PROFILE") != nullptr;
  double tstage[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  auto tick = [&](int k, std::chrono::steady_clock::time_point& t0) {
    if (!prof) return;
    (void)hipStreamSynchronize(c->stream);
    auto t1 = std::chrono::steady_clock::now();
    tstage[k] += std::chrono::duration<double>(t1 - t0).count();
    t0 = t1;
  };
  // Batched SVDs are latency-bound at small batch counts: size the batch from free
  // device memory (about 40 MB of work space per pair at the paper's fine grids).
  int batch = 32;
  {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
      const int nfmax = fine_count(rmax, fp) + 2 * fp.n_ell;
      const double per_pair = 8.0 * (2.0 * (4.0 * mf) * (4.0 * nfmax) + 2.0 * (4.0 * nfmax) * (4.0 * nfmax) +
                                     6.0 * (4.0 * mf + 2.0 * mp) * 4.0 * kMaxCol / 4.0);
      const double cap = 0.5 * (double)free_b / per_pair;
      batch = (int)std::max(1.0, std::min(256.0, cap));
    }
    if (c->pre_batch > 0) batch = c->pre_batch;
    const char* env = std::getenv("MFS_PRECOMPUTE_BATCH");
    if (env) batch = std::max(1, std::atoi(env));
  }
  for (int b0 = 0; b0 < C;) {
    auto t0 = std::chrono::steady_clock::now();
    int nb = 0;
    while (nb < batch && b0 + nb < C && type_of(order[b0 + nb]) == type_of(order[b0]) &&
           symp[order[b0 + nb]] == symp[order[b0]])
      ++nb;
    const bool sym = symp[order[b0]] != 0;
    const int ci0 = c->cls[c->pairs[2 * order[b0]]], ck0 = c->cls[c->pairs[2 * order[b0] + 1]];
    BatchDims d;
    d.nfpad[0] = d.nfpad[1] = 0;
    for (int q = 0; q < nb; ++q) {
      d.nfpad[0] = std::max(d.nfpad[0], nfe0[order[b0 + q]]);
      d.nfpad[1] = std::max(d.nfpad[1], nfe1[order[b0 + q]]);
    }
    d.nc[0] = ct.nc[ci0];
    d.nc[1] = ct.nc[ck0];
    d.mf[0] = fine_nodes_of(ct.radius[ci0]);
    d.mf[1] = fine_nodes_of(ct.radius[ck0]);
    d.mp = mp;
    d.ldF = 2 * (d.mf[0] + d.mf[1]);
    d.ldD = 2 * mp;
    const int64_t m = d.ldF, n = 2 * (d.nfpad[0] + d.nfpad[1]), nx = 2 * (d.nc[0] + d.nc[1]), mpp = 2 * mp;
    d.sF = m * (n + nx);   // [F X] of a pair side by side, leading dimension m (X at column n)
    d.sX = d.sF;
    d.sD = mpp * n;
    d.sC = mpp * nx;
    // host staging: geometry
    const int64_t per_pair = 2 * (d.nfpad[0] + d.nfpad[1]) + 2 * (d.nc[0] + d.nc[1]) + 2 * (d.mf[0] + d.mf[1]) + 2 * mp;
    std::vector<double> stage((size_t)per_pair * nb, 0.0);
    std::vector<PairGeo> geo(nb);
    DevMem dstage, dgeo;
    MFS_HIP(dstage.alloc(c, sizeof(double) * stage.size()));
    MFS_HIP(dgeo.alloc(c, sizeof(PairGeo) * nb));
    const double* dbase = (const double*)dstage.p;
    std::vector<int64_t> eoff(nb);
    for (int q = 0; q < nb; ++q) {
      const int p = order[b0 + q];
      const int i = c->pairs[2 * p], k = c->pairs[2 * p + 1];
      const Pt ci{c->centers[2 * i], c->centers[2 * i + 1]}, ck{c->centers[2 * k], c->centers[2 * k + 1]};
      const double ai = c->radii[i], ak = c->radii[k];
      std::vector<Pt> yi, yk, xi, xk, z;
      pair_fine_sources(ci, ck, fp, yi, yk, ai, ak);
      pair_fine_nodes(ci, ck, fp, xi, xk, ai, ak);
      peanut(ci, ck, mp, z, ai, ak);
      if ((int)xi.size() != d.mf[0] || (int)xk.size() != d.mf[1] || (int)yi.size() > d.nfpad[0] ||
          (int)yk.size() > d.nfpad[1])
        return Status{MFS_ERR_ARG, "pair fine set sizes disagree with the batch dimensions"};
      double* base = stage.data() + (size_t)q * per_pair;
      const int64_t o_yf0 = 0, o_yf1 = 2 * d.nfpad[0], o_yc0 = o_yf1 + 2 * d.nfpad[1], o_yc1 = o_yc0 + 2 * d.nc[0],
                    o_xf = o_yc1 + 2 * d.nc[1], o_z = o_xf + 2 * (d.mf[0] + d.mf[1]);
      for (size_t s = 0; s < yi.size(); ++s) {
        base[o_yf0 + 2 * s] = yi[s].x;
        base[o_yf0 + 2 * s + 1] = yi[s].y;
      }
      for (size_t s = 0; s < yk.size(); ++s) {
        base[o_yf1 + 2 * s] = yk[s].x;
        base[o_yf1 + 2 * s + 1] = yk[s].y;
      }
      const std::vector<double>& yri = c->h_Yr[c->cls[i]];
      const std::vector<double>& yrk = c->h_Yr[c->cls[k]];
      for (int s = 0; s < d.nc[0]; ++s) {
        base[o_yc0 + 2 * s] = ci.x + yri[2 * s];
        base[o_yc0 + 2 * s + 1] = ci.y + yri[2 * s + 1];
      }
      for (int s = 0; s < d.nc[1]; ++s) {
        base[o_yc1 + 2 * s] = ck.x + yrk[2 * s];
        base[o_yc1 + 2 * s + 1] = ck.y + yrk[2 * s + 1];
      }
      for (int s = 0; s < d.mf[0]; ++s) {
        base[o_xf + 2 * s] = xi[s].x;
        base[o_xf + 2 * s + 1] = xi[s].y;
      }
      for (int s = 0; s < d.mf[1]; ++s) {
        base[o_xf + 2 * d.mf[0] + 2 * s] = xk[s].x;
        base[o_xf + 2 * d.mf[0] + 2 * s + 1] = xk[s].y;
      }
      for (int s = 0; s < mp; ++s) {
        base[o_z + 2 * s] = z[s].x;
        base[o_z + 2 * s + 1] = z[s].y;
      }
      PairGeo& g = geo[q];
      const double* db = dbase + (size_t)q * per_pair;
      g.yf[0] = db + o_yf0;
      g.yf[1] = db + o_yf1;
      g.yc[0] = db + o_yc0;
      g.yc[1] = db + o_yc1;
      g.xf = db + o_xf;
      g.z = db + o_z;
      g.nf[0] = (int)yi.size();
      g.nf[1] = (int)yk.size();
      g.c[0][0] = ci.x;
      g.c[0][1] = ci.y;
      g.c[1][0] = ck.x;
      g.c[1][1] = ck.y;
      ktk_inv(yi, ci.x, ci.y, g.KKf[0]);
      ktk_inv(yk, ck.x, ck.y, g.KKf[1]);
      std::memcpy(g.KKc[0], ct.KtKi[c->cls[i]], sizeof(g.KKc[0]));
      std::memcpy(g.KKc[1], ct.KtKi[c->cls[k]], sizeof(g.KKc[1]));
      eoff[q] = 6 * c->xoff[p];
      if (keep) {
        if ((int)yi.size() != nfe0[p] || (int)yk.size() != nfe1[p])
          return Status{MFS_ERR_ARG, "pair fine source counts disagree with the fine rules"};
        double* yf = h_Yf.data() + ps.yoff[p];
        for (size_t s2 = 0; s2 < yi.size(); ++s2) {
          yf[2 * s2] = yi[s2].x;
          yf[2 * s2 + 1] = yi[s2].y;
        }
        yf += 2 * yi.size();
        for (size_t s2 = 0; s2 < yk.size(); ++s2) {
          yf[2 * s2] = yk[s2].x;
          yf[2 * s2 + 1] = yk[s2].y;
        }
        std::memcpy(h_KKf.data() + 18 * (size_t)p, g.KKf[0], 9 * sizeof(double));
        std::memcpy(h_KKf.data() + 18 * (size_t)p + 9, g.KKf[1], 9 * sizeof(double));
        // peanut: rolling unit circle centred s along the axis and h off it (both sides)
        const double dx = ck.x - ci.x, dy = ck.y - ci.y, dd = std::sqrt(dx * dx + dy * dy);
        const double ex = dx / dd, ey = dy / dd;
        const double sh = ((ai + 1.0) * (ai + 1.0) - (ak + 1.0) * (ak + 1.0) + dd * dd) / (2.0 * dd);
        const double hh = std::sqrt((ai + 1.0) * (ai + 1.0) - sh * sh);
        double* pg = h_pgeo.data() + 12 * (size_t)p;
        const double pv[12] = {ci.x, ci.y, ck.x, ck.y, ai, ak, ci.x + sh * ex + hh * ey, ci.y + sh * ey - hh * ex,
                               ci.x + sh * ex - hh * ey, ci.y + sh * ey + hh * ex};
        std::memcpy(pg, pv, sizeof(pv));
        h_nf[2 * p] = nfe0[p];
        h_nf[2 * p + 1] = nfe1[p];
      }
    }
    MFS_HIP(hipMemcpyAsync(dstage.p, stage.data(), sizeof(double) * stage.size(), hipMemcpyHostToDevice, c->stream));
    MFS_HIP(hipMemcpyAsync(dgeo.p, geo.data(), sizeof(PairGeo) * nb, hipMemcpyHostToDevice, c->stream));
    DevMem deoff;
    MFS_HIP(deoff.alloc(c, sizeof(int64_t) * nb));
    MFS_HIP(hipMemcpyAsync(deoff.p, eoff.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, c->stream));

    DevMem dFX, dD, dC, dG, dDG, dSC, dUC, dVTC, dEC, dT2, dinfo, dinfoC;
    MFS_HIP(dFX.alloc(c, sizeof(double) * d.sF * nb));
    double* const pF = (double*)dFX.p;
    double* const pX = pF + m * n;
    MFS_HIP(dD.alloc(c, sizeof(double) * d.sD * nb));
    MFS_HIP(dC.alloc(c, sizeof(double) * d.sC * nb));
    MFS_HIP(hipMemsetAsync(dFX.p, 0, sizeof(double) * d.sF * nb, c->stream));
    MFS_HIP(hipMemsetAsync(dD.p, 0, sizeof(double) * d.sD * nb, c->stream));
    tick(0, t0);
    {
      const int maxpts = std::max(d.mf[0] + d.mf[1], mp);
      dim3 grid((maxpts + 63) / 64, nb, 4);
      hipLaunchKernelGGL(k_fill, grid, dim3(64), 0, c->stream, (const PairGeo*)dgeo.p, d, mobility, kscale, pF, pX,
                         (double*)dD.p, (double*)dC.p);
      MFS_HIP(hipGetLastError());
    }
    tick(1, t0);
    const double one = 1.0, zero = 0.0, mone = -1.0;
    const int nbs = sym ? 2 * nb : nb;   // matrices per SVD batch
    // index maps of the split form: the rings of disk i's fine sources and fine nodes
    const int sym_nsrc = fine_count(ct.radius[ci0], fp);
    const int sym_nnode = (int)std::ceil(fp.a_f * sym_nsrc - 1e-12);
    MFS_HIP(dinfo.alloc(c, sizeof(int) * nbs));
    MFS_HIP(dinfoC.alloc(c, sizeof(int) * nbs));
    MFS_HIP(dG.alloc(c, sizeof(double) * n * nx * nb));
    // G = F^+ X with the truncated pseudoinverse (singular values below eps_trunc_fine times the
    // largest of the group's matrices dropped) for nmat matrices A = [F X] (rows x (cols + nx),
    // leading dimension rows, stride sA; A is overwritten).  A tall F first goes through a
    // Householder QR of the whole of A, F = Q1 R, whose last nx columns become Q1^T X: F and R
    // share their singular values and right vectors, and U_F = Q1 U_R, so
    // G = V Sigma^+ U_R^T (Q1^T X) and the SVD is of the cols x cols factor R alone.
    auto pinv_apply = [&](double* A, int64_t rows, int64_t cols, int64_t sA, int nmat, int group,
                          double* G) -> Status {
      DevMem dTau, dR, dT0, dS, dU, dVT, dE, dT1;
      double *svA = A, *Xp = A + rows * cols;
      int64_t sr = rows, ssv = sA, ldx = rows, sx = sA;
      if (rows >= cols) {
        const int64_t kq = std::min(rows, cols + nx);
        MFS_HIP(dTau.alloc(c, sizeof(double) * kq * nmat));
        MFS_HIP(dR.alloc(c, sizeof(double) * cols * cols * nmat));
        MFS_HIP(dT0.alloc(c, sizeof(double) * cols * nx * nmat));
        MFS_RB(svd_entry().geqrf_sb(c->blas, (int)rows, (int)(cols + nx), A, (int)rows, sA, (double*)dTau.p, kq,
                                    nmat));
        hipLaunchKernelGGL(k_split_qr, dim3((unsigned)(cols + nx), nmat), dim3(256), 0, c->stream, A, rows, sA,
                           (int)cols, (int)nx, (double*)dR.p, (double*)dT0.p);
        MFS_HIP(hipGetLastError());
        svA = (double*)dR.p;
        Xp = (double*)dT0.p;
        sr = cols;
        ssv = cols * cols;
        ldx = cols;
        sx = cols * nx;
      }
      const int64_t k = std::min(sr, cols);
      MFS_HIP(dS.alloc(c, sizeof(double) * k * nmat));
      MFS_HIP(dU.alloc(c, sizeof(double) * sr * k * nmat));
      MFS_HIP(dVT.alloc(c, sizeof(double) * k * cols * nmat));
      MFS_HIP(dE.alloc(c, sizeof(double) * k * nmat));
      MFS_HIP(dT1.alloc(c, sizeof(double) * k * nx * nmat));
      MFS_RB(svd_entry().gesvd_sb(c->blas, rocblas_svect_singular, rocblas_svect_singular, (int)sr, (int)cols, svA,
                                  (int)sr, ssv, (double*)dS.p, k, (double*)dU.p, (int)sr, sr * k, (double*)dVT.p,
                                  (int)k, k * cols, (double*)dE.p, k, rocblas_outofplace, (int*)dinfo.p, nmat));
      if (prof) {
        const double before = tstage[2];
        tick(2, t0);
        std::fprintf(stderr, "[mfs precompute] F %lld x %lld -> SVD %lld x %lld, %d matrices: %.3f s\n",
                     (long long)rows, (long long)cols, (long long)sr, (long long)cols, nmat, tstage[2] - before);
      }
      // T1 = U^T (Q1^T X), scaled by the kept 1 / sigma_j; G = V T1
      MFS_RB(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_transpose, rocblas_operation_none, (int)k,
                                           (int)nx, (int)sr, &one, (const double*)dU.p, (int)sr, sr * k,
                                           (const double*)Xp, (int)ldx, sx, &zero, (double*)dT1.p, (int)k, k * nx,
                                           nmat));
      {
        dim3 grid((unsigned)((k * nx + 255) / 256), nmat);
        hipLaunchKernelGGL(k_trunc_scale, grid, dim3(256), 0, c->stream, (int)k, (const double*)dS.p, k,
                           c->prm.eps_trunc_fine, (double*)dT1.p, k, (int)nx, k * nx, group);
        MFS_HIP(hipGetLastError());
      }
      MFS_RB(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_transpose, rocblas_operation_none, (int)cols,
                                           (int)nx, (int)k, &one, (const double*)dVT.p, (int)k, k * cols,
                                           (const double*)dT1.p, (int)k, k * nx, &zero, G, (int)cols, cols * nx,
                                           nmat));
      MFS_HIP(hipStreamSynchronize(c->stream));   // the work buffers are released at the end of this scope
      return Status{};
    };
    if (sym) {
      // [F_e X_e] (mh x (nh + nx)), e = +, -: half the rows and columns
      const int64_t mh = m / 2, nh = n / 2;
      DevMem dFXs, dGs;
      MFS_HIP(dFXs.alloc(c, sizeof(double) * mh * (nh + nx) * nbs));
      hipLaunchKernelGGL(k_sym_split_F, dim3((unsigned)(nh + nx), nbs), dim3(256), 0, c->stream, (const double*)pF,
                         m, d.sF, (const double*)pX, d.sX, (int)mh, (int)nh, (int)nx, sym_nsrc, sym_nnode,
                         (double*)dFXs.p);
      MFS_HIP(hipGetLastError());
      MFS_HIP(dGs.alloc(c, sizeof(double) * nh * nx * nbs));
      tick(7, t0);
      Status st = pinv_apply((double*)dFXs.p, mh, nh, mh * (nh + nx), nbs, 2, (double*)dGs.p);
      if (st.code != MFS_OK) return st;
      hipLaunchKernelGGL(k_sym_join_G, dim3((unsigned)nx, nb), dim3(256), 0, c->stream, (const double*)dGs.p, (int)nh,
                         (int)nx, sym_nsrc, (double*)dG.p, n * nx);
      MFS_HIP(hipGetLastError());
      MFS_HIP(hipStreamSynchronize(c->stream));   // the split buffers are released at the end of this scope
    } else {
      Status st = pinv_apply(pF, m, n, d.sF, nb, 1, (double*)dG.p);
      if (st.code != MFS_OK) return st;
    }
    tick(3, t0);
    if (keep) {
      std::vector<int32_t> nfq(2 * nb);
      std::vector<int64_t> gq(nb);
      for (int q = 0; q < nb; ++q) {
        nfq[2 * q] = nfe0[order[b0 + q]];
        nfq[2 * q + 1] = nfe1[order[b0 + q]];
        gq[q] = ps.goff[order[b0 + q]];
      }
      DevMem dnfq, dgq;
      MFS_HIP(dnfq.alloc(c, sizeof(int32_t) * 2 * nb));
      MFS_HIP(dgq.alloc(c, sizeof(int64_t) * nb));
      MFS_HIP(hipMemcpyAsync(dnfq.p, nfq.data(), sizeof(int32_t) * 2 * nb, hipMemcpyHostToDevice, c->stream));
      MFS_HIP(hipMemcpyAsync(dgq.p, gq.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, c->stream));
      hipLaunchKernelGGL(k_store_fine, dim3((unsigned)nx, nb), dim3(256), 0, c->stream, (int)nx, d.nfpad[0],
                         (const int32_t*)dnfq.p, (const double*)dG.p, n * nx, n, ps.G, (const int64_t*)dgq.p);
      MFS_HIP(hipGetLastError());
      MFS_HIP(hipStreamSynchronize(c->stream));   // nfq, gq are released at the end of this scope
    }
    // DG = D G  (2mp x nx)
    MFS_HIP(dDG.alloc(c, sizeof(double) * mpp * nx * nb));
    MFS_RB(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none, rocblas_operation_none, (int)mpp, (int)nx,
                                         (int)n, &one, (const double*)dD.p, (int)mpp, d.sD, (const double*)dG.p,
                                         (int)n, n * nx, &zero, (double*)dDG.p, (int)mpp, mpp * nx, nb));
    tick(3, t0);
    // SVD of C (2mp x nx), then A = -V_C Sigma_C^+ U_C^T (D G)
    if (sym) {
      const int64_t zh = mp, nxh = nx / 2, mnc = std::min(zh, nxh);
      const int ncc = ct.nc[ci0];
      std::vector<int64_t> aq(nb);
      for (int q = 0; q < nb; ++q) aq[q] = c->aoff[order[b0 + q]];
      DevMem dCs, dDGs, dAs, daq;
      MFS_HIP(dCs.alloc(c, sizeof(double) * zh * nxh * nbs));
      MFS_HIP(dDGs.alloc(c, sizeof(double) * zh * nx * nbs));
      MFS_HIP(daq.alloc(c, sizeof(int64_t) * nb));
      MFS_HIP(hipMemcpyAsync(daq.p, aq.data(), sizeof(int64_t) * nb, hipMemcpyHostToDevice, c->stream));
      hipLaunchKernelGGL(k_sym_split_C, dim3((unsigned)(nxh + nx), nbs), dim3(256), 0, c->stream, (const double*)dC.p,
                         d.sC, (const double*)dDG.p, mpp * nx, (int)zh, (int)nxh, (int)nx, ncc, (double*)dCs.p,
                         (double*)dDGs.p);
      MFS_HIP(hipGetLastError());
      MFS_HIP(dSC.alloc(c, sizeof(double) * mnc * nbs));
      MFS_HIP(dUC.alloc(c, sizeof(double) * zh * mnc * nbs));
      MFS_HIP(dVTC.alloc(c, sizeof(double) * mnc * nxh * nbs));
      MFS_HIP(dEC.alloc(c, sizeof(double) * mnc * nbs));
      MFS_RB(svd_entry().gesvd_sb(c->blas, rocblas_svect_singular, rocblas_svect_singular, (int)zh,
                                              (int)nxh, (double*)dCs.p, (int)zh, zh * nxh, (double*)dSC.p, mnc,
                                              (double*)dUC.p, (int)zh, zh * mnc, (double*)dVTC.p, (int)mnc,
                                              mnc * nxh, (double*)dEC.p, mnc, rocblas_outofplace, (int*)dinfoC.p, nbs));
      tick(4, t0);
      MFS_HIP(dT2.alloc(c, sizeof(double) * mnc * nx * nbs));
      MFS_HIP(dAs.alloc(c, sizeof(double) * nxh * nx * nbs));
      MFS_RB(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_transpose, rocblas_operation_none, (int)mnc,
                                           (int)nx, (int)zh, &one, (const double*)dUC.p, (int)zh, zh * mnc,
                                           (const double*)dDGs.p, (int)zh, zh * nx, &zero, (double*)dT2.p, (int)mnc,
                                           mnc * nx, nbs));
      {
        dim3 grid((unsigned)((mnc * nx + 255) / 256), nbs);
        hipLaunchKernelGGL(k_trunc_scale, grid, dim3(256), 0, c->stream, (int)mnc, (const double*)dSC.p, mnc,
                           c->prm.eps_trunc, (double*)dT2.p, mnc, (int)nx, mnc * nx, 2);
      }
      MFS_RB(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_transpose, rocblas_operation_none, (int)nxh,
                                           (int)nx, (int)mnc, &mone, (const double*)dVTC.p, (int)mnc, mnc * nxh,
                                           (const double*)dT2.p, (int)mnc, mnc * nx, &zero, (double*)dAs.p, (int)nxh,
                                           nxh * nx, nbs));
      hipLaunchKernelGGL(k_sym_join_A, dim3((unsigned)nx, nb), dim3(256), 0, c->stream, (const double*)dAs.p,
                         (int)nxh, (int)nx, ncc, ps.A, (const int64_t*)daq.p);
      MFS_HIP(hipGetLastError());
      MFS_HIP(hipStreamSynchronize(c->stream));   // the split buffers are released at the end of this scope
    } else {
      const int64_t mnc = std::min(mpp, nx);
      MFS_HIP(dSC.alloc(c, sizeof(double) * mnc * nb));
      MFS_HIP(dUC.alloc(c, sizeof(double) * mpp * mnc * nb));
      MFS_HIP(dVTC.alloc(c, sizeof(double) * mnc * nx * nb));
      MFS_HIP(dEC.alloc(c, sizeof(double) * mnc * nb));
      MFS_RB(svd_entry().gesvd_sb(c->blas, rocblas_svect_singular, rocblas_svect_singular, (int)mpp,
                                              (int)nx, (double*)dC.p, (int)mpp, d.sC, (double*)dSC.p, mnc,
                                              (double*)dUC.p, (int)mpp, mpp * mnc, (double*)dVTC.p, (int)mnc,
                                              mnc * nx, (double*)dEC.p, mnc, rocblas_outofplace, (int*)dinfoC.p, nb));
      tick(4, t0);
      MFS_HIP(dT2.alloc(c, sizeof(double) * mnc * nx * nb));
      MFS_RB(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_transpose, rocblas_operation_none, (int)mnc,
                                           (int)nx, (int)mpp, &one, (const double*)dUC.p, (int)mpp, mpp * mnc,
                                           (const double*)dDG.p, (int)mpp, mpp * nx, &zero, (double*)dT2.p, (int)mnc,
                                           mnc * nx, nb));
      {
        dim3 grid((unsigned)((mnc * nx + 255) / 256), nb);
        hipLaunchKernelGGL(k_trunc_scale, grid, dim3(256), 0, c->stream, (int)mnc, (const double*)dSC.p, mnc,
                           c->prm.eps_trunc, (double*)dT2.p, mnc, (int)nx, mnc * nx, 1);
      }
      // A into place; pairs of a batch are not contiguous in the pair order, so one GEMM per pair
      for (int q = 0; q < nb; ++q) {
        const int p = order[b0 + q];
        MFS_RB(rocblas_dgemm(c->blas, rocblas_operation_transpose, rocblas_operation_none, (int)nx, (int)nx,
                             (int)mnc, &mone, (const double*)dVTC.p + q * mnc * nx, (int)mnc,
                             (const double*)dT2.p + q * mnc * nx, (int)mnc, &zero, ps.A + c->aoff[p], (int)nx));
      }
    }
    {
      dim3 grid((unsigned)((nx + 63) / 64), nb);
      hipLaunchKernelGGL(k_extract, grid, dim3(64), 0, c->stream, (const PairGeo*)dgeo.p, d, (const double*)dG.p,
                         n * nx, mobility ? 1.0 : -1.0, ps.E, (const int64_t*)deoff.p);
    }
    std::vector<int> info(2 * nbs);
    MFS_HIP(hipMemcpyAsync(info.data(), dinfo.p, sizeof(int) * nbs, hipMemcpyDeviceToHost, c->stream));
    MFS_HIP(hipMemcpyAsync(info.data() + nbs, dinfoC.p, sizeof(int) * nbs, hipMemcpyDeviceToHost, c->stream));
    MFS_HIP(hipStreamSynchronize(c->stream));
    for (int q = 0; q < 2 * nbs; ++q)
      if (info[q] != 0) return Status{MFS_ERR_NUMERIC, "pair SVD did not converge"};
    tick(5, t0);
    if (prof) std::fprintf(stderr, "[mfs precompute] %d / %d pairs (batch %d)\n", b0 + nb, C, batch);
    b0 += nb;
  }
  if (prof)
    std::fprintf(stderr, "[mfs precompute] pairs %d: host+upload %.3fs fill %.3fs split %.3fs svdF %.3fs gemm %.3fs "
                 "svdC %.3fs rest %.3fs (rocSOLVER: %s)\n",
                 C, tstage[0], tstage[1], tstage[7], tstage[2], tstage[3], tstage[4], tstage[5], svd_entry().origin);
  if (keep) {
    auto up = [&](void** dst, const void* src, size_t bytes) -> Status {
      MFS_HIP(dev_malloc(c, dst, std::max<size_t>(bytes, 8)));
      if (bytes) MFS_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
      return Status{};
    };
    Status st;
    if ((st = up((void**)&ps.Yf, h_Yf.data(), sizeof(double) * h_Yf.size())).code) return st;
    if ((st = up((void**)&ps.KKf, h_KKf.data(), sizeof(double) * h_KKf.size())).code) return st;
    if ((st = up((void**)&ps.pgeo, h_pgeo.data(), sizeof(double) * h_pgeo.size())).code) return st;
    if ((st = up((void**)&ps.nf, h_nf.data(), sizeof(int32_t) * h_nf.size())).code) return st;
    if ((st = up((void**)&ps.d_goff, ps.goff.data(), sizeof(int64_t) * ps.goff.size())).code) return st;
    if ((st = up((void**)&ps.d_yoff, ps.yoff.data(), sizeof(int64_t) * ps.yoff.size())).code) return st;
    ps.fine = true;
  }
  ps.ready = true;
  return Status{};
}

}  // namespace mfs
