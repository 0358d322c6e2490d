// gfx950 kernels of the matvec T mu (Alg. 3), the right-hand side, the
// post-processing and the GMRES vector operations.
//
// Layout: per-node and per-source 2-vectors are (x, y) interleaved, bodies in
// order (offsets src_off / col_off).  Every reduction over several producers
// (pair contributions to a body, source splits of the kernel sum, block partials
// of a dot product) runs in a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>

#include "internal.h"

// Scratch of mfs_apply_noalloc: the kernel sum's split partials for callers that cannot
// allocate device memory.  One copy per device, held until the process ends; host code
// uses the address hipGetSymbolAddress returns for the current device, never this name.
static __device__ __align__(256) double scratch[mfs::kScratchDoubles];

namespace mfs {

namespace {

constexpr int kBodyThreads = 128;

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Work counters of a kernel-sum launch: each wave adds its lanes' counts (direct pair
// evaluations, disk expansions, cluster expansions, cluster-to-local translations, local
// expansion evaluations) to work[0..4] with one atomic each.
__device__ __forceinline__ void add_work(unsigned long long* work, unsigned d, unsigned e, unsigned c, unsigned m,
                                         unsigned l) {
  if (!work) return;
  for (int off = 32; off > 0; off >>= 1) {
    d += __shfl_down(d, off, 64);
    e += __shfl_down(e, off, 64);
    c += __shfl_down(c, off, 64);
    m += __shfl_down(m, off, 64);
    l += __shfl_down(l, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(work, (unsigned long long)d);
    atomicAdd(work + 1, (unsigned long long)e);
    atomicAdd(work + 2, (unsigned long long)c);
    atomicAdd(work + 3, (unsigned long long)m);
    atomicAdd(work + 4, (unsigned long long)l);
  }
}

// Sum over a block of up to 1024 threads; every thread gets the result.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
  static_assert(NT % 64 == 0 && NT <= 1024, "block size");
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += red[w];
  return s;
}

// Natural log of a normal FP64 x > 0.  x = m 2^e with m in [1/sqrt 2, sqrt 2) (frexp),
// ln m = 2 artanh(f) = 2 f (1 + f^2/3 + ... + f^18/19), f = (m - 1)/(m + 1), |f| <= 0.172:
// the truncated series is below 3e-17 relative; ln 2 is split so e ln2_hi is exact.
__device__ __forceinline__ double ln_f64(double x) {
  double m = __builtin_amdgcn_frexp_mant(x);
  int e = __builtin_amdgcn_frexp_exp(x);
  const bool lo = m < 0.70710678118654752440;
  m = lo ? 2.0 * m : m;
  e = lo ? e - 1 : e;
  const double d = m + 1.0;
  double r = __builtin_amdgcn_rcp(d);
  r = fma(fma(-d, r, 1.0), r, r);
  const double f = (m - 1.0) * r;
  const double s = f * f;
  double p = 1.0 / 19.0;
  p = fma(p, s, 1.0 / 17.0);
  p = fma(p, s, 1.0 / 15.0);
  p = fma(p, s, 1.0 / 13.0);
  p = fma(p, s, 1.0 / 11.0);
  p = fma(p, s, 1.0 / 9.0);
  p = fma(p, s, 1.0 / 7.0);
  p = fma(p, s, 1.0 / 5.0);
  p = fma(p, s, 1.0 / 3.0);
  p = fma(p, s, 1.0);
  const double ln2_hi = 6.93147180369123816490e-01, ln2_lo = 1.90821492927058770002e-10;
  const double de = (double)e;
  return fma(de, ln2_hi, fma(de, ln2_lo, 2.0 * f * p));
}

// 1/x for normal FP64 x: hardware reciprocal and one Newton step.
__device__ __forceinline__ double rcp_f64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  return fma(fma(-x, r, 1.0), r, r);
}

// In-place (I - L) of a body's source strengths held in LDS: lambda - K (K^T K)^{-1} K^T lambda,
// with K rows [1, 0, -yr_y; 0, 1, yr_x] (eq. Kmat, Sec. 4.1).
template <int NT>
__device__ void project_rigid(double* s_l, int nc, const double* Yr, const double* KtKi, double* red) {
  double f0 = 0, f1 = 0, f2 = 0;
  for (int j = threadIdx.x; j < nc; j += NT) {
    double lx = s_l[2 * j], ly = s_l[2 * j + 1];
    double yx = Yr[2 * j], yy = Yr[2 * j + 1];
    f0 += lx;
    f1 += ly;
    f2 += -yy * lx + yx * ly;
  }
  f0 = block_sum<NT>(f0, red);
  f1 = block_sum<NT>(f1, red + 16);
  f2 = block_sum<NT>(f2, red + 32);
  const double a0 = KtKi[0] * f0 + KtKi[1] * f1 + KtKi[2] * f2;
  const double a1 = KtKi[3] * f0 + KtKi[4] * f1 + KtKi[5] * f2;
  const double a2 = KtKi[6] * f0 + KtKi[7] * f1 + KtKi[8] * f2;
  __syncthreads();
  for (int j = threadIdx.x; j < nc; j += NT) {
    double yx = Yr[2 * j], yy = Yr[2 * j + 1];
    s_l[2 * j] -= a0 - a2 * yy;
    s_l[2 * j + 1] -= a1 + a2 * yx;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Step 1a: lambda_bar = V Sigma^+ (U^T mu) per body, shared factors per class (eq. howG+, eq. SL).
// ob <= kObBodies consecutive bodies per workgroup: when they share a class each factor element
// read from L2 serves all of them (the factors, 2 x 144 x 120 doubles per class, are otherwise
// read once per body); each body's sums keep the one-body order, so the result does not depend
// on the grouping.  Dynamic LDS: ob x (m2max + rmax) doubles (2 max n_col, max rank).
constexpr int kObBodies = 4;
__global__ __launch_bounds__(kBodyThreads) void k_onebody(int P, const int* __restrict__ cls,
                                                          const int* __restrict__ src_off,
                                                          const int* __restrict__ col_off, ClassTab ct,
                                                          const double* __restrict__ mu,
                                                          double* __restrict__ lam, int ob, int m2max, int rmax) {
  const int b0 = blockIdx.x * ob;
  if (b0 >= P) return;
  const int nb = min(ob, P - b0);
  extern __shared__ double s_ob[];
  double* s_mu = s_ob;                  // [ob][m2max]
  double* s_t = s_ob + ob * m2max;      // [ob][rmax]
  const int k0 = cls[b0];
  bool same = true;
  for (int i = 1; i < nb; ++i) same = same && cls[b0 + i] == k0;
  // bodies processed together: all nb of one class, else one at a time
  for (int g0 = 0; g0 < nb; g0 += same ? nb : 1) {
    const int gn = same ? nb : 1;
    const int k = cls[b0 + g0];
    const int m2 = 2 * ct.mc[k], n2 = 2 * ct.nc[k], r = ct.rank[k];
    // LDS slots 0..ob-1; the accumulators beyond ob read slot 0 and are not stored
    for (int i = 0; i < ob; ++i) {
      const double* mub = mu + 2 * (int64_t)col_off[b0 + g0 + (i < gn ? i : 0)];
      for (int q = threadIdx.x; q < m2; q += kBodyThreads) s_mu[i * m2max + q] = i < gn ? mub[q] : 0.0;
    }
    __syncthreads();
    const double* U = ct.U[k];
    const double* si = ct.sinv[k];
    for (int j = threadIdx.x; j < r; j += kBodyThreads) {
      double acc[kObBodies] = {};
#pragma unroll 8
      for (int q = 0; q < m2; ++q) {
        const double u = U[(int64_t)q * r + j];
#pragma unroll
        for (int i = 0; i < kObBodies; ++i) acc[i] = fma(u, s_mu[(i < ob ? i : 0) * m2max + q], acc[i]);
      }
#pragma unroll
      for (int i = 0; i < kObBodies; ++i)
        if (i < ob) s_t[i * rmax + j] = acc[i] * si[j];
    }
    __syncthreads();
    const double* Vt = ct.Vt[k];
    for (int o = threadIdx.x; o < n2; o += kBodyThreads) {
      double acc[kObBodies] = {};
#pragma unroll 8
      for (int j = 0; j < r; ++j) {
        const double v = Vt[(int64_t)j * n2 + o];
#pragma unroll
        for (int i = 0; i < kObBodies; ++i) acc[i] = fma(v, s_t[(i < ob ? i : 0) * rmax + j], acc[i]);
      }
#pragma unroll
      for (int i = 0; i < kObBodies; ++i)
        if (i < gn) lam[2 * (int64_t)src_off[b0 + g0 + i] + o] = acc[i];
    }
    __syncthreads();   // s_mu and s_t are reused by the next group
  }
}

// ---------------------------------------------------------------------------
// Step 1b: lambda_tilde^c = A^c [lambda_bar^(i); lambda_bar^(k)] per close pair (eq. correction).
// A^c column-major: for a fixed column the threads of a block read consecutive rows.
constexpr int kPairThreads = 256;
__global__ __launch_bounds__(kPairThreads) void k_pair_A(int C, const int* __restrict__ pairs,
                                                         const int* __restrict__ src_off,
                                                         const int64_t* __restrict__ xoff,
                                                         const int64_t* __restrict__ aoff,
                                                         const double* __restrict__ A,
                                                         const double* __restrict__ lam,
                                                         double* __restrict__ ltil) {
  const int c = blockIdx.x;
  if (c >= C) return;
  const int i = pairs[2 * c], k = pairs[2 * c + 1];
  const int ni = 2 * (src_off[i + 1] - src_off[i]);
  const int n = (int)(xoff[c + 1] - xoff[c]);
  __shared__ double s_x[4 * kMaxCol];
  for (int q = threadIdx.x; q < n; q += kPairThreads)
    s_x[q] = q < ni ? lam[2 * (int64_t)src_off[i] + q] : lam[2 * (int64_t)src_off[k] + (q - ni)];
  __syncthreads();
  const double* Ac = A + aoff[c];
  for (int row = threadIdx.x; row < n; row += kPairThreads) {
    double acc = 0.0;
    // the loads of 16 columns in flight per thread (A^c streams from HBM); the sum keeps the
    // column order of the stacked form k_pair_A_rhs, so both give the same bits
#pragma unroll 16
    for (int col = 0; col < n; ++col) acc = fma(Ac[(int64_t)col * n + row], s_x[col], acc);
    ltil[xoff[c] + row] = acc;
  }
}

// Stacked right-hand sides: lambda_tilde^c_r = A^c [lambda_bar_r^(i); lambda_bar_r^(k)] for
// R <= 16 vectors at once on the matrix cores: L (n x 16) = A^c (n x n) X (n x 16) in
// 16 x 16 x 4 FP64 MFMA steps, the columns beyond R zero.  Each A^c element is read from
// HBM once for all R vectors; X (R n doubles) sits in dynamic LDS.  Operand layout of
// v_mfma_f64_16x16x4f64 (64 lanes, l = lane; checked on the device): A element
// (l % 16, l / 16), B element (l / 16, l % 16), result item q = 0..3 at row l / 16 + 4 q,
// column l % 16.
typedef double mfs_double4_t __attribute__((ext_vector_type(4)));

template <int R>
__global__ __launch_bounds__(kPairThreads) void k_pair_A_rhs(int C, const int* __restrict__ pairs,
                                                             const int* __restrict__ src_off,
                                                             const int64_t* __restrict__ xoff,
                                                             const int64_t* __restrict__ aoff,
                                                             const double* __restrict__ A,
                                                             const double* __restrict__ lam, int64_t lam_stride,
                                                             double* __restrict__ ltil, int64_t ltil_stride) {
  static_assert(R >= 1 && R <= 16, "at most 16 stacked vectors");
  extern __shared__ double s_xr[];   // [r][n]
  const int c = blockIdx.x;
  if (c >= C) return;
  const int i = pairs[2 * c], k = pairs[2 * c + 1];
  const int ni = 2 * (src_off[i + 1] - src_off[i]);
  const int n = (int)(xoff[c + 1] - xoff[c]);
  for (int e = threadIdx.x; e < R * n; e += kPairThreads) {
    const int r = e / n, q = e - r * n;
    const double* l = lam + r * lam_stride;
    s_xr[e] = q < ni ? l[2 * (int64_t)src_off[i] + q] : l[2 * (int64_t)src_off[k] + (q - ni)];
  }
  __syncthreads();
  const double* Ac = A + aoff[c];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nrb = (n + 15) >> 4;
  for (int rb = wave; rb < nrb; rb += kPairThreads / 64) {
    const int row = rb * 16 + li;
    mfs_double4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += 4) {
      const int kk = k0 + lk;
      const double a = (row < n && kk < n) ? Ac[(int64_t)kk * n + row] : 0.0;
      const double b = (li < R && kk < n) ? s_xr[li * n + kk] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    if (li < R) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rr = rb * 16 + lk + 4 * q;
        if (rr < n) ltil[li * ltil_stride + xoff[c] + rr] = acc[q];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// eq. total_corr + projection: lambda^(b) = lambda_bar^(b) + sum_{c contains b} lambda_tilde^c_b,
// sigma = (I - L) lambda (mobility) or lambda (resistance); packed for the kernel sum as
// (y, sigma) per source, FP64, in the caller's disk order.
__global__ __launch_bounds__(kBodyThreads) void k_gather_project(
    int P, int mobility, const int* __restrict__ cls, const int* __restrict__ src_off, ClassTab ct,
    const int* __restrict__ bp_off, const int* __restrict__ bp_list, const int* __restrict__ pairs,
    const int64_t* __restrict__ xoff, const double* __restrict__ ltil, const double* __restrict__ lam_bar,
    int with_pairs, const double* __restrict__ centers, double4* __restrict__ src64) {
  const int b = blockIdx.x;
  if (b >= P) return;
  const int k = cls[b];
  const int nc = ct.nc[k];
  const int64_t so = src_off[b];
  __shared__ double s_l[2 * kMaxCol];
  __shared__ double red[64];
  for (int q = threadIdx.x; q < 2 * nc; q += kBodyThreads) {
    double v = lam_bar[2 * so + q];
    if (with_pairs) {
      for (int e = bp_off[b]; e < bp_off[b + 1]; ++e) {
        const int c = bp_list[e] >> 1, side = bp_list[e] & 1;
        const int64_t off = xoff[c] + (side ? 2 * (src_off[pairs[2 * c] + 1] - src_off[pairs[2 * c]]) : 0);
        v += ltil[off + q];
      }
    }
    s_l[q] = v;
  }
  __syncthreads();
  if (mobility) project_rigid<kBodyThreads>(s_l, nc, ct.Yr[k], ct.KtKi[k], red);
  const double* Yr = ct.Yr[k];
  const double cx = centers[2 * b], cy = centers[2 * b + 1];
  for (int j = threadIdx.x; j < nc; j += kBodyThreads)
    src64[so + j] = make_double4(cx + Yr[2 * j], cy + Yr[2 * j + 1], s_l[2 * j], s_l[2 * j + 1]);
}

// ---------------------------------------------------------------------------
// Step 2a: all-pairs Stokeslet sum u_t = sum_s S(x_t, y_s) sigma_s (eq. getall, eq. stokeslet2d),
//   u = 1/(4 pi mu) [ sum (d.sigma / r^2) d  -  (ln 2 / 2) sum log2(r^2) sigma ].
// Two kernels evaluate it.  The context's own sum (every matvec, the right-hand side) is the
// hierarchical k_ksum_fmm_mixed / k_ksum_fmm_fp64 at the end of this file.  Sums at arbitrary points (flow
// evaluation) use the two-level FP64 k_ksum_fp64: a workgroup owns T * 256 consecutive
// targets, thread i the T targets from T i on; it streams one split's clusters of disks
// through LDS, one cluster per tile; a cluster far from every target of a wave is summed
// from its expansion, a disk beyond 7 ring radii from its multipole expansion (k_moments64),
// the rest directly.
constexpr int KS_THREADS = 256;
constexpr int KS_TILE = 1024;   // sources per LDS tile (16 KB of float4)

// ---- local expansions of far clusters (M2L, L2P; the oracle's local_expansion, eval_local) ----
// With w = x - T about the workgroup's target centre T and a cluster's moments about C,
// Delta = T - C, the cluster's field is Phi1 + conj(Psi) - w conj(Phi1') + A_0 / 2 with
//   Phi1 = -(A_0/2) log Z + sum_k A_k Z^-k / (2k),
//   Psi  = -(conj A_0/2) log Z + sum_k [conj(B_k)/(2k) - D_{k-1}/2 + conj(Delta) A_{k-1}/2] Z^-k,
// and (w + Delta)^-k = sum_l (-1)^l binom(k + l - 1, l) Delta^-(k+l) w^l: the coefficient of
// w^l is (-1)^l Delta^-l sum_k binom(k + l - 1, l) c_k Delta^-k plus the log term's.  A wave
// translates one cluster: lane l < 32 holds Phi1's coefficient of w^l, lane 32 + l Psi's;
// lane k first scales its function's c_k by Delta^-k into the wave's LDS row, then every lane
// sums the row with its binomials.  Only Re log enters the velocity, so log Delta = ln |Delta|.
// The binomials: with a factorial table in LDS (fac), binom(k + l - 1, l) = (k + l - 1)! /
// (l! (k - 1)!), the row scaled by 1/(k - 1)! and the sum by 1/l!, two FMAs per term; without
// it, by the recurrence binom(k + l, l) = binom(k + l - 1, l) (k + l) / k.
__constant__ double kInvInt[32] = {0.0,        1.0,        1.0 / 2,  1.0 / 3,  1.0 / 4,  1.0 / 5,  1.0 / 6,
                                   1.0 / 7,    1.0 / 8,    1.0 / 9,  1.0 / 10, 1.0 / 11, 1.0 / 12, 1.0 / 13,
                                   1.0 / 14,   1.0 / 15,   1.0 / 16, 1.0 / 17, 1.0 / 18, 1.0 / 19, 1.0 / 20,
                                   1.0 / 21,   1.0 / 22,   1.0 / 23, 1.0 / 24, 1.0 / 25, 1.0 / 26, 1.0 / 27,
                                   1.0 / 28,   1.0 / 29,   1.0 / 30, 1.0 / 31};

constexpr int kFactN = 64;
// j! and 1/j! for j = 0..63, correctly rounded: the translation's binomials
// binom(k + l - 1, l) = (k + l - 1)! / (l! (k - 1)!) from three rounded factors
__constant__ double kFact[2 * kFactN] = {
    1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0, 5040.0, 40320.0, 362880.0, 3628800.0, 39916800.0, 479001600.0,
    6227020800.0, 87178291200.0, 1307674368000.0, 20922789888000.0, 355687428096000.0, 6402373705728000.0,
    1.21645100408832e+17, 2.43290200817664e+18, 5.109094217170944e+19, 1.1240007277776077e+21,
    2.585201673888498e+22, 6.204484017332394e+23, 1.5511210043330986e+25, 4.0329146112660565e+26,
    1.0888869450418352e+28, 3.0488834461171387e+29, 8.841761993739702e+30, 2.6525285981219107e+32,
    8.222838654177922e+33, 2.631308369336935e+35, 8.683317618811886e+36, 2.9523279903960416e+38,
    1.0333147966386145e+40, 3.7199332678990125e+41, 1.3763753091226346e+43, 5.230226174666011e+44,
    2.0397882081197444e+46, 8.159152832478977e+47, 3.345252661316381e+49, 1.40500611775288e+51,
    6.041526306337383e+52, 2.658271574788449e+54, 1.1962222086548019e+56, 5.502622159812089e+57,
    2.5862324151116818e+59, 1.2413915592536073e+61, 6.082818640342675e+62, 3.0414093201713376e+64,
    1.5511187532873822e+66, 8.065817517094388e+67, 4.2748832840600255e+69, 2.308436973392414e+71,
    1.2696403353658276e+73, 7.109985878048635e+74, 4.0526919504877214e+76, 2.3505613312828785e+78,
    1.3868311854568984e+80, 8.32098711274139e+81, 5.075802138772248e+83, 3.146997326038794e+85,
    1.98260831540444e+87, 1.0, 1.0, 0.5, 0.16666666666666666, 0.041666666666666664, 0.008333333333333333,
    0.001388888888888889, 0.0001984126984126984, 2.48015873015873e-05, 2.7557319223985893e-06,
    2.755731922398589e-07, 2.505210838544172e-08, 2.08767569878681e-09, 1.6059043836821613e-10,
    1.1470745597729725e-11, 7.647163731819816e-13, 4.779477332387385e-14, 2.8114572543455206e-15,
    1.5619206968586225e-16, 8.22063524662433e-18, 4.110317623312165e-19, 1.9572941063391263e-20,
    8.896791392450574e-22, 3.868170170630684e-23, 1.6117375710961184e-24, 6.446950284384474e-26,
    2.4795962632247976e-27, 9.183689863795546e-29, 3.279889237069838e-30, 1.1309962886447716e-31,
    3.7699876288159054e-33, 1.216125041553518e-34, 3.8003907548547434e-36, 1.151633562077195e-37,
    3.387157535521162e-39, 9.67759295863189e-41, 2.6882202662866363e-42, 7.265460179153071e-44,
    1.911963205040282e-45, 4.902469756513544e-47, 1.2256174391283858e-48, 2.9893108271424046e-50,
    7.117406731291439e-52, 1.6552108677421951e-53, 3.7618428812322616e-55, 8.359650847182804e-57,
    1.817315401561479e-58, 3.866628513960594e-60, 8.055476070751236e-62, 1.643974708316579e-63,
    3.287949416633158e-65, 6.446959640457172e-67, 1.2397999308571486e-68, 2.3392451525606576e-70,
    4.331935467704922e-72, 7.876246304918039e-74, 1.4064725544496498e-75, 2.4674957095607893e-77,
    4.254302947518602e-79, 7.2106829618959365e-81, 1.2017804936493226e-82, 1.9701319568021682e-84,
    3.1776321883905942e-86, 5.043860616493007e-88};

// wave-level fence for LDS rows written and read by lanes of one wave (no workgroup barrier:
// the waves of a workgroup translate different clusters)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A cluster (centre cx, cy, radius R) goes into the workgroup's local expansion when it is
// beyond both 4 R + rb (every target then beyond 4 R: a far cluster holds no target's disk or
// contact partner, by the cluster radii) and sep (R + rb) (theta <= 1/sep) from the centre
// (bx, by) of the workgroup's targets; the same expression in every pass that decides it
__device__ __forceinline__ bool le_far(double cx, double cy, double R, double bx, double by, double rb, double sep) {
  const double dx = __dsub_rn(cx, bx), dy = __dsub_rn(cy, by);
  const double thr = fmax(__dadd_rn(__dmul_rn(4.0 * (1.0 + 1e-6), R), rb), __dmul_rn(sep, __dadd_rn(R, rb)));
  return __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)) > __dmul_rn(thr, thr);
}

// Workgroup bounding circle of its targets: centre (bx, by), radius rb (padded)
template <int T>
__device__ __forceinline__ void target_bounds(const double (&x)[T], const double (&y)[T], double (*s_bb)[KS_THREADS / 64],
                                              double& bx, double& by, double& rb) {
  double xl = x[0], xh = x[0], yl = y[0], yh = y[0];
#pragma unroll
  for (int j = 1; j < T; ++j) {
    xl = fmin(xl, x[j]);
    xh = fmax(xh, x[j]);
    yl = fmin(yl, y[j]);
    yh = fmax(yh, y[j]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    xl = fmin(xl, __shfl_xor(xl, off, 64));
    xh = fmax(xh, __shfl_xor(xh, off, 64));
    yl = fmin(yl, __shfl_xor(yl, off, 64));
    yh = fmax(yh, __shfl_xor(yh, off, 64));
  }
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_bb[0][wid] = xl;
    s_bb[1][wid] = xh;
    s_bb[2][wid] = yl;
    s_bb[3][wid] = yh;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < KS_THREADS / 64; ++w) {
    xl = fmin(xl, s_bb[0][w]);
    xh = fmax(xh, s_bb[1][w]);
    yl = fmin(yl, s_bb[2][w]);
    yh = fmax(yh, s_bb[3][w]);
  }
  bx = 0.5 * (xl + xh);
  by = 0.5 * (yl + yh);
  rb = 0.5 * sqrt((xh - xl) * (xh - xl) + (yh - yl) * (yh - yl)) * (1.0 + 1e-9) + 1e-9;
}

// Add the local expansion about (bx, by) of the cluster whose FP64 record (k_cluster_moments64)
// is rec and centre (cx, cy) to the lane's coefficient (Lr, Li); K source and Q local orders.
template <int K, int Q>
__device__ __forceinline__ void m2l_add(const double2* __restrict__ rec, double cx, double cy, double bx,
                                        double by, double2* row, double& Lr, double& Li,
                                        const double* fac = nullptr) {
  static_assert(K < 32 && Q < 32, "one lane per order");
  const int lane = threadIdx.x & 63, f = lane >> 5, l = lane & 31;
  const double dx = bx - cx, dy = by - cy;   // Delta = T - C
  const double d2 = fma(dx, dx, dy * dy);
  const double id2 = rcp_f64(d2);
  const double ix = dx * id2, iy = -dy * id2;   // 1/Delta
  // Delta^-l by binary powering over l's five bits, unrolled and branch-free (l < 32)
  double pr = (l & 1) ? ix : 1.0, pi = (l & 1) ? iy : 0.0;
  {
    double br = ix * ix - iy * iy, bi = 2.0 * ix * iy;
#pragma unroll
    for (int bit = 1; bit < 5; ++bit) {
      const double t = pr * br - pi * bi;
      const double v = fma(pr, bi, pi * br);
      if ((l >> bit) & 1) {
        pr = t;
        pi = v;
      }
      if (bit < 4) {
        const double u = br * br - bi * bi;
        bi = 2.0 * br * bi;
        br = u;
      }
    }
  }
  wave_lds_sync();   // the row's previous reads are done
  if (l >= 1 && l <= K) {
    double cr, ci;
    if (f == 0) {   // A_k / (2k)
      cr = rec[l - 1].x;
      ci = rec[l - 1].y;
    } else {        // conj(B_k)/(2k) - D_{k-1}/2 + conj(Delta) A_{k-1}/2 (the record holds conj(D), conj(A))
      const double2 b = rec[kCl64Order + l - 1], dd = rec[3 * kCl64Order + l], a = rec[2 * kCl64Order + l - 1];
      cr = b.x - 0.5 * dd.x + 0.5 * (dx * a.x - dy * a.y);
      ci = -b.y + 0.5 * dd.y - 0.5 * (dx * a.y + dy * a.x);
    }
    // with the factorial table the row holds c_l Delta^-l / (l - 1)!
    const double sc = fac ? fac[kFactN + l - 1] : 1.0;
    row[lane] = make_double2((cr * pr - ci * pi) * sc, fma(cr, pi, ci * pr) * sc);
  }
  wave_lds_sync();
  double ar = 0.0, ai = 0.0;
  const double2* rf = row + (f << 5);
  if (fac) {
    // sum_k (k + l - 1)! [c_k Delta^-k / (k - 1)!], then / l!  (the factorials in LDS)
    const double* fk = fac + l;
#pragma unroll 4
    for (int k = 1; k <= K; ++k) {
      const double2 c = rf[k];
      const double g = fk[k - 1];
      ar = fma(g, c.x, ar);
      ai = fma(g, c.y, ai);
    }
    ar *= fac[kFactN + l];
    ai *= fac[kFactN + l];
  } else {
    double bn = 1.0;   // binom(k + l - 1, l), k = 1
#pragma unroll 2
    for (int k = 1; k <= K; ++k) {
      const double2 c = rf[k];
      ar = fma(bn, c.x, ar);
      ai = fma(bn, c.y, ai);
      bn *= (double)(k + l) * kInvInt[k];
    }
  }
  if (l > Q) return;
  const double2 a0 = rec[2 * kCl64Order];   // conj(A_0)
  const double lr = -0.5 * a0.x, li = f == 0 ? 0.5 * a0.y : -0.5 * a0.y;   // log coefficient
  const double sg = (l & 1) ? -1.0 : 1.0;
  double tr = sg * (ar * pr - ai * pi), ti = sg * fma(ar, pi, ai * pr);
  if (l == 0) {
    const double lg = 0.5 * ln_f64(d2);
    tr = fma(lr, lg, tr);
    ti = fma(li, lg, ti);
    if (f == 0) {   // the constant A_0 / 2
      tr = fma(0.5, a0.x, tr);
      ti = fma(-0.5, a0.y, ti);
    }
  } else {
    const double s2 = -sg * kInvInt[l];
    tr = fma(s2, lr * pr - li * pi, tr);
    ti = fma(s2, fma(lr, pi, li * pr), ti);
  }
  Lr += tr;
  Li += ti;
}

// The workgroup's local expansion: the waves' coefficients summed in LDS (s_le, 64 double2),
// then evaluated at offset (wx, wy): u = L1 + conj(L2) - w conj(L1') (units of 4 pi mu).
template <int Q>
__device__ __forceinline__ void le_reduce(double Lr, double Li, double2 (*s_part)[64], double2* s_le) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  s_part[wid][lane] = make_double2(Lr, Li);
  __syncthreads();
  if (threadIdx.x < 64) {
    double2 t = s_part[0][threadIdx.x];
    for (int w = 1; w < KS_THREADS / 64; ++w) {
      t.x += s_part[w][threadIdx.x].x;
      t.y += s_part[w][threadIdx.x].y;
    }
    s_le[threadIdx.x] = t;
  }
  __syncthreads();
}

template <int Q>
__device__ __forceinline__ void l2p(const double2* s_le, double wx, double wy, double& ux, double& uy) {
  double vr = s_le[Q].x, vi = s_le[Q].y, dr = 0.0, di = 0.0;   // L1 and L1' by Horner
  double gr = s_le[32 + Q].x, gi = s_le[32 + Q].y;             // L2
#pragma unroll 1
  for (int l = Q - 1; l >= 0; --l) {
    const double t = fma(dr, wx, -di * wy) + vr;
    di = fma(dr, wy, di * wx) + vi;
    dr = t;
    const double u = fma(vr, wx, -vi * wy) + s_le[l].x;
    vi = fma(vr, wy, vi * wx) + s_le[l].y;
    vr = u;
    const double g = fma(gr, wx, -gi * wy) + s_le[32 + l].x;
    gi = fma(gr, wy, gi * wx) + s_le[32 + l].y;
    gr = g;
  }
  // w conj(L1') = (wx dr + wy di) + i (wy dr - wx di)
  ux = vr + gr - fma(wx, dr, wy * di);
  uy = vi - gi - fma(wy, dr, -wx * di);
}
constexpr int KS_MAXB = 64;     // bodies per LDS tile (a cluster is one tile)
static_assert(kClMaxBodies <= KS_MAXB && kClMaxSources <= KS_TILE, "a cluster must fit one LDS tile");

// Skip modes: 0 = every source, 1 = skip the target's own disk, 2 = skip the own disk
// and its contact partners (nbr_off/nbr_list: sorted partner list per disk).  A
// thread walks its target's sorted partner list alongside the increasing source
// body index, so the test costs one compare per (target, source disk).
struct Skip {
  int next;   // next partner >= current source body, or INT_MAX
  int pos, end;
};

__device__ __forceinline__ void skip_init(Skip& sk, int mode, int body, int kb0, const int* __restrict__ nbr_off,
                                          const int* __restrict__ nbr_list) {
  sk.next = 0x7fffffff;
  sk.pos = sk.end = 0;
  if (mode != 2) return;
  sk.pos = nbr_off[body];
  sk.end = nbr_off[body + 1];
  while (sk.pos < sk.end && nbr_list[sk.pos] < kb0) ++sk.pos;
  if (sk.pos < sk.end) sk.next = nbr_list[sk.pos];
}

// true if source body kb must be skipped for this target; advances the partner cursor
__device__ __forceinline__ bool skip_test(Skip& sk, int mode, int kb, int body, const int* __restrict__ nbr_list) {
  if (mode == 0) return false;
  if (kb == body) return true;
  if (kb == sk.next) {
    ++sk.pos;
    sk.next = sk.pos < sk.end ? nbr_list[sk.pos] : 0x7fffffff;
    return true;
  }
  return false;
}

// FP64 far-field coefficients of a packed FP64 source array (the expansion of
// k_gather_project to order kMp64Order): per disk A_k/(2k) (k = 1..p), B_k/(2k) (k = 1..p),
// conj(A_k) (k = 0..p), conj(B_1) and (rho^2, 0).  The offsets w are the class ring Yr
// (the packed positions are c + Yr); the strengths are the packed ones.  Truncation of the
// FP64 sum's expansion beyond kMp64Far2: below sum |sigma| (1/7)^19 / (6/7) = 1e-16 sum |sigma|.
constexpr int kMp64Coef = kMp64CoefPerDisk;
constexpr double kMp64Far2 = 49.0;

__global__ __launch_bounds__(kBodyThreads) void k_moments64(int P, const int* __restrict__ cls,
                                                            const int* __restrict__ src_off, ClassTab ct,
                                                            const double4* __restrict__ src,
                                                            double2* __restrict__ mp64) {
  const int b = blockIdx.x;
  if (b >= P) return;
  const int k = cls[b];
  const double* Yr = ct.Yr[k];
  const int nc = ct.nc[k];
  const int64_t so = src_off[b];
  double ar[kMp64Order], ai[kMp64Order], br[kMp64Order], bi[kMp64Order];
#pragma unroll
  for (int m = 0; m < kMp64Order; ++m) ar[m] = ai[m] = br[m] = bi[m] = 0.0;
  double s0r = 0.0, s0i = 0.0;
  for (int j = threadIdx.x; j < nc; j += kBodyThreads) {
    const double4 v = src[so + j];
    const double wx = Yr[2 * j], wy = Yr[2 * j + 1];
    s0r += v.z;
    s0i += v.w;
    double pr = v.z, pi = v.w, qr = v.z, qi = v.w;   // sigma w^m and sigma conj(w)^m
#pragma unroll
    for (int m = 0; m < kMp64Order; ++m) {
      const double tr = pr * wx - pi * wy, ti = pr * wy + pi * wx;
      const double ur = qr * wx + qi * wy, ui = qi * wx - qr * wy;
      pr = tr;
      pi = ti;
      qr = ur;
      qi = ui;
      ar[m] += pr;
      ai[m] += pi;
      br[m] += qr;
      bi[m] += qi;
    }
  }
  __shared__ double mred[2][4 * kMp64Order + 2];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  auto put = [&](int slot, double v) {
    v = wave_sum(v);
    if (lane == 0) mred[wid][slot] = v;
  };
#pragma unroll
  for (int m = 0; m < kMp64Order; ++m) {
    put(4 * m, ar[m]);
    put(4 * m + 1, ai[m]);
    put(4 * m + 2, br[m]);
    put(4 * m + 3, bi[m]);
  }
  put(4 * kMp64Order, s0r);
  put(4 * kMp64Order + 1, s0i);
  __syncthreads();
  static_assert(kBodyThreads == 128, "two waves per body block");
  for (int e = threadIdx.x; e < 4 * kMp64Order + 2; e += kBodyThreads) mred[0][e] += mred[1][e];
  __syncthreads();
  if (threadIdx.x == 0) {
    double2* o = mp64 + (int64_t)b * kMp64Coef;
    for (int m = 1; m <= kMp64Order; ++m) {
      const double* r = &mred[0][4 * (m - 1)];
      o[m - 1] = make_double2(r[0] / (2 * m), r[1] / (2 * m));
      o[kMp64Order + m - 1] = make_double2(r[2] / (2 * m), r[3] / (2 * m));
      o[2 * kMp64Order + m] = make_double2(r[0], -r[1]);
    }
    o[2 * kMp64Order] = make_double2(mred[0][4 * kMp64Order], -mred[0][4 * kMp64Order + 1]);
    o[3 * kMp64Order + 1] = make_double2(mred[0][2], -mred[0][3]);
    o[3 * kMp64Order + 2] = make_double2(Yr[0] * Yr[0] + Yr[1] * Yr[1], 0.0);
  }
}

// FP64 expansion of each cluster about its centre C: the moments A_k = sum sigma w^k,
// B_k = sum sigma conj(w)^k and D_k = sum sigma conj(w) w^k of the sources' offsets w = y - C,
// to order kCl64Order, from a packed FP64 source array (src: absolute positions and strengths,
// body order).  They serve the two-level sum's per-target cluster expansions and its local
// expansions.  One workgroup per cluster, thread e forms the order-e moments over the
// cluster's sources in slot order (w^e by binary powering).  Record: A_k/(2k), B_k/(2k)
// (k = 1..p), conj(A_k), conj(D_k) (k = 0..p).  Truncation at theta <= 1/4: below
// sum |sigma| 4^-27 / (3/4) = 7e-17 sum |sigma|.
constexpr int kCl64Coef = kCl64CoefPerCluster;

__global__ __launch_bounds__(64) void k_cluster_moments64(int ncl, const int* __restrict__ cl_start,
                                                          const int* __restrict__ slot_body,
                                                          const int* __restrict__ src_off,
                                                          const double* __restrict__ ccent,
                                                          const double4* __restrict__ src,
                                                          double2* __restrict__ cmp) {
  const int q = blockIdx.x;
  const int e = threadIdx.x;
  if (q >= ncl || e > kCl64Order) return;
  const double Cx = ccent[2 * q], Cy = ccent[2 * q + 1];
  double Ar = 0, Ai = 0, Br = 0, Bi = 0, Dr = 0, Di = 0;
  for (int sl = cl_start[q]; sl < cl_start[q + 1]; ++sl) {
    const int b = slot_body[sl];
    for (int j = src_off[b]; j < src_off[b + 1]; ++j) {
      const double4 v = src[j];
      const double wx = v.x - Cx, wy = v.y - Cy;
      double pr = 1.0, pi = 0.0, br = wx, bi = wy;   // w^e
      for (int k = e; k; k >>= 1) {
        if (k & 1) {
          const double tr = pr * br - pi * bi;
          pi = pr * bi + pi * br;
          pr = tr;
        }
        const double ur = br * br - bi * bi;
        bi = 2.0 * br * bi;
        br = ur;
      }
      const double sr = v.z * pr - v.w * pi, si = v.z * pi + v.w * pr;   // sigma w^e
      Ar += sr;
      Ai += si;
      Br += v.z * pr + v.w * pi;   // sigma conj(w^e)
      Bi += v.w * pr - v.z * pi;
      Dr += wx * sr + wy * si;     // conj(w) sigma w^e
      Di += wx * si - wy * sr;
    }
  }
  double2* o = cmp + (int64_t)q * kCl64Coef;
  if (e >= 1) {
    o[e - 1] = make_double2(Ar / (2 * e), Ai / (2 * e));
    o[kCl64Order + e - 1] = make_double2(Br / (2 * e), Bi / (2 * e));
  }
  o[2 * kCl64Order + e] = make_double2(Ar, -Ai);
  o[3 * kCl64Order + 1 + e] = make_double2(Dr, -Di);
}

// Far test of a cluster (centre cx, cy; lim = 16 R^2) for every target of a thread, without
// contraction, so that every pass that decides it decides alike
template <int T>
__device__ __forceinline__ bool cl_far64(const double (&x)[T], const double (&y)[T], double cx, double cy,
                                         double lim) {
  bool far = true;
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const double dx = __dsub_rn(x[j], cx), dy = __dsub_rn(y[j], cy);
    far = far && __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)) > lim;
  }
  return far;
}

// A cluster's FP64 expansion (record cf, centre cx, cy; k_cluster_moments64) added at a thread's
// targets: four complex Horner series of degree kCl64Order
template <int T>
__device__ __forceinline__ void cluster_expansion64(const double2* __restrict__ cf, double cx, double cy,
                                                    const double (&x)[T], const double (&y)[T], double (&ax)[T],
                                                    double (&ay)[T]) {
  double Zx[T], Zy[T], R2[T], zr[T], zi[T], h1r[T], h1i[T], h2r[T], h2i[T], h3r[T], h3i[T], h4r[T], h4i[T];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    Zx[j] = x[j] - cx;
    Zy[j] = y[j] - cy;
    R2[j] = fma(Zx[j], Zx[j], Zy[j] * Zy[j]);
    const double ir2 = rcp_f64(R2[j]);
    zr[j] = Zx[j] * ir2;
    zi[j] = Zy[j] * ir2;
    h1r[j] = cf[kCl64Order - 1].x;
    h1i[j] = cf[kCl64Order - 1].y;
    h2r[j] = cf[2 * kCl64Order - 1].x;
    h2i[j] = cf[2 * kCl64Order - 1].y;
    h3r[j] = cf[3 * kCl64Order].x;
    h3i[j] = cf[3 * kCl64Order].y;
    h4r[j] = cf[4 * kCl64Order + 1].x;
    h4i[j] = cf[4 * kCl64Order + 1].y;
  }
#pragma unroll 2
  for (int m = kCl64Order - 1; m >= 1; --m) {
    const double2 a = cf[m - 1], bq = cf[kCl64Order + m - 1], g = cf[2 * kCl64Order + m], e = cf[3 * kCl64Order + 1 + m];
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const double t1r = fma(zr[j], h1r[j], fma(zi[j], h1i[j], a.x));
      const double t1i = fma(zr[j], h1i[j], fma(-zi[j], h1r[j], a.y));
      const double t2r = fma(zr[j], h2r[j], fma(-zi[j], h2i[j], bq.x));
      const double t2i = fma(zr[j], h2i[j], fma(zi[j], h2r[j], bq.y));
      const double t3r = fma(zr[j], h3r[j], fma(-zi[j], h3i[j], g.x));
      const double t3i = fma(zr[j], h3i[j], fma(zi[j], h3r[j], g.y));
      const double t4r = fma(zr[j], h4r[j], fma(-zi[j], h4i[j], e.x));
      const double t4i = fma(zr[j], h4i[j], fma(zi[j], h4r[j], e.y));
      h1r[j] = t1r;
      h1i[j] = t1i;
      h2r[j] = t2r;
      h2i[j] = t2i;
      h3r[j] = t3r;
      h3i[j] = t3i;
      h4r[j] = t4r;
      h4i[j] = t4i;
    }
  }
  const double2 g0 = cf[2 * kCl64Order], e0 = cf[3 * kCl64Order + 1];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    const double pr = fma(zr[j], h3r[j], fma(-zi[j], h3i[j], g0.x));
    const double pi = fma(zr[j], h3i[j], fma(zi[j], h3r[j], g0.y));
    const double qr = fma(zr[j], h4r[j], fma(-zi[j], h4i[j], e0.x));
    const double qi = fma(zr[j], h4i[j], fma(zi[j], h4r[j], e0.y));
    const double p1r = fma(zr[j], h1r[j], zi[j] * h1i[j]);
    const double p1i = fma(zr[j], h1i[j], -zi[j] * h1r[j]);
    const double p2r = fma(zr[j], h2r[j], -zi[j] * h2i[j]);
    const double p2i = fma(zr[j], h2i[j], zi[j] * h2r[j]);
    const double mr = fma(Zx[j], pr, fma(-Zy[j], pi, -qr));   // Z P - Q
    const double mi = fma(Zx[j], pi, fma(Zy[j], pr, -qi));
    const double t3r = 0.5 * fma(zr[j], mr, -zi[j] * mi);
    const double t3i = 0.5 * fma(zr[j], mi, zi[j] * mr);
    const double lZ = fma(-0.5, ln_f64(R2[j]), 0.5);          // -ln|Z| + 1/2
    ax[j] += fma(g0.x, lZ, p1r + p2r + t3r);                  // S0 = conj(g0)
    ay[j] += fma(-g0.y, lZ, p1i + p2i + t3i);
  }
}

// Two-level FP64 sum at arbitrary points (flow evaluation; the context's own kernel sum is the
// hierarchical k_ksum_fmm_* below), absolute coordinates (ln_f64, rcp_f64 above): the split's
// clusters one LDS tile each, in slot order.  A cluster far from the
// workgroup (le_far) goes into its local expansion; one beyond 4 cluster radii from every
// target of a wave is summed by that wave from its FP64 expansion (order kCl64Order); the
// tile of a cluster that every wave takes that way is not staged.  Otherwise each disk of the
// cluster is summed from its FP64 expansion (k_moments64, order kMp64Order) by a wave whose
// targets are all beyond 7 ring radii, else directly over its sources.  src: FP64 packed
// sources in body order (src_off); ssrc_off: the same counts in slot order.  Skip modes as in
// ksum_fmm_body (partner lists in slots); mode 0 reads no body index (flow-evaluation points
// may have body -1).  mp64 NULL: every disk direct; cmp64 NULL: no cluster expansions.
template <int T>
__global__ __launch_bounds__(KS_THREADS) void k_ksum_fp64(int ncl, const int* __restrict__ cl_start,
                                                          const int* __restrict__ slot_body,
                                                          const int* __restrict__ ssrc_off,
                                                          const int* __restrict__ src_off,
                                                          const double4* __restrict__ src, int64_t Nt,
                                                          const int* __restrict__ tgt_body,
                                                          const int* __restrict__ slot_of,
                                                          const double* __restrict__ X, int clusters_per_split,
                                                          int mode, const int* __restrict__ nbr_off,
                                                          const int* __restrict__ nbr_slot, double scale,
                                                          double* __restrict__ out,
                                                          const double* __restrict__ centers,
                                                          const double2* __restrict__ mp64,
                                                          const double* __restrict__ ccent,
                                                          const double* __restrict__ crad,
                                                          const double2* __restrict__ cmp64,
                                                          const int* __restrict__ tperm,
                                                          unsigned long long* __restrict__ work, int local) {
  __shared__ double4 s_src[kClMaxSources];
  __shared__ int s_off[KS_MAXB + 1];
  const int split = blockIdx.y;
  const int q0 = min(ncl, split * clusters_per_split);
  const int q1 = min(ncl, q0 + clusters_per_split);
  int64_t t[T];    // position in the visiting order
  int64_t tt[T];   // the target there
  int bt[T];       // the target's disk, in slot order (skip modes 1, 2)
  double x[T], y[T], ax[T], ay[T];
  Skip sk[T];
  unsigned n_dir = 0, n_dexp = 0, n_cexp = 0, n_m2l = 0, n_l2p = 0;   // this lane's work
#pragma unroll
  for (int j = 0; j < T; ++j) {
    t[j] = (int64_t)blockIdx.x * (KS_THREADS * T) + threadIdx.x * T + j;   // a wave: 64 T consecutive targets
    const int64_t tc = t[j] < Nt ? t[j] : Nt - 1;
    tt[j] = tperm ? tperm[tc] : tc;
    const int body = mode != 0 ? tgt_body[tt[j]] : -1;
    bt[j] = mode != 0 ? slot_of[body] : -1;
    x[j] = X[2 * tt[j]];
    y[j] = X[2 * tt[j] + 1];
    ax[j] = 0.0;
    ay[j] = 0.0;
    skip_init(sk[j], mode, body, cl_start[q0], nbr_off, nbr_slot);
  }
  __shared__ double s_bb[4][KS_THREADS / 64];
  __shared__ double2 s_row[KS_THREADS / 64][64];
  __shared__ double2 s_le[64];
  double bx = 0.0, by = 0.0, rb = 0.0;
  if (cmp64) target_bounds<T>(x, y, s_bb, bx, by, rb);
  const bool use_le = cmp64 && local;
  const int wid = threadIdx.x >> 6;
  double Lr = 0.0, Li = 0.0;
  bool le_used = false;   // uniform over the workgroup
  for (int cq = q0; cq < q1; ++cq) {
    const int kt = cl_start[cq], ke = cl_start[cq + 1];
    const int nb = ke - kt;
    bool wfar = false;   // this wave sums the cluster from its expansion
    if (cmp64) {
      const double cx = ccent[2 * cq], cy = ccent[2 * cq + 1], R = crad[cq];
      if (use_le && le_far(cx, cy, R, bx, by, rb, kLocSep64)) {
        if ((cq & (KS_THREADS / 64 - 1)) == wid) {
          m2l_add<kLoc64, kLoc64>(cmp64 + (int64_t)cq * kCl64Coef, cx, cy, bx, by, s_row[wid], Lr, Li);
          n_m2l += (threadIdx.x & 63) == 0;
        }
        le_used = true;
        continue;
      }
      // beyond 4 R + rb of the targets' centre: every target beyond 4 R (uniform, no barrier)
      bool bfar;
      {
        const double dx = cx - bx, dy = cy - by;
        const double thr = 4.0 * (1.0 + 1e-6) * R + rb;
        bfar = dx * dx + dy * dy > thr * thr;
      }
      wfar = bfar || __all(cl_far64<T>(x, y, cx, cy, __dmul_rn(16.0, __dmul_rn(R, R))));
      if (wfar) {
        ++n_cexp;
        cluster_expansion64<T>(cmp64 + (int64_t)cq * kCl64Coef, cx, cy, x, y, ax, ay);
      }
      if (bfar) continue;
    }
    // the barrier also ends the reads of the previous tile before this one is staged
    if (__syncthreads_and(wfar ? 1 : 0)) continue;
    const int s0 = ssrc_off[kt];
    for (int kk = 0; kk < nb; ++kk) {
      const int o = ssrc_off[kt + kk] - s0, n = ssrc_off[kt + kk + 1] - s0 - o;
      const int64_t g = src_off[slot_body[kt + kk]];
      for (int q = threadIdx.x; q < n; q += KS_THREADS) s_src[o + q] = src[g + q];
    }
    for (int q = threadIdx.x; q <= nb; q += KS_THREADS) s_off[q] = ssrc_off[kt + q] - s0;
    __syncthreads();
    if (wfar) continue;
    for (int kk = 0; kk < nb; ++kk) {
      const int kslot = kt + kk;
      const int kbody = slot_body[kslot];
      if (mp64) {
        // far disk for every target of this wave: its FP64 expansion (three complex series
        // to order kMp64Order)
        const double2* cf = mp64 + (int64_t)kbody * kMp64Coef;
        const double q = cf[3 * kMp64Order + 2].x;
        const double cx = centers[2 * kbody], cy = centers[2 * kbody + 1];
        double Zx[T], Zy[T], R2[T];
        bool far = true;
#pragma unroll
        for (int j = 0; j < T; ++j) {
          Zx[j] = x[j] - cx;
          Zy[j] = y[j] - cy;
          R2[j] = fma(Zx[j], Zx[j], Zy[j] * Zy[j]);
          far = far && R2[j] > kMp64Far2 * q;
        }
        if (__all(far)) {   // one decision per wave
          ++n_dexp;
          double zr[T], zi[T], h1r[T], h1i[T], h2r[T], h2i[T], h3r[T], h3i[T];
#pragma unroll
          for (int j = 0; j < T; ++j) {
            const double ir2 = rcp_f64(R2[j]);
            zr[j] = Zx[j] * ir2;
            zi[j] = Zy[j] * ir2;
            h1r[j] = cf[kMp64Order - 1].x;
            h1i[j] = cf[kMp64Order - 1].y;
            h2r[j] = cf[2 * kMp64Order - 1].x;
            h2i[j] = cf[2 * kMp64Order - 1].y;
            h3r[j] = cf[3 * kMp64Order].x;
            h3i[j] = cf[3 * kMp64Order].y;
          }
#pragma unroll 2
          for (int m = kMp64Order - 1; m >= 1; --m) {   // coefficients loaded per step (uniform)
            const double2 a = cf[m - 1], bq = cf[kMp64Order + m - 1], g = cf[2 * kMp64Order + m];
#pragma unroll
            for (int j = 0; j < T; ++j) {
              const double t1r = fma(zr[j], h1r[j], fma(zi[j], h1i[j], a.x));
              const double t1i = fma(zr[j], h1i[j], fma(-zi[j], h1r[j], a.y));
              const double t2r = fma(zr[j], h2r[j], fma(-zi[j], h2i[j], bq.x));
              const double t2i = fma(zr[j], h2i[j], fma(zi[j], h2r[j], bq.y));
              const double t3r = fma(zr[j], h3r[j], fma(-zi[j], h3i[j], g.x));
              const double t3i = fma(zr[j], h3i[j], fma(zi[j], h3r[j], g.y));
              h1r[j] = t1r;
              h1i[j] = t1i;
              h2r[j] = t2r;
              h2i[j] = t2i;
              h3r[j] = t3r;
              h3i[j] = t3i;
            }
          }
          const double2 g0 = cf[2 * kMp64Order], dl = cf[3 * kMp64Order + 1];
#pragma unroll
          for (int j = 0; j < T; ++j) {
            const double p3r = fma(zr[j], h3r[j], fma(-zi[j], h3i[j], g0.x));
            const double p3i = fma(zr[j], h3i[j], fma(zi[j], h3r[j], g0.y));
            const double p1r = fma(zr[j], h1r[j], zi[j] * h1i[j]);
            const double p1i = fma(zr[j], h1i[j], -zi[j] * h1r[j]);
            const double p2r = fma(zr[j], h2r[j], -zi[j] * h2i[j]);
            const double p2i = fma(zr[j], h2i[j], zi[j] * h2r[j]);
            const double f = fma(-q, zr[j] * zr[j] + zi[j] * zi[j], 1.0);
            const double mr = f * fma(Zx[j], p3r, -Zy[j] * p3i) - dl.x;
            const double mi = f * fma(Zx[j], p3i, Zy[j] * p3r) - dl.y;
            const double t3r = 0.5 * fma(zr[j], mr, -zi[j] * mi);
            const double t3i = 0.5 * fma(zr[j], mi, zi[j] * mr);
            const double lZ = fma(-0.5, ln_f64(R2[j]), 0.5);   // -ln|Z| + 1/2
            if (!skip_test(sk[j], mode, kslot, bt[j], nbr_slot)) {
              ax[j] += fma(g0.x, lZ, p1r + p2r + t3r);          // S0 = conj(g0)
              ay[j] += fma(-g0.y, lZ, p1i + p2i + t3i);
            }
          }
          continue;
        }
      }
      double lx[T], ly[T], tx[T], ty[T];
#pragma unroll
      for (int j = 0; j < T; ++j) lx[j] = ly[j] = tx[j] = ty[j] = 0.0;
      const int qe = s_off[kk + 1];
      n_dir += qe - s_off[kk];
      for (int q = s_off[kk]; q < qe; ++q) {
        const double4 s = s_src[q];
#pragma unroll
        for (int j = 0; j < T; ++j) {
          const double dx = x[j] - s.x;
          const double dy = y[j] - s.y;
          const double r2 = fma(dx, dx, dy * dy);
          const double lg = ln_f64(r2);
          const double dot = fma(dx, s.z, dy * s.w) * rcp_f64(r2);
          lx[j] = fma(lg, s.z, lx[j]);
          ly[j] = fma(lg, s.w, ly[j]);
          tx[j] = fma(dot, dx, tx[j]);
          ty[j] = fma(dot, dy, ty[j]);
        }
      }
#pragma unroll
      for (int j = 0; j < T; ++j) {
        if (!skip_test(sk[j], mode, kslot, bt[j], nbr_slot)) {
          ax[j] += fma(-0.5, lx[j], tx[j]);
          ay[j] += fma(-0.5, ly[j], ty[j]);
        }
      }
    }
  }
  if (le_used) {
    __syncthreads();   // the last tile's reads of LDS are done
    le_reduce<kLoc64>(Lr, Li, s_row, s_le);
#pragma unroll
    for (int j = 0; j < T; ++j) {
      double ux, uy;
      l2p<kLoc64>(s_le, x[j] - bx, y[j] - by, ux, uy);
      ax[j] += ux;
      ay[j] += uy;
    }
    n_l2p = T;
  }
  add_work(work, T * n_dir, T * n_dexp, T * n_cexp, n_m2l, n_l2p);
#pragma unroll
  for (int j = 0; j < T; ++j) {
    if (t[j] < Nt) {
      out[((int64_t)split * Nt + tt[j]) * 2] = ax[j] * scale;
      out[((int64_t)split * Nt + tt[j]) * 2 + 1] = ay[j] * scale;
    }
  }
}

__global__ void k_zero_work(unsigned long long* work) {
  if (threadIdx.x < 5) work[threadIdx.x] = 0ull;
}

__global__ void k_reduce_splits(int64_t n2, int nsplit, const double* __restrict__ part, double* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  double s = 0.0;
  for (int p = 0; p < nsplit; ++p) s += part[(int64_t)p * n2 + i];
  u[i] = s;
}



// ---------------------------------------------------------------------------
// Step 2b, per pair, in source form.  The kernel sum skipped each disk's own
// sources and those of its contact partners; in exact arithmetic Alg. 3 leaves, on
// body i of pair c = (i, k), the field of k's corrections from its other pairs:
//   corr^c_i = S^(ik) Pi sum_{c' contains k, c' != c} lambda_tilde^{c'}_k
// (the self blocks P Pi (.) of step 2b and the neighbour one-body terms H mu cancel
// exactly against the skipped terms).  Evaluated directly in FP64, relative to c_k.
// Five waves per pair: the 2 (M_i + M_k) (node, half of the partner's sources) items of a pair of
// 72-node disks fill 288 of the 320 lanes in one pass.
constexpr int kFieldThreads = 320;
__global__ __launch_bounds__(kFieldThreads) void k_pair_field(
    int C, int mobility, const int* __restrict__ pairs, const int* __restrict__ cls,
    const int* __restrict__ src_off, const int* __restrict__ col_off, ClassTab ct,
    const double* __restrict__ centers, const int64_t* __restrict__ xoff, const int64_t* __restrict__ coff,
    const int* __restrict__ bp_off, const int* __restrict__ bp_list, const double* __restrict__ ltil,
    double inv4pimu, double* __restrict__ corr) {
  const int c = blockIdx.x;
  if (c >= C) return;
  const int i = pairs[2 * c], k = pairs[2 * c + 1];
  const int ci = cls[i], ck = cls[k];
  const int nci = ct.nc[ci], nck = ct.nc[ck], mci = ct.mc[ci], mck = ct.mc[ck];
  __shared__ double s_vi[2 * kMaxCol];
  __shared__ double s_vk[2 * kMaxCol];
  __shared__ double red[64];
  // sums over the other pairs of i (for the field on k) and of k (for the field on i)
  const bool other_i = bp_off[i + 1] - bp_off[i] > 1, other_k = bp_off[k + 1] - bp_off[k] > 1;
  if (!other_i && !other_k) {
    for (int q = threadIdx.x; q < 2 * (mci + mck); q += kFieldThreads) corr[coff[c] + q] = 0.0;
    return;
  }
  for (int side = 0; side < 2; ++side) {
    const int b = side ? k : i;
    const int n2 = 2 * (side ? nck : nci);
    double* s_v = side ? s_vk : s_vi;
    for (int q = threadIdx.x; q < n2; q += kFieldThreads) {
      double v = 0.0;
      for (int e = bp_off[b]; e < bp_off[b + 1]; ++e) {
        const int cc = bp_list[e] >> 1, sd = bp_list[e] & 1;
        if (cc == c) continue;
        const int64_t off = xoff[cc] + (sd ? 2 * (src_off[pairs[2 * cc] + 1] - src_off[pairs[2 * cc]]) : 0);
        v += ltil[off + q];
      }
      s_v[q] = v;
    }
  }
  __syncthreads();
  if (mobility) {
    project_rigid<kFieldThreads>(s_vi, nci, ct.Yr[ci], ct.KtKi[ci], red);
    project_rigid<kFieldThreads>(s_vk, nck, ct.Yr[ck], ct.KtKi[ck], red);
  }
  const double dcx = centers[2 * i] - centers[2 * k], dcy = centers[2 * i + 1] - centers[2 * k + 1];
  // item it: node q = it / 2, half h = it % 2 of the partner's sources; the two halves sit in
  // adjacent lanes (the item count is even) and are added with one shuffle
  for (int it = threadIdx.x; it < 2 * (mci + mck); it += kFieldThreads) {
    const int q = it >> 1, h = it & 1;
    double tx, ty;
    const double* Ys;
    const double* vs;
    int ns;
    if (q < mci) {  // node q of body i, sources of body k (coordinates relative to c_k)
      tx = ct.Xr[ci][2 * q] + dcx;
      ty = ct.Xr[ci][2 * q + 1] + dcy;
      Ys = ct.Yr[ck];
      vs = s_vk;
      ns = other_k ? nck : 0;
    } else {        // node of body k, sources of body i (relative to c_i)
      const int qq = q - mci;
      tx = ct.Xr[ck][2 * qq] - dcx;
      ty = ct.Xr[ck][2 * qq + 1] - dcy;
      Ys = ct.Yr[ci];
      vs = s_vi;
      ns = other_i ? nci : 0;
    }
    double lx = 0, ly = 0, px = 0, py = 0;
    const int s1 = h ? ns : ns / 2;
    for (int s = h ? ns / 2 : 0; s < s1; ++s) {
      const double dx = tx - Ys[2 * s], dy = ty - Ys[2 * s + 1];
      const double r2 = fma(dx, dx, dy * dy);
      const double lg = ln_f64(r2);
      const double sx = vs[2 * s], sy = vs[2 * s + 1];
      const double dot = fma(dx, sx, dy * sy) * rcp_f64(r2);
      lx = fma(lg, sx, lx);
      ly = fma(lg, sy, ly);
      px = fma(dot, dx, px);
      py = fma(dot, dy, py);
    }
    double ox = fma(-0.5, lx, px), oy = fma(-0.5, ly, py);
    ox += __shfl_xor(ox, 1, 64);
    oy += __shfl_xor(oy, 1, 64);
    if (h == 0) {
      corr[coff[c] + 2 * q] = ox * inv4pimu;
      corr[coff[c] + 2 * q + 1] = oy * inv4pimu;
    }
  }
}

// Identity fix and gather of the pair field corrections:
// u^(b) = u_sum^(b) + mu^(b) + sum_{c contains b} corr^c_b.
__global__ __launch_bounds__(kBodyThreads) void k_finish(int P, const int* __restrict__ col_off,
                                                         const int* __restrict__ bp_off,
                                                         const int* __restrict__ bp_list,
                                                         const int* __restrict__ pairs,
                                                         const int64_t* __restrict__ coff,
                                                         const double* __restrict__ usum,
                                                         const double* __restrict__ mu,
                                                         const double* __restrict__ corr, int with_pairs,
                                                         double* __restrict__ uout) {
  const int b = blockIdx.x;
  if (b >= P) return;
  const int64_t o = 2 * (int64_t)col_off[b];
  const int m2 = 2 * (col_off[b + 1] - col_off[b]);
  for (int q = threadIdx.x; q < m2; q += kBodyThreads) {
    double v = usum[o + q] + mu[o + q];
    if (with_pairs) {
      for (int e = bp_off[b]; e < bp_off[b + 1]; ++e) {
        const int c = bp_list[e] >> 1, side = bp_list[e] & 1;
        const int i = pairs[2 * c];
        const int64_t off = coff[c] + (side ? 2 * (col_off[i + 1] - col_off[i]) : 0);
        v += corr[off + q];
      }
    }
    uout[o + q] = v;
  }
}

// ---------------------------------------------------------------------------
// Mobility RHS sources: lambda_0^(b) = K (K^T K)^{-1} [f; t]^(b) (Sec. 4.1), packed with absolute coordinates.
__global__ __launch_bounds__(kBodyThreads) void k_rhs_sources(int P, const int* __restrict__ cls,
                                                             const int* __restrict__ src_off, ClassTab ct,
                                                             const double* __restrict__ centers,
                                                             const double* __restrict__ given,
                                                             double4* __restrict__ src64, int accumulate) {
  const int b = blockIdx.x;
  if (b >= P) return;
  const int k = cls[b];
  const double* Q = ct.KtKi[k];
  const double f0 = given[3 * b], f1 = given[3 * b + 1], f2 = given[3 * b + 2];
  const double a0 = Q[0] * f0 + Q[1] * f1 + Q[2] * f2;
  const double a1 = Q[3] * f0 + Q[4] * f1 + Q[5] * f2;
  const double a2 = Q[6] * f0 + Q[7] * f1 + Q[8] * f2;
  const double cx = centers[2 * b], cy = centers[2 * b + 1];
  const double* Yr = ct.Yr[k];
  for (int j = threadIdx.x; j < ct.nc[k]; j += kBodyThreads) {
    const double yx = Yr[2 * j], yy = Yr[2 * j + 1];
    const int64_t o = src_off[b] + j;
    if (accumulate) {   // add lambda_0 to strengths already packed with their positions
      src64[o].z += a0 - a2 * yy;
      src64[o].w += a1 + a2 * yx;
    } else {
      src64[o] = make_double4(cx + yx, cy + yy, a0 - a2 * yy, a1 + a2 * yx);
    }
  }
}

// Resistance RHS: b = v + omega (x - c)^perp at every coarse node (eq. rigidbc).
__global__ void k_rhs_resistance(int64_t Nt, const int* __restrict__ tgt_body, const double* __restrict__ X,
                                 const double* __restrict__ centers, const double* __restrict__ given,
                                 double* __restrict__ b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Nt) return;
  const int p = tgt_body[t];
  const double rx = X[2 * t] - centers[2 * p], ry = X[2 * t + 1] - centers[2 * p + 1];
  b[2 * t] = given[3 * p] - given[3 * p + 2] * ry;
  b[2 * t + 1] = given[3 * p + 1] + given[3 * p + 2] * rx;
}

// Post-processing, per pair: e^c = E^c [lambda_bar^(i); lambda_bar^(k)] (6 values).
__global__ __launch_bounds__(64) void k_post_pairs(int C, const int* __restrict__ pairs,
                                                   const int* __restrict__ src_off, const int64_t* __restrict__ xoff,
                                                   const double* __restrict__ E, const double* __restrict__ lam,
                                                   double* __restrict__ epair) {
  const int c = blockIdx.x;
  if (c >= C) return;
  const int i = pairs[2 * c], k = pairs[2 * c + 1];
  const int ni = 2 * (src_off[i + 1] - src_off[i]);
  const int n = (int)(xoff[c + 1] - xoff[c]);
  const double* Ec = E + 6 * xoff[c];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int q = threadIdx.x; q < n; q += 64) {
    const double x = q < ni ? lam[2 * (int64_t)src_off[i] + q] : lam[2 * (int64_t)src_off[k] + q - ni];
#pragma unroll
    for (int r = 0; r < 6; ++r) acc[r] = fma(Ec[(int64_t)q * 6 + r], x, acc[r]);
  }
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    const double s = wave_sum(acc[r]);
    if (threadIdx.x == 0) epair[6 * c + r] = s;
  }
}

// Per body: out = sgn K^T lambda_bar + sum_c e^c_b (mobility: sgn = -1, eq. rbm_ansatz; resistance: +1).
__global__ __launch_bounds__(64) void k_post_bodies(int P, int mobility, const int* __restrict__ cls,
                                                    const int* __restrict__ src_off, ClassTab ct,
                                                    const int* __restrict__ bp_off, const int* __restrict__ bp_list,
                                                    const double* __restrict__ epair,
                                                    const double* __restrict__ lam, int with_pairs,
                                                    double* __restrict__ out3) {
  const int b = blockIdx.x;
  if (b >= P) return;
  const int k = cls[b];
  const double* Yr = ct.Yr[k];
  const double* lb = lam + 2 * (int64_t)src_off[b];
  double f0 = 0, f1 = 0, f2 = 0;
  for (int j = threadIdx.x; j < ct.nc[k]; j += 64) {
    const double lx = lb[2 * j], ly = lb[2 * j + 1];
    f0 += lx;
    f1 += ly;
    f2 += -Yr[2 * j + 1] * lx + Yr[2 * j] * ly;
  }
  f0 = wave_sum(f0);
  f1 = wave_sum(f1);
  f2 = wave_sum(f2);
  if (threadIdx.x == 0) {
    const double sg = mobility ? -1.0 : 1.0;
    double o0 = sg * f0, o1 = sg * f1, o2 = sg * f2;
    if (with_pairs) {
      for (int e = bp_off[b]; e < bp_off[b + 1]; ++e) {
        const int c = bp_list[e] >> 1, side = bp_list[e] & 1;
        o0 += epair[6 * c + 3 * side];
        o1 += epair[6 * c + 3 * side + 1];
        o2 += epair[6 * c + 3 * side + 2];
      }
    }
    out3[3 * b] = o0;
    out3[3 * b + 1] = o1;
    out3[3 * b + 2] = o2;
  }
}

// ---------------------------------------------------------------------------
// GMRES vector kernels.  Dot products: block partials in a fixed order, then a
// per-vector sum over blocks in a fixed order.
constexpr int kDotThreads = 256;

__global__ __launch_bounds__(kDotThreads) void k_mdot(int64_t n, int k, const double* __restrict__ V, int64_t ldv,
                                                      const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double red[16];
  const int64_t chunk = ((n + gridDim.x - 1) / gridDim.x + kDotThreads - 1) / kDotThreads * kDotThreads;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = min(n, lo + chunk);
  int j = 0;
  // four products per pass over w (each summed in the same order as alone)
  for (; j + 4 <= k; j += 4) {
    const double* v = V + (int64_t)j * ldv;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kDotThreads) {
      const double wi = w[i];
      a0 = fma(v[i], wi, a0);
      a1 = fma(v[ldv + i], wi, a1);
      a2 = fma(v[2 * ldv + i], wi, a2);
      a3 = fma(v[3 * ldv + i], wi, a3);
    }
    a0 = block_sum<kDotThreads>(a0, red);
    a1 = block_sum<kDotThreads>(a1, red);
    a2 = block_sum<kDotThreads>(a2, red);
    a3 = block_sum<kDotThreads>(a3, red);
    if (threadIdx.x == 0) {
      part[(int64_t)j * gridDim.x + blockIdx.x] = a0;
      part[(int64_t)(j + 1) * gridDim.x + blockIdx.x] = a1;
      part[(int64_t)(j + 2) * gridDim.x + blockIdx.x] = a2;
      part[(int64_t)(j + 3) * gridDim.x + blockIdx.x] = a3;
    }
  }
  for (; j < k; ++j) {
    const double* v = V + (int64_t)j * ldv;
    double acc = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kDotThreads) acc = fma(v[i], w[i], acc);
    acc = block_sum<kDotThreads>(acc, red);
    if (threadIdx.x == 0) part[(int64_t)j * gridDim.x + blockIdx.x] = acc;
  }
}

// out[j] = sum over the nblk block partials of product j (part: k rows of nblk), one
// workgroup per product in a fixed order (strided per-thread sums, then the block tree)
__global__ __launch_bounds__(kDotThreads) void k_mdot_reduce(int k, int nblk, const double* __restrict__ part,
                                                             double* __restrict__ out) {
  __shared__ double red[16];
  const int j = blockIdx.x;
  if (j >= k) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kDotThreads) s += part[(int64_t)j * nblk + b];
  s = block_sum<kDotThreads>(s, red);
  if (threadIdx.x == 0) out[j] = s;
}

__global__ void k_maxpy(int64_t n, int k, const double* __restrict__ V, int64_t ldv, const double* __restrict__ h,
                        double* __restrict__ w) {
  __shared__ double s_h[1024];
  for (int j = threadIdx.x; j < k; j += blockDim.x) s_h[j] = h[j];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = w[i];
#pragma unroll 8
  for (int j = 0; j < k; ++j) acc = fma(-s_h[j], V[(int64_t)j * ldv + i], acc);
  w[i] = acc;
}

__global__ void k_gemv_n(int64_t n, int k, const double* __restrict__ V, int64_t ldv, const double* __restrict__ y,
                         double* __restrict__ x) {
  __shared__ double s_y[1024];
  for (int j = threadIdx.x; j < k; j += blockDim.x) s_y[j] = y[j];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = x[i];
  for (int j = 0; j < k; ++j) acc = fma(s_y[j], V[(int64_t)j * ldv + i], acc);
  x[i] = acc;
}

// ---------------------------------------------------------------------------
// GMRES least squares on the device (Alg. 2, GMRES).  One wave per right-hand side r adds
// column j to the Hessenberg matrix (the two CGS2 coefficient sets plus the norm of the
// orthogonalised vector), applies the previous Givens rotations and a new one, updates the
// rotated right-hand side g and records the residual estimate |g_{j+1}| / beta.  Once the
// estimate reaches tol beta (or h_{j+1,j} = 0) the right-hand side is done: later calls leave
// its state alone and set its scale to 0, so its next basis vectors are zero.  Per right-hand
// side: H column-major (cap + 1) x cap, cs and sn (cap), g (cap + 1), ctl (kGmCtl values) and,
// per iteration, rec[(j R + r) 4 ..] = estimate, done, iterations, non-finite flag (for the host).
__global__ __launch_bounds__(64) void k_givens(int j, int cap, int R, const double* __restrict__ hdev,
                                               int64_t hstride, double* __restrict__ H, double* __restrict__ cs,
                                               double* __restrict__ sn, double* __restrict__ g,
                                               double* __restrict__ ctl, double* __restrict__ rec) {
  __shared__ double col[1026];
  __shared__ double s_cs[1024], s_sn[1024];
  const int r = blockIdx.x;
  if (r >= R || j >= cap) return;
  double* c = ctl + (int64_t)r * kGmCtl;
  const bool done = c[kGmDone] != 0.0;
  const double* hq = hdev + (int64_t)r * hstride;
  double* csr = cs + (int64_t)r * cap;
  double* snr = sn + (int64_t)r * cap;
  if (!done) {
    for (int i = threadIdx.x; i <= j; i += 64) col[i] = hq[i] + hq[(cap + 2) + i];
    for (int i = threadIdx.x; i < j; i += 64) {
      s_cs[i] = csr[i];
      s_sn[i] = snr[i];
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double* o = rec + ((int64_t)j * R + r) * 4;
  if (done) {
    c[kGmInv] = 0.0;
    o[0] = c[kGmEst];
    o[1] = 1.0;
    o[2] = c[kGmK];
    o[3] = c[kGmBad];
    return;
  }
  const double hn = sqrt(fmax(0.0, hq[2 * (cap + 2)]));
  bool bad = !isfinite(hn);
  for (int i = 0; i <= j; ++i) bad = bad || !isfinite(col[i]);
  if (bad) {
    c[kGmBad] = 1.0;
    c[kGmDone] = 1.0;
    c[kGmInv] = 0.0;
    o[0] = c[kGmEst];
    o[1] = 1.0;
    o[2] = c[kGmK];
    o[3] = 1.0;
    return;
  }
  // previous rotations, the running entry kept in a register
  double a = col[0];
  for (int i = 0; i < j; ++i) {
    const double b = col[i + 1];
    col[i] = s_cs[i] * a + s_sn[i] * b;
    a = -s_sn[i] * a + s_cs[i] * b;
  }
  const double den = hypot(a, hn);
  const double cj = a / den, sj = hn / den;
  col[j] = den;
  double* Hc = H + (int64_t)r * (cap + 1) * cap + (int64_t)j * (cap + 1);
  for (int i = 0; i <= j; ++i) Hc[i] = col[i];
  Hc[j + 1] = 0.0;
  csr[j] = cj;
  snr[j] = sj;
  double* gr = g + (int64_t)r * (cap + 1);
  const double gj = gr[j];
  gr[j + 1] = -sj * gj;
  gr[j] = cj * gj;
  const double est = fabs(gr[j + 1]) / c[kGmBeta];
  const bool conv = fabs(gr[j + 1]) <= c[kGmTol] || hn == 0.0;
  c[kGmK] = (double)(j + 1);
  c[kGmEst] = est;
  c[kGmInv] = hn > 0.0 ? 1.0 / hn : 0.0;
  if (conv) c[kGmDone] = 1.0;
  o[0] = est;
  o[1] = conv ? 1.0 : 0.0;
  o[2] = (double)(j + 1);
  o[3] = 0.0;
}

// y = x * ctl[kGmInv] for each right-hand side (blockIdx.y): the next basis vector
__global__ void k_scale_ctl(int64_t n, const double* __restrict__ ctl, const double* __restrict__ x,
                            double* __restrict__ y) {
  const int r = blockIdx.y;
  const double a = ctl[(int64_t)r * kGmCtl + kGmInv];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[(int64_t)r * n + i] = x[(int64_t)r * n + i] * a;
}

// y = H(0:k, 0:k)^{-1} g(0:k) by back substitution, k = ctl[kGmK] (one workgroup per
// right-hand side, the solution held in LDS, a column of H per step)
__global__ __launch_bounds__(256) void k_backsolve(int cap, const double* __restrict__ H,
                                                   const double* __restrict__ g, const double* __restrict__ ctl,
                                                   double* __restrict__ y) {
  __shared__ double s_y[1024];
  const int r = blockIdx.x;
  const int k = (int)ctl[(int64_t)r * kGmCtl + kGmK];
  const double* Hr = H + (int64_t)r * (cap + 1) * cap;
  const double* gr = g + (int64_t)r * (cap + 1);
  for (int i = threadIdx.x; i < k; i += 256) s_y[i] = gr[i];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const double* Hi = Hr + (int64_t)i * (cap + 1);
    const double yi = s_y[i] / Hi[i];
    __syncthreads();
    for (int q = threadIdx.x; q < i; q += 256) s_y[q] -= Hi[q] * yi;
    if (threadIdx.x == 0) s_y[i] = yi;
    __syncthreads();
  }
  for (int i = threadIdx.x; i < k; i += 256) y[(int64_t)r * (cap + 1) + i] = s_y[i];
}

__global__ void k_scale_copy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = fma(a, x[i], b * y[i]);
}

// ---------------------------------------------------------------------------
// Flow evaluation (Sec. 3.3, eq. chi; the source triplet Alg. 2 returns for flowEval).
// The far field is the FP64 all-pairs sum of the total coarse strengths Pi (lambda_bar +
// sum lambda_tilde) (plus lambda_0 for mobility) at the evaluation points; at a point
// near pair c (on one of its disks, or in the fluid inside its peanut) the pair's
// compressed strengths Pi lambda_tilde^c are taken out again and its fine correction
// -S(x, Yf^c) sigma_f^c put in, sigma_f^c = Pi_f G^c [lambda_bar_i; lambda_bar_k].

// Per pair: sigma_f (rows of the compact G times the pair's lambda_bar, then the
// per-disk rigid projection of the fine sources for mobility) and Pi lambda_tilde.
__global__ __launch_bounds__(kPairThreads) void k_fine_strengths(
    int C, int mobility, const int* __restrict__ pairs, const int* __restrict__ cls,
    const int* __restrict__ src_off, ClassTab ct, const double* __restrict__ centers,
    const int64_t* __restrict__ xoff, const double* __restrict__ lam_bar, const double* __restrict__ ltil,
    const double* __restrict__ G, const int64_t* __restrict__ goff, const double* __restrict__ Yf,
    const int64_t* __restrict__ yoff, const int32_t* __restrict__ nf, const double* __restrict__ KKf,
    double* __restrict__ ptil, double* __restrict__ sigf) {
  const int c = blockIdx.x;
  if (c >= C) return;
  __shared__ double s_x[4 * kMaxCol];
  __shared__ double red[48];
  const int i = pairs[2 * c], k = pairs[2 * c + 1];
  const int ni = 2 * (src_off[i + 1] - src_off[i]);
  const int n = (int)(xoff[c + 1] - xoff[c]);
  for (int q = threadIdx.x; q < n; q += kPairThreads)
    s_x[q] = q < ni ? lam_bar[2 * (int64_t)src_off[i] + q] : lam_bar[2 * (int64_t)src_off[k] + (q - ni)];
  __syncthreads();
  const int nf0 = nf[2 * c], nf1 = nf[2 * c + 1];
  const int nfr = 2 * (nf0 + nf1);
  const double* Gc = G + goff[c];
  double* sc = sigf + yoff[c];
  for (int r = threadIdx.x; r < nfr; r += kPairThreads) {
    double acc = 0.0;
    for (int q = 0; q < n; ++q) acc = fma(Gc[(int64_t)q * nfr + r], s_x[q], acc);
    sc[r] = acc;
  }
  __syncthreads();
  if (mobility) {
    const double* yf = Yf + yoff[c];
    for (int b = 0; b < 2; ++b) {
      const int s0 = b ? nf0 : 0, s1 = b ? nf0 + nf1 : nf0;
      const double cx = centers[2 * (b ? k : i)], cy = centers[2 * (b ? k : i) + 1];
      double f0 = 0, f1 = 0, f2 = 0;
      for (int q = s0 + threadIdx.x; q < s1; q += kPairThreads) {
        const double bx = sc[2 * q], by = sc[2 * q + 1];
        f0 += bx;
        f1 += by;
        f2 += -(yf[2 * q + 1] - cy) * bx + (yf[2 * q] - cx) * by;
      }
      f0 = block_sum<kPairThreads>(f0, red);
      f1 = block_sum<kPairThreads>(f1, red + 16);
      f2 = block_sum<kPairThreads>(f2, red + 32);
      const double* Q = KKf + 18 * (int64_t)c + 9 * b;
      const double a0 = Q[0] * f0 + Q[1] * f1 + Q[2] * f2;
      const double a1 = Q[3] * f0 + Q[4] * f1 + Q[5] * f2;
      const double a2 = Q[6] * f0 + Q[7] * f1 + Q[8] * f2;
      __syncthreads();
      for (int q = s0 + threadIdx.x; q < s1; q += kPairThreads) {
        sc[2 * q] -= a0 - a2 * (yf[2 * q + 1] - cy);
        sc[2 * q + 1] -= a1 + a2 * (yf[2 * q] - cx);
      }
      __syncthreads();
    }
  }
  // Pi lambda_tilde, disk by disk
  for (int b = 0; b < 2; ++b) {
    const int body = b ? k : i;
    const int kc = cls[body];
    const int nc = ct.nc[kc];
    const int64_t off = xoff[c] + (b ? ni : 0);
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * nc; q += kPairThreads) s_x[q] = ltil[off + q];
    __syncthreads();
    if (mobility) project_rigid<kPairThreads>(s_x, nc, ct.Yr[kc], ct.KtKi[kc], red);
    for (int q = threadIdx.x; q < 2 * nc; q += kPairThreads) ptil[off + q] = s_x[q];
  }
}

// Point in the peanut of a pair: pg = c_i, c_k, a_i, a_k, lower and upper centres of the
// rolling unit circle.  Inside a disk, or in the waist: inside the quadrilateral
// c_i, m_lo, c_k, m_hi (the rolling circle touches the disks on its edges) and outside
// both rolling circles.
__device__ __forceinline__ bool in_peanut(const double* __restrict__ pg, double x, double y) {
  const double cix = pg[0], ciy = pg[1], ckx = pg[2], cky = pg[3], ai = pg[4], ak = pg[5];
  const double mx = 0.5 * (cix + ckx), my = 0.5 * (ciy + cky);
  const double hd = 0.5 * sqrt((ckx - cix) * (ckx - cix) + (cky - ciy) * (cky - ciy));
  const double rb = hd + fmax(ai, ak);
  if ((x - mx) * (x - mx) + (y - my) * (y - my) > rb * rb) return false;
  if ((x - cix) * (x - cix) + (y - ciy) * (y - ciy) <= ai * ai) return true;
  if ((x - ckx) * (x - ckx) + (y - cky) * (y - cky) <= ak * ak) return true;
  const double qx[4] = {cix, pg[6], ckx, pg[8]}, qy[4] = {ciy, pg[7], cky, pg[9]};
  for (int e = 0; e < 4; ++e) {
    const double ax = qx[e], ay = qy[e], bx = qx[(e + 1) & 3], by = qy[(e + 1) & 3];
    if ((bx - ax) * (y - ay) - (by - ay) * (x - ax) < 0.0) return false;
  }
  const double dlx = x - pg[6], dly = y - pg[7], dhx = x - pg[8], dhy = y - pg[9];
  return dlx * dlx + dly * dly >= 1.0 && dhx * dhx + dhy * dhy >= 1.0;
}

__device__ __forceinline__ void stokes_acc(double x, double y, double sx, double sy, double gx, double gy, double& lx,
                                           double& ly, double& tx, double& ty) {
  const double dx = x - sx, dy = y - sy;
  const double r2 = fma(dx, dx, dy * dy);
  const double lg = ln_f64(r2);
  const double dot = fma(dx, gx, dy * gy) * rcp_f64(r2);
  lx = fma(lg, gx, lx);
  ly = fma(lg, gy, ly);
  tx = fma(dot, dx, tx);
  ty = fma(dot, dy, ty);
}

// One thread per evaluation point: subtract the compressed field and the fine correction
// of every pair the point is near to.  Boundary points (body >= 0) take the pairs of their
// disk; fluid points (body < 0) test every pair's peanut.
__global__ __launch_bounds__(256) void k_flow_near(
    int64_t n_pts, const double* __restrict__ pts, const int32_t* __restrict__ body, int C,
    const int* __restrict__ pairs, const int* __restrict__ src_off, const double* __restrict__ Y,
    const int64_t* __restrict__ xoff, const double* __restrict__ ptil, const double* __restrict__ Yf,
    const int64_t* __restrict__ yoff, const int32_t* __restrict__ nf, const double* __restrict__ sigf,
    const double* __restrict__ pgeo, const int* __restrict__ bp_off, const int* __restrict__ bp_list,
    double scale, double* __restrict__ u) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_pts) return;
  const double x = pts[2 * t], y = pts[2 * t + 1];
  const int b = body[t];
  double lx = 0, ly = 0, tx = 0, ty = 0;
  auto apply = [&](int c) {
    const int i = pairs[2 * c], k = pairs[2 * c + 1];
    const int ni = 2 * (src_off[i + 1] - src_off[i]);
    for (int s = src_off[i]; s < src_off[i + 1]; ++s) {
      const int64_t o = xoff[c] + 2 * (s - src_off[i]);
      stokes_acc(x, y, Y[2 * (int64_t)s], Y[2 * (int64_t)s + 1], ptil[o], ptil[o + 1], lx, ly, tx, ty);
    }
    for (int s = src_off[k]; s < src_off[k + 1]; ++s) {
      const int64_t o = xoff[c] + ni + 2 * (s - src_off[k]);
      stokes_acc(x, y, Y[2 * (int64_t)s], Y[2 * (int64_t)s + 1], ptil[o], ptil[o + 1], lx, ly, tx, ty);
    }
    const int nfp = nf[2 * c] + nf[2 * c + 1];
    const double* yf = Yf + yoff[c];
    const double* sf = sigf + yoff[c];
    for (int q = 0; q < nfp; ++q) stokes_acc(x, y, yf[2 * q], yf[2 * q + 1], sf[2 * q], sf[2 * q + 1], lx, ly, tx, ty);
  };
  if (b >= 0) {
    for (int e = bp_off[b]; e < bp_off[b + 1]; ++e) apply(bp_list[e] >> 1);
  } else {
    for (int c = 0; c < C; ++c)
      if (in_peanut(pgeo + 12 * (int64_t)c, x, y)) apply(c);
  }
  u[2 * t] -= scale * fma(-0.5, lx, tx);
  u[2 * t + 1] -= scale * fma(-0.5, ly, ty);
}

// n points per disk on its boundary at angles 2 pi (j + 1/2) / n.
__global__ void k_boundary_nodes(int P, int n, const int* __restrict__ cls, ClassTab ct,
                                 const double* __restrict__ centers, double* __restrict__ pts,
                                 int32_t* __restrict__ body) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)P * n) return;
  const int b = (int)(t / n), j = (int)(t - (int64_t)b * n);
  const double th = (j + 0.5) * (2.0 * 3.14159265358979323846 / n);
  const double a = ct.radius[cls[b]];
  pts[2 * t] = centers[2 * b] + a * cos(th);
  pts[2 * t + 1] = centers[2 * b + 1] + a * sin(th);
  body[t] = b;
}

// eps_t = |u_t - g(x_t)|, g = v + omega (x - c)^perp of the point's body (eq. residual_x);
// per block the largest eps and |g| go to maxima[2 blk], maxima[2 blk + 1].
__global__ __launch_bounds__(256) void k_boundary_residual(int64_t n_pts, const double* __restrict__ pts,
                                                           const int32_t* __restrict__ body,
                                                           const double* __restrict__ centers,
                                                           const double* __restrict__ u,
                                                           const double* __restrict__ rigid,
                                                           double* __restrict__ eps, double* __restrict__ maxima) {
  __shared__ double s_e[256], s_g[256];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0, gn = 0.0;
  if (t < n_pts) {
    const int b = body[t];
    const double rx = pts[2 * t] - centers[2 * b], ry = pts[2 * t + 1] - centers[2 * b + 1];
    const double gx = rigid[3 * b] - rigid[3 * b + 2] * ry, gy = rigid[3 * b + 1] + rigid[3 * b + 2] * rx;
    const double dx = u[2 * t] - gx, dy = u[2 * t + 1] - gy;
    e = sqrt(dx * dx + dy * dy);
    gn = sqrt(gx * gx + gy * gy);
    if (eps) eps[t] = e;
  }
  s_e[threadIdx.x] = e;
  s_g[threadIdx.x] = gn;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s_e[threadIdx.x] = fmax(s_e[threadIdx.x], s_e[threadIdx.x + h]);
      s_g[threadIdx.x] = fmax(s_g[threadIdx.x], s_g[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    maxima[2 * blockIdx.x] = s_e[0];
    maxima[2 * blockIdx.x + 1] = s_g[0];
  }
}

// One block folds the per-block maxima: out[0] = max eps, out[1] = max |g|.
__global__ __launch_bounds__(256) void k_max_pairs(int nblk, const double* __restrict__ maxima,
                                                   double* __restrict__ out) {
  __shared__ double s_e[256], s_g[256];
  double e = 0.0, g = 0.0;
  for (int q = threadIdx.x; q < nblk; q += 256) {
    e = fmax(e, maxima[2 * q]);
    g = fmax(g, maxima[2 * q + 1]);
  }
  s_e[threadIdx.x] = e;
  s_g[threadIdx.x] = g;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s_e[threadIdx.x] = fmax(s_e[threadIdx.x], s_e[threadIdx.x + h]);
      s_g[threadIdx.x] = fmax(s_g[threadIdx.x], s_g[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s_e[0];
    out[1] = s_g[0];
  }
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------------------
// Hierarchical kernel sum over the context's own targets (Alg. 3 step 2a, eq. getall; the
// paper evaluates it with a fast multipole method, Sec. 6).  Tree and per-wave lists:
// fmm_tree.hip.  Per matvec: the disks' ring expansions and the cells' moments (upward pass),
// then one wave per 64 kFmmT targets: the M2L list into the wave's local expansion, its
// evaluation at the targets (L2P), and the near list, disk by disk, from each disk's ring
// expansion at the lowest tier order whose distance every target of the wave meets, else
// directly over the disk's sources (FP64).  The mixed form evaluates the ring expansions in
// FP32 (coefficients from FP64 moments, which keep the cancellation between the strengths);
// translations, local expansions and direct sums are FP64 in both forms.

// w^e for 0 <= e < 64 by binary powering
__device__ __forceinline__ void cpow_int(double wx, double wy, int e, double& pr, double& pi) {
  pr = 1.0;
  pi = 0.0;
  double br = wx, bi = wy;
  for (; e; e >>= 1) {
    if (e & 1) {
      const double t = pr * br - pi * bi;
      pi = fma(pr, bi, pi * br);
      pr = t;
    }
    const double u = br * br - bi * bi;
    bi = 2.0 * br * bi;
    br = u;
  }
}

// One disk per workgroup, lane e forms the order-e moments of its sources about its centre,
// A_e = sum sigma w^e, B_e = sum sigma conj(w)^e, D_e = sum sigma conj(w) w^e (w = y - c from
// the class ring, sigma from the packed src64), and writes the disk's ring records (FP64 order
// kRing64Order, FP32 order kRing32Order, slot order, with the class's tier distances) and its
// leaf cell (raw moments and the order-kCl64Order record of k_cluster_moments64's layout).
// In the ring records the k = 1 term of the conj(zeta) series, B_1 conj(zeta) / 2, and the
// term -conj(zeta) conj(B_1) / 2 of the third part are merged into i Im(B_1) conj(zeta), and
// conj(B_1) is stored as 0: the dilation moment Re(B_1) = sum y . sigma has no field outside
// the ring, and the one-body map makes it large (the near-null radial mode of the ring), so
// the two terms would otherwise cancel in the evaluation's precision.
__global__ __launch_bounds__(64) void k_ring_moments(int P, const int* __restrict__ cls,
                                                     const int* __restrict__ src_off, ClassTab ct,
                                                     const double4* __restrict__ src64,
                                                     const int* __restrict__ slot_of, const double* __restrict__ centers,
                                                     double2* __restrict__ ring64, float2* __restrict__ ring32,
                                                     double2* __restrict__ cellraw, double2* __restrict__ cellrec) {
  const int b = blockIdx.x;
  if (b >= P) return;
  const double cx = centers[2 * b], cy = centers[2 * b + 1];
  const int e = threadIdx.x;
  const int k = cls[b];
  const int nc = ct.nc[k];
  const double* Yr = ct.Yr[k];
  const int64_t so = src_off[b];
  const int sl = slot_of[b];
  // the disk's strengths and ring offsets staged in LDS with one load per lane (a loop of
  // dependent global loads would wait on memory once per source); the launch gives 2 x the
  // largest class's source count double2 of dynamic LDS
  extern __shared__ double2 s_dyn[];
  double2* s_sig = s_dyn;
  double2* s_w = s_dyn + nc;
  for (int j = e; j < nc; j += 64) {
    const double4 v = src64[so + j];
    s_sig[j] = make_double2(v.z, v.w);
    s_w[j] = make_double2(Yr[2 * j], Yr[2 * j + 1]);
  }
  __syncthreads();
  // The sources are the class's ring w_j = rho exp(2 pi i j / nc) from angle 0 (Yr[0] = (rho, 0)),
  // so w_j^e = rho^(e-1) w_m with m = j e mod nc: one lookup and a real scaling per source
  // instead of a complex power (rho^(e-1) by binary powering once per lane).
  const double rho = Yr[0];
  double re = 1.0;
  {
    double bb = rho;
    for (int t = e - 1; t > 0; t >>= 1) {
      if (t & 1) re *= bb;
      bb *= bb;
    }
  }
  const int em = e % nc;
  int m = 0;
  double Ar = 0, Ai = 0, Br = 0, Bi = 0, Dr = 0, Di = 0;
  for (int j = 0; j < nc; ++j) {
    const double2 sg = s_sig[j], wv = s_w[j], wm = s_w[m];
    m += em;
    if (m >= nc) m -= nc;
    const double4 v = make_double4(0.0, 0.0, sg.x, sg.y);
    const double wx = wv.x, wy = wv.y;
    const double pr = e ? re * wm.x : 1.0, pi = e ? re * wm.y : 0.0;   // w_j^e
    const double sr = v.z * pr - v.w * pi, si = v.z * pi + v.w * pr;   // sigma w^e
    Ar += sr;
    Ai += si;
    Br += v.z * pr + v.w * pi;   // sigma conj(w)^e
    Bi += v.w * pr - v.z * pi;
    Dr += wx * sr + wy * si;     // conj(w) sigma w^e
    Di += wx * si - wy * sr;
  }
  const double rho2 = Yr[0] * Yr[0] + Yr[1] * Yr[1];
  {
    constexpr int Pq = kRing64Order;
    double2* o = ring64 + (int64_t)sl * kRing64Coef;
    if (e >= 1 && e <= Pq) {
      o[e - 1] = make_double2(Ar / (2 * e), Ai / (2 * e));
      o[Pq + e - 1] = e == 1 ? make_double2(0.0, Bi) : make_double2(Br / (2 * e), Bi / (2 * e));
    }
    if (e <= Pq) o[2 * Pq + e] = make_double2(Ar, -Ai);
    if (e == 1) o[3 * Pq + 1] = make_double2(0.0, 0.0);
    if (e == 0) {
      o[3 * Pq + 2] = make_double2(rho2, ct.tier64[k][2]);
      o[3 * Pq + 3] = make_double2(ct.tier64[k][0], ct.tier64[k][1]);
      o[3 * Pq + 4] = make_double2(cx, cy);
      o[3 * Pq + 5] = make_double2((double)b, 0.0);
    }
  }
  if (ring32) {
    constexpr int Pq = kRing32Order;
    float2* o = ring32 + (int64_t)sl * kRing32Coef;
    if (e >= 1 && e <= Pq) {
      o[e - 1] = make_float2((float)(Ar / (2 * e)), (float)(Ai / (2 * e)));
      o[Pq + e - 1] = e == 1 ? make_float2(0.0f, (float)Bi) : make_float2((float)(Br / (2 * e)), (float)(Bi / (2 * e)));
    }
    if (e <= Pq) o[2 * Pq + e] = make_float2((float)Ar, (float)-Ai);
    if (e == 1) o[3 * Pq + 1] = make_float2(0.0f, 0.0f);
    if (e == 0) {
      // distances rounded up in FP32, so that the FP32 comparison never admits a nearer target
      auto up = [](double v) {   // v > 0
        float f = (float)v;
        if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);
        return f;
      };
      o[3 * Pq + 2] = make_float2((float)rho2, up(ct.tier32[k][2]));
      o[3 * Pq + 3] = make_float2(up(ct.tier32[k][0]), up(ct.tier32[k][1]));
      const double hv[3] = {cx, cy, (double)b};
      for (int h = 0; h < 3; ++h) {
        const unsigned long long u = (unsigned long long)__double_as_longlong(hv[h]);
        o[3 * Pq + 4 + h] = make_float2(__uint_as_float((unsigned)u), __uint_as_float((unsigned)(u >> 32)));
      }
      o[3 * Pq + 7] = make_float2(0.0f, 0.0f);
    }
  }
  if (e <= kCl64Order) {
    double2* r = cellraw + (int64_t)sl * kCellRaw;
    r[e] = make_double2(Ar, Ai);
    r[kCl64Order + 1 + e] = make_double2(Br, Bi);
    r[2 * (kCl64Order + 1) + e] = make_double2(Dr, Di);
    double2* o = cellrec + (int64_t)sl * kCellRec;
    if (e >= 1) {
      o[e - 1] = make_double2(Ar / (2 * e), Ai / (2 * e));
      o[kCl64Order + e - 1] = make_double2(Br / (2 * e), Bi / (2 * e));
    }
    o[2 * kCl64Order + e] = make_double2(Ar, -Ai);
    o[3 * kCl64Order + 1 + e] = make_double2(Dr, -Di);
    if (e == 0) {
      o[kCl64CoefPerCluster] = make_double2(cx, cy);
      o[kCl64CoefPerCluster + 1] = make_double2(0.0, 0.0);
    }
  }
}

// Upward pass, one wave per internal cell of one height: its children's moments moved to the
// cell's centre C and summed.  With delta = C_child - C, w' = w + delta:
//   A'_k = sum_j binom(k, j) delta^(k-j) A_j,   B'_k = sum_j binom(k, j) conj(delta)^(k-j) B_j,
//   D'_k = sum_j binom(k, j) delta^(k-j) (D_j + conj(delta) A_j).
// Lane k <= kCl64Order forms A'_k and D'_k, lane 32 + k forms B'_k; each child's raw moments and
// the powers of its delta are staged in LDS first.
// One workgroup per cell, one wave per child (children w, w + 4, ... to wave w); the waves' sums
// are added in wave order.
constexpr int kM2mWaves = 4;
__global__ __launch_bounds__(64 * kM2mWaves) void k_cell_m2m(int n, const int* __restrict__ cells,
                                                 const int* __restrict__ child_off, const int* __restrict__ child,
                                                 const double* __restrict__ cell_c, double2* __restrict__ raw,
                                                 double2* __restrict__ rec) {
  static_assert(kCl64Order < 32 && kCellRaw <= 128, "one lane per order, two raw entries per lane");
  if ((int)blockIdx.x >= n) return;
  const int q = cells[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, f = lane >> 5, k = lane & 31;
  const double cx = cell_c[2 * q], cy = cell_c[2 * q + 1];
  __shared__ double2 s_pw_all[kM2mWaves][32];          // delta^m
  __shared__ double2 s_raw_all[kM2mWaves][kCellRaw];   // the child's A, B, D
  __shared__ double4 s_acc[kM2mWaves - 1][64];         // the sums of waves 1, 2, 3
  double2* s_pw = s_pw_all[wv];
  double2* s_raw = s_raw_all[wv];
  double ar = 0, ai = 0, dr = 0, di = 0;
  for (int e = child_off[q] + wv; e < child_off[q + 1]; e += kM2mWaves) {
    const int ch = child[e];
    const double dx = cell_c[2 * ch] - cx, dy = cell_c[2 * ch + 1] - cy;
    const double2* cr = raw + (int64_t)ch * kCellRaw;
    const double2 v0 = cr[lane];
    const double2 v1 = lane + 64 < kCellRaw ? cr[lane + 64] : make_double2(0.0, 0.0);
    double pr = 0.0, pi = 0.0;
    if (lane < 32) cpow_int(dx, dy, lane, pr, pi);
    wave_lds_sync();   // the previous child's reads are done
    s_raw[lane] = v0;
    if (lane + 64 < kCellRaw) s_raw[lane + 64] = v1;
    if (lane < 32) s_pw[lane] = make_double2(pr, pi);
    wave_lds_sync();
    if (k <= kCl64Order) {
      double bn = 1.0;   // binom(k, j)
      for (int j = 0; j <= k; ++j) {
        const double2 pw = s_pw[k - j];
        const double pwr = pw.x, pwi = f == 0 ? pw.y : -pw.y;
        const double cr2 = bn * pwr, ci2 = bn * pwi;
        if (f == 0) {
          const double2 a = s_raw[j], d = s_raw[2 * (kCl64Order + 1) + j];
          ar = fma(cr2, a.x, fma(-ci2, a.y, ar));
          ai = fma(cr2, a.y, fma(ci2, a.x, ai));
          // D_j + conj(delta) A_j
          const double gr = d.x + (dx * a.x + dy * a.y), gi = d.y + (dx * a.y - dy * a.x);
          dr = fma(cr2, gr, fma(-ci2, gi, dr));
          di = fma(cr2, gi, fma(ci2, gr, di));
        } else {
          const double2 bq = s_raw[kCl64Order + 1 + j];
          ar = fma(cr2, bq.x, fma(-ci2, bq.y, ar));
          ai = fma(cr2, bq.y, fma(ci2, bq.x, ai));
        }
        bn = bn * (double)(k - j) * kInvInt[j + 1];
      }
    }
  }
  if (wv > 0) s_acc[wv - 1][lane] = make_double4(ar, ai, dr, di);
  __syncthreads();
  if (wv > 0) return;
#pragma unroll
  for (int w = 0; w < kM2mWaves - 1; ++w) {
    const double4 t = s_acc[w][lane];
    ar += t.x;
    ai += t.y;
    dr += t.z;
    di += t.w;
  }
  if (lane == 0) {
    double2* o = rec + (int64_t)q * kCellRec;
    o[kCl64CoefPerCluster] = make_double2(cx, cy);
    o[kCl64CoefPerCluster + 1] = make_double2(0.0, 0.0);
  }
  if (k > kCl64Order) return;
  double2* r = raw + (int64_t)q * kCellRaw;
  double2* o = rec + (int64_t)q * kCellRec;
  if (f == 0) {
    r[k] = make_double2(ar, ai);
    r[2 * (kCl64Order + 1) + k] = make_double2(dr, di);
    if (k >= 1) o[k - 1] = make_double2(ar / (2 * k), ai / (2 * k));
    o[2 * kCl64Order + k] = make_double2(ar, -ai);
    o[3 * kCl64Order + 1 + k] = make_double2(dr, -di);
  } else {
    r[kCl64Order + 1 + k] = make_double2(ar, ai);
    if (k >= 1) o[kCl64Order + k - 1] = make_double2(ar / (2 * k), ai / (2 * k));
  }
}

// Ring expansion of one disk (record cf of order Pq, evaluated to order p <= Pq) added at a
// thread's targets (offsets Zx, Zy from the disk's centre, R2 = |Z|^2, q = rho^2) where not
// skipped: the series of k_gather_project's far field in precision Real.
template <typename Real, typename C2, int T>
__device__ __forceinline__ void ring_m2p(const C2* __restrict__ cf, int Pq, int p, Real q, const Real (&Zx)[T],
                                         const Real (&Zy)[T], const Real (&R2)[T], const bool (&skip)[T],
                                         double (&ax)[T], double (&ay)[T]) {
  Real zr[T], zi[T], h1r[T], h1i[T], h2r[T], h2i[T], h3r[T], h3i[T];
  const C2 c1 = cf[p - 1], c2 = cf[Pq + p - 1], c3 = cf[2 * Pq + p];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    Real ir2;
    if constexpr (sizeof(Real) == 4)
      ir2 = __builtin_amdgcn_rcpf(R2[j]);
    else
      ir2 = rcp_f64(R2[j]);
    zr[j] = Zx[j] * ir2;   // zeta = conj(Z) / R^2 = (zr, -zi); conj(zeta) = (zr, zi)
    zi[j] = Zy[j] * ir2;
    h1r[j] = c1.x;
    h1i[j] = c1.y;
    h2r[j] = c2.x;
    h2i[j] = c2.y;
    h3r[j] = c3.x;
    h3i[j] = c3.y;
  }
  // Horner: h1 over zeta (A_k/2k), h2 over conj(zeta) (B_k/2k), h3 over conj(zeta) (conj A_k)
#pragma unroll 2
  for (int m = p - 1; m >= 1; --m) {
    const C2 a = cf[m - 1], bq = cf[Pq + m - 1], g = cf[2 * Pq + m];
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const Real t1r = fma(zr[j], h1r[j], fma(zi[j], h1i[j], a.x));
      const Real t1i = fma(zr[j], h1i[j], fma(-zi[j], h1r[j], a.y));
      const Real t2r = fma(zr[j], h2r[j], fma(-zi[j], h2i[j], bq.x));
      const Real t2i = fma(zr[j], h2i[j], fma(zi[j], h2r[j], bq.y));
      const Real t3r = fma(zr[j], h3r[j], fma(-zi[j], h3i[j], g.x));
      const Real t3i = fma(zr[j], h3i[j], fma(zi[j], h3r[j], g.y));
      h1r[j] = t1r;
      h1i[j] = t1i;
      h2r[j] = t2r;
      h2i[j] = t2i;
      h3r[j] = t3r;
      h3i[j] = t3i;
    }
  }
  const C2 g0 = cf[2 * Pq], dl = cf[3 * Pq + 1];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    // P3 = conj(A_0) + conj(zeta) h3; P1 = zeta h1; P2 = conj(zeta) h2
    const Real p3r = fma(zr[j], h3r[j], fma(-zi[j], h3i[j], g0.x));
    const Real p3i = fma(zr[j], h3i[j], fma(zi[j], h3r[j], g0.y));
    const Real p1r = fma(zr[j], h1r[j], zi[j] * h1i[j]);
    const Real p1i = fma(zr[j], h1i[j], -zi[j] * h1r[j]);
    const Real p2r = fma(zr[j], h2r[j], -zi[j] * h2i[j]);
    const Real p2i = fma(zr[j], h2i[j], zi[j] * h2r[j]);
    // conj(zeta)/2 [(Z - rho^2 conj(zeta)) P3 - conj(B_1)], Z - rho^2 conj(zeta) = Z (1 - q / R^2)
    const Real fq = fma(-q, zr[j] * zr[j] + zi[j] * zi[j], Real(1));
    const Real mr = fq * fma(Zx[j], p3r, -Zy[j] * p3i) - dl.x;
    const Real mi = fq * fma(Zx[j], p3i, Zy[j] * p3r) - dl.y;
    const Real t3r = Real(0.5) * fma(zr[j], mr, -zi[j] * mi);
    const Real t3i = Real(0.5) * fma(zr[j], mi, zi[j] * mr);
    // -S0 ln|Z| + S0 / 2
    Real lZ;
    if constexpr (sizeof(Real) == 4)
      lZ = fmaf(-0.34657359027997264f, __builtin_amdgcn_logf(R2[j]), 0.5f);
    else
      lZ = fma(-0.5, ln_f64(R2[j]), 0.5);
    const Real fx = fma(g0.x, lZ, p1r + p2r + t3r);   // S0 = conj(g0)
    const Real fy = fma(-g0.y, lZ, p1i + p2i + t3i);
    if (!skip[j]) {
      ax[j] += (double)fx;
      ay[j] += (double)fy;
    }
  }
}

// The same in FP32 with two of the three series merged.
template <typename Real, typename C2, int T>
__device__ __forceinline__ void ring_m2p_merged(const C2* __restrict__ cf, int Pq, int p, Real q, const Real (&Zx)[T],
                                         const Real (&Zy)[T], const Real (&R2)[T], const bool (&skip)[T],
                                         double (&ax)[T], double (&ay)[T]) {
  // The three series of the far field, with zeta = conj(Z) / R^2 (so Z = R^2 conj(zeta)):
  //   P1 = sum_k A_k/(2k) zeta^k, P2 = sum_k B_k/(2k) conj(zeta)^k, P3 = sum_k conj(A_k) conj(zeta)^k,
  //   u = P1 + P2 + conj(zeta)/2 [(Z - rho^2 conj(zeta)) P3 - conj(B_1)] - S0 ln|Z| + S0/2.
  // (Z - rho^2 conj(zeta)) conj(zeta)/2 = s conj(zeta)^2 with s = (R^2 - rho^2)/2 real, so P2 and the
  // P3 term are one polynomial in conj(zeta) whose coefficients are B_{j+1}/(2j+2) + s conj(A_{j-1})
  // (degree p + 1), evaluated by one Horner series: 10 FMAs a step instead of 12.  (In FP64 the
  // separate series of ring_m2p keep the solve's attainable residual about half as large.)
  Real zr[T], zi[T], s[T], h1r[T], h1i[T], hr[T], hi[T];
  const C2 c1 = cf[p - 1], gp = cf[2 * Pq + p], gq = cf[2 * Pq + p - 1];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    Real ir2;
    if constexpr (sizeof(Real) == 4)
      ir2 = __builtin_amdgcn_rcpf(R2[j]);
    else
      ir2 = rcp_f64(R2[j]);
    zr[j] = Zx[j] * ir2;   // zeta = (zr, -zi); conj(zeta) = (zr, zi)
    zi[j] = Zy[j] * ir2;
    s[j] = Real(0.5) * (R2[j] - q);
    h1r[j] = c1.x;
    h1i[j] = c1.y;
    // the two leading coefficients, s conj(A_p) and s conj(A_{p-1}) (no B beyond order p)
    const Real er = s[j] * gq.x, ei = s[j] * gq.y;
    const Real tr = s[j] * gp.x, ti = s[j] * gp.y;
    hr[j] = fma(zr[j], tr, fma(-zi[j], ti, er));
    hi[j] = fma(zr[j], ti, fma(zi[j], tr, ei));
  }
#pragma unroll 2
  for (int m = p - 1; m >= 1; --m) {
    const C2 a = cf[m - 1], bq = cf[Pq + m], g = cf[2 * Pq + m - 1];
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const Real t1r = fma(zr[j], h1r[j], fma(zi[j], h1i[j], a.x));
      const Real t1i = fma(zr[j], h1i[j], fma(-zi[j], h1r[j], a.y));
      const Real er = fma(s[j], g.x, bq.x), ei = fma(s[j], g.y, bq.y);
      const Real tr = fma(zr[j], hr[j], fma(-zi[j], hi[j], er));
      const Real ti = fma(zr[j], hi[j], fma(zi[j], hr[j], ei));
      h1r[j] = t1r;
      h1i[j] = t1i;
      hr[j] = tr;
      hi[j] = ti;
    }
  }
  const C2 g0 = cf[2 * Pq], b1 = cf[Pq], dl = cf[3 * Pq + 1];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    // the constant coefficient B_1/2 - conj(B_1)/2, then one more factor conj(zeta)
    const Real er = fma(Real(-0.5), dl.x, b1.x), ei = fma(Real(-0.5), dl.y, b1.y);
    const Real tr = fma(zr[j], hr[j], fma(-zi[j], hi[j], er));
    const Real ti = fma(zr[j], hi[j], fma(zi[j], hr[j], ei));
    const Real p2r = fma(zr[j], tr, -zi[j] * ti);
    const Real p2i = fma(zr[j], ti, zi[j] * tr);
    const Real p1r = fma(zr[j], h1r[j], zi[j] * h1i[j]);   // P1 = zeta h1
    const Real p1i = fma(zr[j], h1i[j], -zi[j] * h1r[j]);
    // -S0 ln|Z| + S0 / 2
    Real lZ;
    if constexpr (sizeof(Real) == 4)
      lZ = fmaf(-0.34657359027997264f, __builtin_amdgcn_logf(R2[j]), 0.5f);
    else
      lZ = fma(-0.5, ln_f64(R2[j]), 0.5);
    const Real fx = fma(g0.x, lZ, p1r + p2r);   // S0 = conj(g0)
    const Real fy = fma(-g0.y, lZ, p1i + p2i);
    if (!skip[j]) {
      ax[j] += (double)fx;
      ay[j] += (double)fy;
    }
  }
}

__device__ __forceinline__ double bits_to_double(float2 v) {
  return __longlong_as_double((long long)(((unsigned long long)__float_as_uint(v.y) << 32) | __float_as_uint(v.x)));
}

// One wave per 64 T targets.  The records a wave reads (a cell's for each translation, a disk's
// ring record for each near disk) are staged in LDS, two buffers deep: the global loads of the
// next record are in flight while the current one is used.
template <bool MIXED, int T>
__device__ __forceinline__ void ksum_fmm_body(
    const int* __restrict__ wstart, const int* __restrict__ tperm, const int* __restrict__ tgt_body,
    const int* __restrict__ slot_of, const double* __restrict__ X, const int* __restrict__ src_off,
    const double4* __restrict__ src64,
    const int* __restrict__ m2l_off, const int* __restrict__ m2l, const int* __restrict__ near_off,
    const int* __restrict__ near, const double* __restrict__ wcent, const double2* __restrict__ cellrec,
    const double2* __restrict__ rings, int mode, const int* __restrict__ nbr_off,
    const int* __restrict__ nbr_slot, double scale, double* __restrict__ out, unsigned long long* __restrict__ work,
    int nwave, int group) {
  constexpr int Q = MIXED ? kLoc32 : kLoc64;
  // a ring record in 16-byte units (FP32 records: two float2 per unit)
  constexpr int RU = MIXED ? kRing32Coef / 2 : kRing64Coef;
  constexpr int SU = RU > kCellRec ? RU : kCellRec;
  static_assert(SU <= 192, "three 16-byte units per lane");
  __shared__ double2 s_buf[2][SU];
  __shared__ double2 s_row[64];
  __shared__ double s_fac[2 * kFactN];   // j!, then 1/j! (the translations' binomials)
  // Workgroups go to the 8 XCDs in turn (workgroup b to XCD b mod 8).  Runs of `group`
  // consecutive waves along the curve, which read mostly the same cell and ring records, are
  // kept on one XCD (its L2), and the runs are dealt to the XCDs in turn, so that every XCD
  // gets waves from all over the domain (group 1: workgroup b runs wave b).
  const int b = blockIdx.x, i = b >> 3;
  const int w = ((i / group) * 8 + (b & 7)) * group + i % group;
  if (w >= nwave) return;
  const int lane = threadIdx.x;
  for (int e = lane; e < 2 * kFactN; e += 64) s_fac[e] = kFact[e];   // read after the fences of m2l_add
  const int p0 = wstart[w], p1 = wstart[w + 1];   // this wave's positions in the visiting order
  int t[T];
  int64_t tt[T];
  int bt[T];
  double x[T], y[T], ax[T], ay[T];
  Skip sk[T];
#pragma unroll
  for (int j = 0; j < T; ++j) {
    t[j] = p0 + lane * T + j;
    const int tc = t[j] < p1 ? t[j] : p1 - 1;
    tt[j] = tperm[tc];
    const int body = tgt_body[tt[j]];
    bt[j] = mode != 0 ? slot_of[body] : -1;
    x[j] = X[2 * tt[j]];
    y[j] = X[2 * tt[j] + 1];
    ax[j] = 0.0;
    ay[j] = 0.0;
    skip_init(sk[j], mode, body, 0, nbr_off, nbr_slot);
  }
  unsigned n_dir = 0, n_exp = 0, n_terms = 0, n_m2l = 0, n_l2p = 0;
  double2 pre[3];
  auto fetch = [&](const double2* g, int units) {
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int i = lane + 64 * u;
      pre[u] = i < units ? g[i] : make_double2(0.0, 0.0);
    }
  };
  auto stage = [&](double2* buf, int units) {
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int i = lane + 64 * u;
      if (i < units) buf[i] = pre[u];
    }
  };
  // far field: the wave's local expansion about its centre B
  const double bx = wcent[2 * w], by = wcent[2 * w + 1];
  const int m0 = m2l_off[w], m1 = m2l_off[w + 1];
  if (m1 > m0) {
    double Lr = 0.0, Li = 0.0;
    fetch(cellrec + (int64_t)m2l[m0] * kCellRec, kCellRec);
    for (int e = m0; e < m1; ++e) {
      double2* buf = s_buf[e & 1];
      stage(buf, kCellRec);   // its previous reads (two translations back) are done
      wave_lds_sync();
      if (e + 1 < m1) fetch(cellrec + (int64_t)m2l[e + 1] * kCellRec, kCellRec);
      const double2 cc = buf[kCl64CoefPerCluster];
      m2l_add<Q, Q>(buf, cc.x, cc.y, bx, by, s_row, Lr, Li, s_fac);   // source order = local order
    }
    wave_lds_sync();   // the last translation's reads of the row are done
    s_row[lane] = make_double2(Lr, Li);
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < T; ++j) {
      double ux, uy;
      l2p<Q>(s_row, x[j] - bx, y[j] - by, ux, uy);
      ax[j] += ux;
      ay[j] += uy;
    }
    n_m2l = lane == 0 ? (unsigned)(m1 - m0) : 0u;
    n_l2p = T;
  }
  // near disks, in increasing slot order (the skip cursors rely on it)
  const int n0 = near_off[w], n1 = near_off[w + 1];
  if (n1 > n0) fetch(rings + (int64_t)near[n0] * RU, RU);
  for (int e = n0; e < n1; ++e) {
    const int s = near[e];
    double2* buf = s_buf[e & 1];
    stage(buf, RU);
    wave_lds_sync();
    if (e + 1 < n1) fetch(rings + (int64_t)near[e + 1] * RU, RU);
    // header: tier distances (squared, d1 > d2 > d3), the disk's centre and body
    double d1, d2, d3, cx, cy;
    int b;
    if (MIXED) {
      const float2* o = (const float2*)buf;
      d1 = o[3 * kRing32Order + 3].x;
      d2 = o[3 * kRing32Order + 3].y;
      d3 = o[3 * kRing32Order + 2].y;
      cx = bits_to_double(o[3 * kRing32Order + 4]);
      cy = bits_to_double(o[3 * kRing32Order + 5]);
      b = (int)bits_to_double(o[3 * kRing32Order + 6]);
    } else {
      const double2* o = buf;
      d1 = o[3 * kRing64Order + 3].x;
      d2 = o[3 * kRing64Order + 3].y;
      d3 = o[3 * kRing64Order + 2].y;
      cx = o[3 * kRing64Order + 4].x;
      cy = o[3 * kRing64Order + 4].y;
      b = (int)o[3 * kRing64Order + 5].x;
    }
    double Zx[T], Zy[T], R2[T];
    bool skip[T];
    bool all_skip = true, ok1 = true, ok2 = true, ok3 = true;
#pragma unroll
    for (int j = 0; j < T; ++j) {
      Zx[j] = x[j] - cx;
      Zy[j] = y[j] - cy;
      R2[j] = fma(Zx[j], Zx[j], Zy[j] * Zy[j]);
      skip[j] = skip_test(sk[j], mode, s, bt[j], nbr_slot);
      all_skip = all_skip && skip[j];
      ok1 = ok1 && (skip[j] || R2[j] > d1);
      ok2 = ok2 && (skip[j] || R2[j] > d2);
      ok3 = ok3 && (skip[j] || R2[j] > d3);
    }
    if (__all(all_skip)) continue;
    int p = 0;
    if (__all(ok1))
      p = MIXED ? 14 : 27;
    else if (__all(ok2))
      p = MIXED ? 24 : 40;
    else if (__all(ok3))
      p = MIXED ? kRing32Order : kRing64Order;
    if (p > 0) {
      ++n_exp;
      n_terms += p;
      if (MIXED) {
        const float2* cf = (const float2*)buf;
        float fZx[T], fZy[T], fR2[T];
#pragma unroll
        for (int j = 0; j < T; ++j) {
          fZx[j] = (float)Zx[j];
          fZy[j] = (float)Zy[j];
          fR2[j] = fmaf(fZx[j], fZx[j], fZy[j] * fZy[j]);
        }
        ring_m2p_merged<float, float2, T>(cf, kRing32Order, p, cf[3 * kRing32Order + 2].x, fZx, fZy, fR2, skip, ax,
                                          ay);
      } else {
        ring_m2p<double, double2, T>(buf, kRing64Order, p, buf[3 * kRing64Order + 2].x, Zx, Zy, R2, skip, ax, ay);
      }
      continue;
    }
    // direct FP64 sum over the disk's sources
    double lx[T], ly[T], txx[T], tyy[T];
#pragma unroll
    for (int j = 0; j < T; ++j) lx[j] = ly[j] = txx[j] = tyy[j] = 0.0;
    const int q0 = src_off[b], q1 = src_off[b + 1];
    n_dir += q1 - q0;
    for (int qq = q0; qq < q1; ++qq) {
      const double4 sv = src64[qq];
#pragma unroll
      for (int j = 0; j < T; ++j) {
        const double dx = x[j] - sv.x;
        const double dy = y[j] - sv.y;
        const double r2 = fma(dx, dx, dy * dy);
        const double lg = ln_f64(r2);
        const double dot = fma(dx, sv.z, dy * sv.w) * rcp_f64(r2);
        lx[j] = fma(lg, sv.z, lx[j]);
        ly[j] = fma(lg, sv.w, ly[j]);
        txx[j] = fma(dot, dx, txx[j]);
        tyy[j] = fma(dot, dy, tyy[j]);
      }
    }
#pragma unroll
    for (int j = 0; j < T; ++j) {
      if (!skip[j]) {
        ax[j] += fma(-0.5, lx[j], txx[j]);
        ay[j] += fma(-0.5, ly[j], tyy[j]);
      }
    }
  }
  add_work(work, T * n_dir, T * n_exp, T * n_terms, n_m2l, n_l2p);
#pragma unroll
  for (int j = 0; j < T; ++j) {
    if (t[j] < p1) {
      out[tt[j] * 2] = ax[j] * scale;
      out[tt[j] * 2 + 1] = ay[j] * scale;
    }
  }
}

// The two forms as kernels, each with its register budget (waves per SIMD): 104 VGPRs and 4 waves
// for the mixed form, 138 and 3 for the FP64 form.  More waves were slower: the mixed form at 5
// (88 VGPRs, no spills) and at 6 (14 spilled), the FP64 form at 4 (14 spilled).
// MFS_KSUM_WAVES_MIXED / MFS_KSUM_WAVES_64 override the targets at build time.
#ifndef MFS_KSUM_WAVES_MIXED
#define MFS_KSUM_WAVES_MIXED 4
#endif
#ifndef MFS_KSUM_WAVES_64
#define MFS_KSUM_WAVES_64 3
#endif
#define MFS_KSUM_FMM_PARAMS                                                                                     \
  const int *__restrict__ wstart, const int *__restrict__ tperm, const int *__restrict__ tgt_body,             \
      const int *__restrict__ slot_of, const double *__restrict__ X, const int *__restrict__ src_off,          \
      const double4 *__restrict__ src64, const int *__restrict__ m2l_off, const int *__restrict__ m2l,        \
      const int *__restrict__ near_off, const int *__restrict__ near, const double *__restrict__ wcent,       \
      const double2 *__restrict__ cellrec, const double2 *__restrict__ rings, int mode,                       \
      const int *__restrict__ nbr_off, const int *__restrict__ nbr_slot, double scale, double *__restrict__ out, \
      unsigned long long *__restrict__ work, int nwave, int group
#define MFS_KSUM_FMM_ARGS                                                                                       \
  wstart, tperm, tgt_body, slot_of, X, src_off, src64, m2l_off, m2l, near_off, near, wcent, cellrec, rings,    \
      mode, nbr_off, nbr_slot, scale, out, work, nwave, group
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MFS_KSUM_WAVES_MIXED, 8))) void
k_ksum_fmm_mixed(MFS_KSUM_FMM_PARAMS) {
  ksum_fmm_body<true, kFmmT>(MFS_KSUM_FMM_ARGS);
}
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MFS_KSUM_WAVES_64, 8))) void
k_ksum_fmm_fp64(MFS_KSUM_FMM_PARAMS) {
  ksum_fmm_body<false, kFmmT>(MFS_KSUM_FMM_ARGS);
}
#undef MFS_KSUM_FMM_PARAMS
#undef MFS_KSUM_FMM_ARGS

// ---------------------------------------------------------------------------
// launchers

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;   // per device: the address of its copy of scratch
}  // namespace

Status scratch_for_current_device(double** ptr) {
  *ptr = nullptr;
  int dev = 0;
  MFS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return Status{MFS_ERR_DEVICE, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e)};
    }
    g_scratch_ptr[dev] = (double*)p;
  }
  *ptr = g_scratch_ptr[dev];
  return Status{};
}

void launch_zero_work(mfs_ctx* c) {
  hipLaunchKernelGGL(k_zero_work, dim3(1), dim3(64), 0, c->stream, c->d_work);
}

void launch_onebody_apply(mfs_ctx* c, int prob, const double* mu, double* lam_bar) {
  int m2max = 1, rmax = 1;
  for (int k = 0; k < c->ct[prob].n; ++k) {
    m2max = std::max(m2max, 2 * c->ct[prob].mc[k]);
    rmax = std::max(rmax, c->ct[prob].rank[k]);
  }
  // four bodies per workgroup while their staging fits 64 KB of LDS, else one
  const int ob = sizeof(double) * kObBodies * (m2max + rmax) <= 65536 ? kObBodies : 1;
  hipLaunchKernelGGL(k_onebody, dim3((c->P + ob - 1) / ob), dim3(kBodyThreads), sizeof(double) * ob * (m2max + rmax),
                     c->stream, c->P, c->d_cls, c->d_src_off, c->d_col_off, c->ct[prob], mu, lam_bar, ob,
                     m2max, rmax);
}

void launch_pair_A(mfs_ctx* c, int prob, const double* lam_bar, double* ltil) {
  const int C = (int)(c->pairs.size() / 2);
  if (C == 0) return;
  hipLaunchKernelGGL(k_pair_A, dim3(C), dim3(kPairThreads), 0, c->stream, C, c->d_pairs, c->d_src_off, c->d_xoff,
                     c->d_aoff, c->ps[prob].A, lam_bar, ltil);
}

void launch_gather_project(mfs_ctx* c, int prob, const double* lam_bar, const double* ltil, bool with_pairs,
                           bool pack32, bool pack64, const FmmRec* fr) {
  (void)pack64;
  launch_gather_project_to(c, prob, lam_bar, ltil, with_pairs, c->d_src64);
  launch_fmm_records(c, prob, c->d_src64, fr ? *fr : fmm_records(c, 0), pack32);
}

void launch_gather_project_to(mfs_ctx* c, int prob, const double* lam_bar, const double* ltil, bool with_pairs,
                              double4* src64) {
  hipLaunchKernelGGL(k_gather_project, dim3(c->P), dim3(kBodyThreads), 0, c->stream, c->P,
                     prob == MFS_MOBILITY ? 1 : 0, c->d_cls, c->d_src_off, c->ct[prob], c->d_bp_off, c->d_bp_list,
                     c->d_pairs, c->d_xoff, ltil, lam_bar, with_pairs ? 1 : 0, c->d_centers, src64);
}

bool launch_pair_A_rhs(mfs_ctx* c, int prob, int R, const double* lam_bar, int64_t lam_stride, double* ltil,
                       int64_t ltil_stride) {
  const int C = (int)(c->pairs.size() / 2);
  if (C == 0) return true;
  int64_t nmax = 0;
  for (int p = 0; p < C; ++p) nmax = std::max<int64_t>(nmax, c->xoff[p + 1] - c->xoff[p]);
  const size_t lds = sizeof(double) * (size_t)R * (size_t)nmax;
  if (lds > 64 * 1024) return false;
#define MFS_PA(RR)                                                                                                  \
  hipLaunchKernelGGL(k_pair_A_rhs<RR>, dim3(C), dim3(kPairThreads), lds, c->stream, C, c->d_pairs, c->d_src_off, \
                     c->d_xoff, c->d_aoff, c->ps[prob].A, lam_bar, lam_stride, ltil, ltil_stride)
  switch (R) {
    case 2: MFS_PA(2); break;
    case 4: MFS_PA(4); break;
    case 8: MFS_PA(8); break;
    default: return false;
  }
#undef MFS_PA
  return true;
}

// Choose the source split so that the grid holds enough workgroups to fill the chip
// (256 CUs, 32 workgroups each).  The split partials (splits x N_t x 16 bytes) then stay
// below 16384 x 512 targets x 16 bytes = 128 MiB.  MFS_KSUM_SPLITS overrides it.
static int ksum_splits(int64_t tblocks, int P) {
  const char* e = std::getenv("MFS_KSUM_SPLITS");
  if (e) return std::max(1, std::min(P, std::atoi(e)));
  int s = 1;
  while (tblocks * s < 8192 && s * 2 <= std::max(1, P / 8) && s < 64) s *= 2;
  return s;
}

static int ksum_targets_per_thread(bool mixed) {
  const char* e = std::getenv(mixed ? "MFS_KSUM_T" : "MFS_KSUM_T64");
  const int t = e ? std::atoi(e) : 2;
  return t == 1 || t == 2 || t == 4 ? t : 2;
}

static bool launch_ksum_fp64_arrays(mfs_ctx* c, int mode, const double4* src, const double2* mp64, int64_t Nt,
                                    const double* X, const int32_t* tgt_body, const int32_t* tperm, double* u,
                                    double scale, const SplitBuf* sb = nullptr);

// Split partials of one kernel sum: the caller's buffer (sb), else the context's own, grown
// on demand.  NULL when it does not fit.
static double* split_buffer(mfs_ctx* c, int64_t need, const SplitBuf* sb) {
  if (sb) return need <= sb->cap ? sb->p : nullptr;
  if (c->upart_cap < need) {
    if (c->d_upart) dev_free(c, c->d_upart);
    c->d_upart = nullptr;
    if (dev_malloc(c, &c->d_upart, need * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      c->d_upart = nullptr;
      c->upart_cap = 0;
      return nullptr;
    }
    c->upart_cap = need;
  }
  return c->d_upart;
}


// Stacked form of launch_kernel_sum: R strength vectors packed into c->d_src64m (R arrays of Ns
// records) and their records (launch_fmm_records); u: R x 2 Nt.
bool launch_kernel_sum_rhs(mfs_ctx* c, bool mixed, int mode, int R, double* u, double scale) {
  for (int r = 0; r < R; ++r)
    launch_ksum_fmm(c, mixed, mode, c->d_src64m + (int64_t)r * c->Ns, fmm_records(c, r), u + (int64_t)r * 2 * c->Nt,
                    scale);
  return true;
}

// MFS_KSUM_LOCAL=0 turns the workgroups' local expansions off (every far cluster is then
// evaluated per target from its expansion)
static bool local_expansions_on() {
  const char* e = std::getenv("MFS_KSUM_LOCAL");
  return !(e && std::atoi(e) == 0);
}

// FP64 kernel sum of a packed source array at Nt points X (mode as in k_ksum_fp64); mp64: the
// far-field coefficients of src (k_moments64), or NULL for the direct sum over every disk.
static bool launch_ksum_fp64_arrays(mfs_ctx* c, int mode, const double4* src, const double2* mp64, int64_t Nt,
                                    const double* X, const int32_t* tgt_body, const int32_t* tperm, double* u,
                                    double scale, const SplitBuf* sb) {
  if (Nt == 0) return true;
  const char* ev = std::getenv("MFS_KSUM_CLUSTERS");
  const double2* cmp64 = mp64 && !(ev && std::atoi(ev) == 0) ? mp64 + (int64_t)c->P * kMp64Coef : nullptr;
  const int T = ksum_targets_per_thread(false);
  const int64_t tblocks = (Nt + KS_THREADS * T - 1) / (KS_THREADS * T);
  const int ns = std::min(ksum_splits(tblocks, c->P), c->ncl);
  const int cps = (c->ncl + ns - 1) / ns;
  double* out = u;
  if (ns > 1 && !(out = split_buffer(c, (int64_t)ns * Nt * 2, sb))) return false;
  // the work counters count the context's own targets only (not flow-evaluation points)
  unsigned long long* work = X == c->d_X ? c->d_work : nullptr;
  dim3 grid((unsigned)tblocks, (unsigned)ns);
#define MFS_KS_FP64(TT)                                                                                      \
  hipLaunchKernelGGL(k_ksum_fp64<TT>, grid, dim3(KS_THREADS), 0, c->stream, c->ncl, c->d_cl_start,           \
                     c->d_slot_body, c->d_ssrc_off, c->d_src_off, src, Nt, tgt_body, c->d_slot_of, X, cps, mode, \
                     c->d_nbr_off, c->d_nbr_slot, scale, out, c->d_centers, mp64, c->d_ccent, c->d_crad64, cmp64,  \
                     tperm, work, local_expansions_on() ? 1 : 0)
  if (T == 4) MFS_KS_FP64(4); else if (T == 1) MFS_KS_FP64(1); else MFS_KS_FP64(2);
#undef MFS_KS_FP64
  if (ns > 1)
    hipLaunchKernelGGL(k_reduce_splits, dim3(nblocks(2 * Nt, 256)), dim3(256), 0, c->stream, 2 * Nt, ns, out, u);
  return true;
}

bool launch_kernel_sum(mfs_ctx* c, bool mixed, int mode, double* u, double scale, const FmmRec* fr) {
  const FmmRec f = fr ? *fr : fmm_records(c, 0);
  launch_ksum_fmm(c, mixed, mode, c->d_src64, f, u, scale);
  return true;
}

FmmRec fmm_records(mfs_ctx* c, int r) {
  FmmRec f;
  f.raw = c->d_cellraw + (int64_t)r * c->ncell * kCellRaw;
  f.rec = c->d_cellrec + (int64_t)r * c->ncell * kCellRec;
  f.r64 = c->d_ring64 + (int64_t)r * c->P * kRing64Coef;
  f.r32 = c->d_ring32 + (int64_t)r * c->P * kRing32Coef;
  return f;
}

// doubles of one vector's records (a float2 counts as one double)
int64_t fmm_record_doubles(const mfs_ctx* c) {
  return 2 * (int64_t)c->ncell * (kCellRaw + kCellRec) + 2 * (int64_t)c->P * kRing64Coef +
         (int64_t)c->P * kRing32Coef;
}

bool fmm_records_in(const mfs_ctx* c, const SplitBuf* sb, FmmRec* out) {
  if (!sb || sb->cap < fmm_record_doubles(c)) return false;
  double* p = sb->p;   // 256-byte aligned; every part below is a multiple of 16 bytes
  out->raw = (double2*)p;
  p += 2 * (int64_t)c->ncell * kCellRaw;
  out->rec = (double2*)p;
  p += 2 * (int64_t)c->ncell * kCellRec;
  out->r64 = (double2*)p;
  p += 2 * (int64_t)c->P * kRing64Coef;
  out->r32 = (float2*)p;
  return true;
}

// Records of the hierarchical kernel sum for a packed source array: ring records and leaf
// cells of every disk, then the internal cells by height.
void launch_fmm_records(mfs_ctx* c, int prob, const double4* src64, const FmmRec& fr, bool ring32) {
  int ncmax = 1;
  for (int k = 0; k < c->ct[prob].n; ++k) ncmax = std::max(ncmax, c->ct[prob].nc[k]);
  hipLaunchKernelGGL(k_ring_moments, dim3(c->P), dim3(64), sizeof(double2) * 2 * ncmax, c->stream, c->P, c->d_cls,
                     c->d_src_off, c->ct[prob],
                     src64, c->d_slot_of, c->d_centers, fr.r64, ring32 ? fr.r32 : (float2*)nullptr, fr.raw, fr.rec);
  for (int h = 1; h <= c->cell_height; ++h) {
    const int n = c->height_off[h + 1] - c->height_off[h];
    if (n > 0)
      hipLaunchKernelGGL(k_cell_m2m, dim3(n), dim3(64 * kM2mWaves), 0, c->stream, n, c->d_cell_by_height + c->height_off[h],
                         c->d_cell_child_off, c->d_cell_child, c->d_cell_c, fr.raw, fr.rec);
  }
}

// The hierarchical kernel sum at the context's targets (records fr of launch_fmm_records,
// direct sums from src64), written to u (2 Nt), scaled.
constexpr int kKsumXcdGroup = 64;

void launch_ksum_fmm(mfs_ctx* c, bool mixed, int mode, const double4* src64, const FmmRec& fr, double* u,
                     double scale) {
  const FmmLists& L = c->fl[mixed ? 1 : 0];
  if (c->nwave == 0) return;
  // runs of `group` consecutive waves per XCD (see ksum_fmm_body; MFS_KSUM_XCD_GROUP overrides)
  const char* ev = std::getenv("MFS_KSUM_XCD_GROUP");
  const int group = std::max(1, ev ? std::atoi(ev) : kKsumXcdGroup);
  const int64_t per = 8 * (int64_t)group;
  const unsigned nwg = (unsigned)((c->nwave + per - 1) / per * per);
#define MFS_KS_FMM(KERNEL, RINGS)                                                                                \
  hipLaunchKernelGGL(KERNEL, dim3(nwg), dim3(64), 0, c->stream, c->d_wstart, c->d_tperm, c->d_tgt_body,          \
                     c->d_slot_of, c->d_X, c->d_src_off, src64, L.d_m2l_off, L.d_m2l, L.d_near_off, L.d_near,     \
                     c->d_wcent, fr.rec, RINGS, mode, c->d_nbr_off, c->d_nbr_slot, scale, u, c->d_work, c->nwave, \
                     group)
  if (mixed) MFS_KS_FMM(k_ksum_fmm_mixed, (const double2*)fr.r32); else MFS_KS_FMM(k_ksum_fmm_fp64, (const double2*)fr.r64);
#undef MFS_KS_FMM
}

void launch_pair_field(mfs_ctx* c, int prob, const double* ltil, double* corr) {
  const int C = (int)(c->pairs.size() / 2);
  if (C == 0) return;
  hipLaunchKernelGGL(k_pair_field, dim3(C), dim3(kFieldThreads), 0, c->stream, C, prob == MFS_MOBILITY ? 1 : 0,
                     c->d_pairs, c->d_cls, c->d_src_off, c->d_col_off, c->ct[prob], c->d_centers, c->d_xoff,
                     c->d_coff, c->d_bp_off, c->d_bp_list, ltil, 1.0 / (4.0 * kPiD * c->prm.mu), corr);
}

void launch_finish(mfs_ctx* c, const double* u_sum, const double* mu, const double* corr, double* u_out,
                   bool with_pairs) {
  hipLaunchKernelGGL(k_finish, dim3(c->P), dim3(kBodyThreads), 0, c->stream, c->P, c->d_col_off, c->d_bp_off,
                     c->d_bp_list, c->d_pairs, c->d_coff, u_sum, mu, corr, with_pairs ? 1 : 0,
                     u_out);
}

void launch_rhs_mobility_sources(mfs_ctx* c, const double* given) {
  hipLaunchKernelGGL(k_rhs_sources, dim3(c->P), dim3(kBodyThreads), 0, c->stream, c->P, c->d_cls, c->d_src_off,
                     c->ct[MFS_MOBILITY], c->d_centers, given, c->d_src64, 0);
  launch_fmm_records(c, MFS_MOBILITY, c->d_src64, fmm_records(c, 0), false);
}

void launch_add_rhs_sources(mfs_ctx* c, const double* given, double4* src64) {
  hipLaunchKernelGGL(k_rhs_sources, dim3(c->P), dim3(kBodyThreads), 0, c->stream, c->P, c->d_cls, c->d_src_off,
                     c->ct[MFS_MOBILITY], c->d_centers, given, src64, 1);
}

void launch_rhs_resistance(mfs_ctx* c, const double* given, double* b) {
  hipLaunchKernelGGL(k_rhs_resistance, dim3(nblocks(c->Nt, 256)), dim3(256), 0, c->stream, c->Nt, c->d_tgt_body,
                     c->d_X, c->d_centers, given, b);
}

void launch_post(mfs_ctx* c, int prob, const double* lam_bar, double* out3) {
  const int C = (int)(c->pairs.size() / 2);
  const bool wp = C > 0 && c->ps[prob].ready;
  if (wp)
    hipLaunchKernelGGL(k_post_pairs, dim3(C), dim3(64), 0, c->stream, C, c->d_pairs, c->d_src_off, c->d_xoff,
                       c->ps[prob].E, lam_bar, c->d_epair);
  hipLaunchKernelGGL(k_post_bodies, dim3(c->P), dim3(64), 0, c->stream, c->P, prob == MFS_MOBILITY ? 1 : 0, c->d_cls,
                     c->d_src_off, c->ct[prob], c->d_bp_off, c->d_bp_list, c->d_epair, lam_bar, wp ? 1 : 0, out3);
}

int mdot_blocks(int64_t n) {
  int64_t b = (n + 4 * kDotThreads - 1) / (4 * kDotThreads);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1024));
}

void launch_mdot(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* w, double* part,
                 double* out, int nblk) {
  hipLaunchKernelGGL(k_mdot, dim3(nblk), dim3(kDotThreads), 0, s, n, k, V, ldv, w, part);
  hipLaunchKernelGGL(k_mdot_reduce, dim3(k), dim3(kDotThreads), 0, s, k, nblk, part, out);
}

void launch_maxpy(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* h, double* w) {
  hipLaunchKernelGGL(k_maxpy, dim3(nblocks(n, 256)), dim3(256), 0, s, n, k, V, ldv, h, w);
}

void launch_gemv_n(hipStream_t s, int64_t n, int k, const double* V, int64_t ldv, const double* y, double* x) {
  hipLaunchKernelGGL(k_gemv_n, dim3(nblocks(n, 256)), dim3(256), 0, s, n, k, V, ldv, y, x);
}

void launch_givens(hipStream_t s, int j, int cap, int R, const double* hdev, int64_t hstride, double* H, double* cs,
                   double* sn, double* g, double* ctl, double* rec) {
  hipLaunchKernelGGL(k_givens, dim3(R), dim3(64), 0, s, j, cap, R, hdev, hstride, H, cs, sn, g, ctl, rec);
}

void launch_scale_ctl(hipStream_t s, int64_t n, int R, const double* ctl, const double* x, double* y) {
  hipLaunchKernelGGL(k_scale_ctl, dim3(nblocks(n, 256), R), dim3(256), 0, s, n, ctl, x, y);
}

void launch_backsolve(hipStream_t s, int cap, int R, const double* H, const double* g, const double* ctl, double* y) {
  hipLaunchKernelGGL(k_backsolve, dim3(R), dim3(256), 0, s, cap, H, g, ctl, y);
}

void launch_scale_copy(hipStream_t s, int64_t n, double a, const double* x, double* y) {
  hipLaunchKernelGGL(k_scale_copy, dim3(nblocks(n, 256)), dim3(256), 0, s, n, a, x, y);
}

void launch_axpby(hipStream_t s, int64_t n, double a, const double* x, double b, double* y) {
  hipLaunchKernelGGL(k_axpby, dim3(nblocks(n, 256)), dim3(256), 0, s, n, a, x, b, y);
}


// ---------------------------------------------------------------------------
// flow evaluation launchers

bool launch_kernel_sum_points(mfs_ctx* c, const double4* src, const double2* mp64, int64_t n_pts,
                              const double* pts, const int32_t* body, double* u) {
  return launch_ksum_fp64_arrays(c, 0, src, mp64, n_pts, pts, body, nullptr, u, 1.0 / (4.0 * kPiD * c->prm.mu));
}

void launch_moments64(mfs_ctx* c, const double4* src64, double2* mp64) {
  hipLaunchKernelGGL(k_moments64, dim3(c->P), dim3(kBodyThreads), 0, c->stream, c->P, c->d_cls, c->d_src_off,
                     c->ct[0], src64, mp64);
  hipLaunchKernelGGL(k_cluster_moments64, dim3(c->ncl), dim3(64), 0, c->stream, c->ncl, c->d_cl_start,
                     c->d_slot_body, c->d_src_off, c->d_ccent, src64, mp64 + (int64_t)c->P * kMp64Coef);
}

void launch_fine_strengths(mfs_ctx* c, int prob, const double* lam_bar, const double* ltil, double* ptil,
                           double* sigf) {
  const int C = (int)(c->pairs.size() / 2);
  if (C == 0) return;
  const PairSet& ps = c->ps[prob];
  hipLaunchKernelGGL(k_fine_strengths, dim3(C), dim3(kPairThreads), 0, c->stream, C, prob == MFS_MOBILITY ? 1 : 0,
                     c->d_pairs, c->d_cls, c->d_src_off, c->ct[prob], c->d_centers, c->d_xoff, lam_bar, ltil, ps.G,
                     ps.d_goff, ps.Yf, ps.d_yoff, ps.nf, ps.KKf, ptil, sigf);
}

void launch_flow_near(mfs_ctx* c, int prob, int64_t n_pts, const double* pts, const int32_t* body,
                      const double* ptil, const double* sigf, double* u) {
  const int C = (int)(c->pairs.size() / 2);
  if (C == 0 || n_pts == 0) return;
  const PairSet& ps = c->ps[prob];
  hipLaunchKernelGGL(k_flow_near, dim3(nblocks(n_pts, 256)), dim3(256), 0, c->stream, n_pts, pts, body, C,
                     c->d_pairs, c->d_src_off, c->d_Y, c->d_xoff, ptil, ps.Yf, ps.d_yoff, ps.nf, sigf, ps.pgeo,
                     c->d_bp_off, c->d_bp_list, 1.0 / (4.0 * kPiD * c->prm.mu), u);
}

void launch_boundary_nodes(mfs_ctx* c, int n_per_body, double* pts, int32_t* body) {
  const int64_t n = (int64_t)c->P * n_per_body;
  hipLaunchKernelGGL(k_boundary_nodes, dim3(nblocks(n, 256)), dim3(256), 0, c->stream, c->P, n_per_body, c->d_cls,
                     c->ct[0], c->d_centers, pts, body);
}

void launch_boundary_residual(mfs_ctx* c, int64_t n_pts, const double* pts, const int32_t* body, const double* u,
                              const double* rigid, double* eps, double* maxima) {
  const unsigned nb = nblocks(n_pts, 256);
  hipLaunchKernelGGL(k_boundary_residual, dim3(nb), dim3(256), 0, c->stream, n_pts, pts, body, c->d_centers, u,
                     rigid, eps, maxima + 2);
  hipLaunchKernelGGL(k_max_pairs, dim3(1), dim3(256), 0, c->stream, (int)nb, maxima + 2, maxima);
}

}  // namespace mfs
