// Host side of the hierarchical kernel sum (Alg. 3 step 2a, eq. getall): the cell tree over
// the disks and the per-wave interaction lists, built once per geometry at setup.
//
// The disks are in slot order (a Morton curve over their centres, build_clusters).  The tree
// is the quadtree of the curve's codes with single-disk leaves: cell s < P is the disk in slot
// s; an internal cell holds the slots of one code prefix, children in curve order, levels
// whose prefix splits nothing skipped.  A cell's centre C is the mean of its disks' centres
// and its radius R = max_b (|c_b - C| + a_b) over its disks, a_b the disk radius: the fields of
// a disk's strengths decay like (a_b / distance)^k in the order k (the ring rule makes the
// top modes of the one-body strengths large, and they stand for boundary data on radius a_b),
// so a_b, not the ring radius, bounds the truncation of a cell's expansion.
//
// A wave of the kernel sum holds up to kFmmT x 64 consecutive targets of the visiting order
// (tperm), a run cut where the curve jumps; its centre B is the midpoint of their bounding
// box and r its largest distance from B.  A cell goes into the wave's M2L list when |C - B| >= sep (R + r) and it holds no
// target's own disk and no contact partner of one (those must stay separable, for the skip
// modes); otherwise a leaf goes into the wave's near list and an internal cell is opened.
// With sep = 4 (FP64 sum, orders 26) the translation truncates below 4^-27 of the sources'
// strength sums, with sep = 3 (mixed sum, local order 20) below 3^-21.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

#include "internal.h"

namespace mfs {

namespace {

uint64_t spread16(uint32_t v) {   // bit k of v -> bit 2k
  uint64_t x = v & 0xffffu;
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

template <class T>
Status upload_vec(mfs_ctx* c, T** dst, const std::vector<T>& h) {
  if (*dst) dev_free(c, *dst);
  *dst = nullptr;
  MFS_HIP(dev_malloc(c, dst, sizeof(T) * std::max<size_t>(1, h.size())));
  if (!h.empty()) MFS_HIP(hipMemcpyAsync(*dst, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, c->stream));
  return Status{};
}

}  // namespace

Status build_fmm(mfs_ctx* c) {
  const int P = c->P;
  // Morton codes per slot (the curve of build_clusters)
  double x0 = c->centers[0], x1 = x0, y0 = c->centers[1], y1 = y0;
  for (int i = 1; i < P; ++i) {
    x0 = std::min(x0, c->centers[2 * i]);
    x1 = std::max(x1, c->centers[2 * i]);
    y0 = std::min(y0, c->centers[2 * i + 1]);
    y1 = std::max(y1, c->centers[2 * i + 1]);
  }
  const double span = std::max(std::max(x1 - x0, y1 - y0), 1e-300);
  std::vector<uint64_t> code(P);
  for (int s = 0; s < P; ++s) {
    const int b = c->slot_body[s];
    const uint32_t qx = (uint32_t)std::min(65535.0, std::floor((c->centers[2 * b] - x0) / span * 65535.0));
    const uint32_t qy = (uint32_t)std::min(65535.0, std::floor((c->centers[2 * b + 1] - y0) / span * 65535.0));
    code[s] = spread16(qx) | (spread16(qy) << 1);
  }
  // cells: leaves first, internal cells in post-order (children before parents)
  std::vector<int32_t> lo(P), hi(P);
  std::vector<std::vector<int32_t>> kids(P);
  for (int s = 0; s < P; ++s) {
    lo[s] = s;
    hi[s] = s + 1;
  }
  std::vector<int32_t> height(P, 0);
  // recursive build (depth <= 17)
  std::function<int(int, int, int)> build = [&](int l, int h, int depth) -> int {
    if (h - l == 1) return l;
    std::vector<std::pair<int, int>> parts;
    while (depth < 16) {
      parts.clear();
      const int shift = 2 * (15 - depth);
      int a = l;
      while (a < h) {
        const uint64_t key = code[a] >> shift;
        int e = a + 1;
        while (e < h && (code[e] >> shift) == key) ++e;
        parts.push_back({a, e});
        a = e;
      }
      if (parts.size() > 1) break;
      ++depth;
    }
    std::vector<int32_t> ch;
    if (depth >= 16) {   // equal codes: every disk its own child
      for (int s = l; s < h; ++s) ch.push_back(s);
    } else {
      for (auto& pr : parts) ch.push_back(build(pr.first, pr.second, depth + 1));
    }
    const int id = (int)lo.size();
    lo.push_back(l);
    hi.push_back(h);
    kids.push_back(ch);
    int hmax = 0;
    for (int q : ch) hmax = std::max(hmax, height[q]);
    height.push_back(hmax + 1);
    return id;
  };
  const int root = build(0, P, 0);
  const int ncell = (int)lo.size();
  c->ncell = ncell;
  c->cell_lo = lo;
  c->cell_hi = hi;
  c->cell_c.assign(2 * (size_t)ncell, 0.0);
  c->cell_r.assign(ncell, 0.0);
  for (int q = 0; q < ncell; ++q) {
    double sx = 0.0, sy = 0.0;
    for (int s = lo[q]; s < hi[q]; ++s) {
      const int b = c->slot_body[s];
      sx += c->centers[2 * b];
      sy += c->centers[2 * b + 1];
    }
    const double cx = sx / (hi[q] - lo[q]), cy = sy / (hi[q] - lo[q]);
    double r = 0.0;
    for (int s = lo[q]; s < hi[q]; ++s) {
      const int b = c->slot_body[s];
      r = std::max(r, std::hypot(c->centers[2 * b] - cx, c->centers[2 * b + 1] - cy) + c->radii[b]);
    }
    c->cell_c[2 * q] = cx;
    c->cell_c[2 * q + 1] = cy;
    c->cell_r[q] = r * (1.0 + 1e-12);
  }
  c->cell_child_off.assign(ncell + 1, 0);
  c->cell_child.clear();
  for (int q = 0; q < ncell; ++q) {
    c->cell_child_off[q + 1] = c->cell_child_off[q] + (int32_t)kids[q].size();
    c->cell_child.insert(c->cell_child.end(), kids[q].begin(), kids[q].end());
  }
  // internal cells by height (the upward pass runs one height per launch)
  int hmax = 0;
  for (int q = P; q < ncell; ++q) hmax = std::max(hmax, height[q]);
  c->cell_height = hmax;
  c->height_off.assign(hmax + 2, 0);
  c->cell_by_height.clear();
  for (int hgt = 1; hgt <= hmax; ++hgt) {
    c->height_off[hgt] = (int32_t)c->cell_by_height.size();
    for (int q = P; q < ncell; ++q)
      if (height[q] == hgt) c->cell_by_height.push_back(q);
  }
  c->height_off[hmax + 1] = (int32_t)c->cell_by_height.size();

  // waves: runs of at most kFmmT x 64 consecutive targets of the visiting order (the nodes of
  // the disks in slot order), cut where the next disk's centre lies more than kWaveReach from
  // the centre of the run's first disk (the curve's jumps), so that every wave stays compact;
  // then the centre and radius of each wave's targets and the slots it must be able to skip
  const int wt = 64 * kFmmT;
  const int64_t Nt = c->Nt;
  std::vector<int32_t> tperm;
  tperm.reserve(Nt);
  std::vector<int32_t> wstart;
  {
    constexpr double kWaveReach = 3.0;
    int64_t pos = 0, wbeg = 0;
    double fx = 0.0, fy = 0.0;   // centre of the current wave's first disk
    bool open = false;
    for (int s = 0; s < P; ++s) {
      const int b = c->slot_body[s];
      const double bx = c->centers[2 * b], by = c->centers[2 * b + 1];
      const double reach = kWaveReach * std::max(1.0, c->radii[b]);
      if (open && std::hypot(bx - fx, by - fy) > reach) {
        wstart.push_back((int32_t)wbeg);
        wbeg = pos;
        open = false;
      }
      for (int q = c->col_off[b]; q < c->col_off[b + 1]; ++q) {
        if (!open) {
          fx = bx;
          fy = by;
          open = true;
        }
        tperm.push_back(q);
        ++pos;
        if (pos - wbeg == wt) {
          wstart.push_back((int32_t)wbeg);
          wbeg = pos;
          open = false;
        }
      }
    }
    if (pos > wbeg) wstart.push_back((int32_t)wbeg);
    wstart.push_back((int32_t)pos);
  }
  const int nwave = (int)wstart.size() - 1;
  c->nwave = nwave;
  std::vector<double> tx(Nt), ty(Nt);
  std::vector<int32_t> tb(Nt);
  for (int i = 0; i < P; ++i) {
    const std::vector<double>& xr = c->h_Xr[c->cls[i]];
    for (int q = 0; q < c->n_col[i]; ++q) {
      const int64_t t = c->col_off[i] + q;
      tx[t] = c->centers[2 * i] + xr[2 * q];
      ty[t] = c->centers[2 * i + 1] + xr[2 * q + 1];
      tb[t] = i;
    }
  }
  std::vector<double> wcent(2 * (size_t)nwave), wrad(nwave);
  std::vector<std::vector<int32_t>> excl(nwave);
  for (int w = 0; w < nwave; ++w) {
    const int64_t p0 = wstart[w], p1 = wstart[w + 1];
    double xl = 1e300, xh = -1e300, yl = 1e300, yh = -1e300;
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t t = tperm[p];
      xl = std::min(xl, tx[t]);
      xh = std::max(xh, tx[t]);
      yl = std::min(yl, ty[t]);
      yh = std::max(yh, ty[t]);
    }
    const double bx = 0.5 * (xl + xh), by = 0.5 * (yl + yh);
    double r = 0.0;
    std::vector<int32_t>& ex = excl[w];
    int last = -1;
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t t = tperm[p];
      r = std::max(r, std::hypot(tx[t] - bx, ty[t] - by));
      const int b = tb[t];
      if (b == last) continue;
      last = b;
      ex.push_back(c->slot_of[b]);
      for (int e = c->nbr_off[b]; e < c->nbr_off[b + 1]; ++e) ex.push_back(c->slot_of[c->nbr_list[e]]);
    }
    std::sort(ex.begin(), ex.end());
    ex.erase(std::unique(ex.begin(), ex.end()), ex.end());
    wcent[2 * w] = bx;
    wcent[2 * w + 1] = by;
    wrad[w] = r * (1.0 + 1e-12) + 1e-12;
  }

  // lists, per separation, built in parallel over waves
  const double seps[2] = {kLocSep64, kLocSep32};
  for (int f = 0; f < 2; ++f) {
    const double sep = seps[f];
    std::vector<std::vector<int32_t>> m2l(nwave), nearl(nwave);
    auto work = [&](int w0, int w1) {
      std::vector<int32_t> stack;
      for (int w = w0; w < w1; ++w) {
        const double bx = wcent[2 * w], by = wcent[2 * w + 1], rw = wrad[w];
        const std::vector<int32_t>& ex = excl[w];
        stack.assign(1, root);
        while (!stack.empty()) {
          const int q = stack.back();
          stack.pop_back();
          const double d = std::hypot(c->cell_c[2 * q] - bx, c->cell_c[2 * q + 1] - by);
          bool adm = d >= sep * (c->cell_r[q] + rw);
          if (adm) {
            // no excluded slot inside [lo, hi)
            auto it = std::lower_bound(ex.begin(), ex.end(), lo[q]);
            adm = it == ex.end() || *it >= hi[q];
          }
          if (adm) {
            m2l[w].push_back(q);
          } else if (q < P) {
            nearl[w].push_back(q);
          } else {
            const std::vector<int32_t>& ch = kids[q];
            for (int e = (int)ch.size() - 1; e >= 0; --e) stack.push_back(ch[e]);
          }
        }
      }
    };
    const int nth = std::max(1, std::min(8, (int)std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    const int per = (nwave + nth - 1) / nth;
    for (int k = 0; k < nth; ++k) {
      const int w0 = k * per, w1 = std::min(nwave, w0 + per);
      if (w0 < w1) th.emplace_back(work, w0, w1);
    }
    for (auto& t : th) t.join();
    FmmLists& L = c->fl[f];
    L.sep = sep;
    L.m2l_off.assign(nwave + 1, 0);
    L.near_off.assign(nwave + 1, 0);
    L.m2l.clear();
    L.near.clear();
    for (int w = 0; w < nwave; ++w) {
      L.m2l_off[w + 1] = L.m2l_off[w] + (int32_t)m2l[w].size();
      L.near_off[w + 1] = L.near_off[w] + (int32_t)nearl[w].size();
      L.m2l.insert(L.m2l.end(), m2l[w].begin(), m2l[w].end());
      L.near.insert(L.near.end(), nearl[w].begin(), nearl[w].end());
    }
    Status st;
    if ((st = upload_vec(c, &L.d_m2l_off, L.m2l_off)).code) return st;
    if ((st = upload_vec(c, &L.d_m2l, L.m2l)).code) return st;
    if ((st = upload_vec(c, &L.d_near_off, L.near_off)).code) return st;
    if ((st = upload_vec(c, &L.d_near, L.near)).code) return st;
  }
  Status st;
  if ((st = upload_vec(c, &c->d_cell_child_off, c->cell_child_off)).code) return st;
  if ((st = upload_vec(c, &c->d_cell_child, c->cell_child)).code) return st;
  if ((st = upload_vec(c, &c->d_cell_by_height, c->cell_by_height)).code) return st;
  if ((st = upload_vec(c, &c->d_cell_c, c->cell_c)).code) return st;
  if ((st = upload_vec(c, &c->d_wcent, wcent)).code) return st;
  if ((st = upload_vec(c, &c->d_wstart, wstart)).code) return st;
  c->h_wstart = wstart;
  c->h_wcent = wcent;
  return ensure_fmm_records(c, 1);
}

// Record buffers of the hierarchical kernel sum for R vectors
Status ensure_fmm_records(mfs_ctx* c, int R) {
  if (c->fmm_rcap >= R) return Status{};
  for (void** p : {(void**)&c->d_cellraw, (void**)&c->d_cellrec, (void**)&c->d_ring64, (void**)&c->d_ring32}) {
    if (*p) dev_free(c, *p);
    *p = nullptr;
  }
  c->fmm_rcap = 0;
  MFS_HIP(dev_malloc(c, &c->d_cellraw, sizeof(double2) * (size_t)R * c->ncell * kCellRaw));
  MFS_HIP(dev_malloc(c, &c->d_cellrec, sizeof(double2) * (size_t)R * c->ncell * kCellRec));
  MFS_HIP(dev_malloc(c, &c->d_ring64, sizeof(double2) * (size_t)R * c->P * kRing64Coef));
  MFS_HIP(dev_malloc(c, &c->d_ring32, sizeof(float2) * (size_t)R * c->P * kRing32Coef));
  c->fmm_rcap = R;
  return Status{};
}

}  // namespace mfs
