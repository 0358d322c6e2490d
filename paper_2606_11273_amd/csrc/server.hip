// Serving layer: continuous batching of independent suspension solves on one device.
//
// Each slot is a HIP stream (default priority) driven by one host worker thread.
// Requests wait in a FIFO; whenever a slot is idle it admits the oldest queued
// request whose device-memory footprint fits in what the budget has left, so
// requests arriving while others run are admitted as slots and memory free up.
// An admitted request runs the whole method on its slot's stream: setup, the pair
// precompute (Alg. 2 precompute loop) and the solve (Alg. 2 with the matvec of
// Alg. 3), with its context, pair matrices and Krylov basis resident until it
// completes.  Work of different slots overlaps on the device through the separate
// streams.  A request's arithmetic depends only on its own inputs (the precompute
// batch size is fixed per request, not taken from the memory free at the time), so
// its result is the same alone and in a mix.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "geometry.h"
#include "internal.h"

namespace {

using clk = std::chrono::steady_clock;

// pairs per precompute batch in the server: fixed, so that the batching (and with it
// every library call's shapes) depends on the request alone
constexpr int kServerPrecomputeBatch = 256;

struct Request {
  int64_t ticket = 0;
  int P = 0;
  std::vector<double> centers, radii, r_src, given;
  std::vector<int32_t> n_src, n_col;
  mfs_problem problem = MFS_MOBILITY;
  mfs_precision precision = MFS_MIXED;
  double tol = 1e-8;
  int max_iter = 300;
  int64_t footprint = 0;
  // results
  bool done = false;
  mfs_status status = MFS_OK;
  std::string err;
  std::vector<double> out;
  mfs_ticket_info info{};
  clk::time_point t_submit, t_admit, t_done;
};

double ms_between(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct mfs_server {
  mfs_params prm{};
  int device = 0;
  int64_t budget = 0, in_use = 0;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<int64_t, std::shared_ptr<Request>> tickets;
  int64_t next_ticket = 1;
  bool stop = false;
  std::string last_err;
};

namespace {

mfs_status srv_fail(mfs_server* s, mfs_status code, const std::string& msg) {
  s->last_err = msg;
  return code;
}

// Validate a request's host inputs and count its close pairs.
mfs_status check_request(const mfs_server* s, const mfs_request* r, int64_t* n_pairs, std::string* err) {
  if (!r || r->P < 1 || !r->centers || !r->radii || !r->n_src || !r->n_col || !r->r_src || !r->given) {
    *err = "request: null input or P < 1";
    return MFS_ERR_ARG;
  }
  if ((r->problem != MFS_RESISTANCE && r->problem != MFS_MOBILITY) ||
      (r->precision != MFS_FP64 && r->precision != MFS_MIXED) || !(r->tol > 0.0) || r->max_iter < 1 ||
      r->max_iter > 1000) {
    *err = "request: invalid problem, precision, tol or max_iter";
    return MFS_ERR_ARG;
  }
  for (int i = 0; i < r->P; ++i)
    if (r->n_src[i] < 1 || r->n_col[i] <= r->n_src[i] || r->n_col[i] > mfs::kMaxCol || !(r->radii[i] > 0.0)) {
      *err = "request: body " + std::to_string(i) + " has invalid sizes or radius";
      return MFS_ERR_ARG;
    }
  std::vector<int32_t> pairs;
  int bi = -1, bk = -1;
  double bg = 0;
  if (!mfs::find_contacts(r->P, r->centers, r->radii, s->prm.delta_c, pairs, &bi, &bk, &bg)) {
    *err = "request: disks " + std::to_string(bi) + " and " + std::to_string(bk) + " overlap or touch";
    return MFS_ERR_GEOMETRY;
  }
  *n_pairs = (int64_t)(pairs.size() / 2);
  return MFS_OK;
}

// Upper bound of the device memory one request allocates (bytes).
int64_t footprint_of(const mfs_server* s, const mfs_request* r, int64_t C) {
  int64_t Ns = 0, Nt = 0, ncmax = 0;
  for (int i = 0; i < r->P; ++i) {
    Ns += r->n_src[i];
    Nt += r->n_col[i];
    ncmax = std::max<int64_t>(ncmax, r->n_src[i]);
  }
  const int64_t nvec = 2 * Nt;
  const int64_t m4 = 4 * ncmax;
  // context: points, strengths (FP64 and packed FP32), offsets, per-body buffers
  int64_t b = 256 * (Ns + Nt) + 64 * (int64_t)r->P;
  // split partials of the kernel sum (at most 64 source splits)
  b += 64 * Nt * 16;
  // pair matrices A and E, the pair strengths and corrections of one problem
  b += C * (m4 * m4 + 6 * m4 + 4 * m4) * 8;
  // precompute work space of one batch: per pair the fine matrix F (m x n), its SVD
  // factors, X, D, C and the products (m = 4 M_f rows, n <= 4 (n_fp + 2 n_ell) columns,
  // nx = 4 N_c, mpp = 2 M_p), plus half again for rocSOLVER's own work space
  const int64_t m = 4 * ((int64_t)std::ceil(s->prm.a_f * s->prm.n_fp) + (int64_t)s->prm.a_ell * s->prm.n_ell);
  const int64_t n = 4 * ((int64_t)s->prm.n_fp + 2 * (int64_t)s->prm.n_ell);
  const int64_t nx = m4, mpp = 2 * (int64_t)s->prm.m_p;
  const int64_t per_pair =
      12 * (2 * m * n + n * n + m * nx + mpp * n + 2 * n * nx + 3 * mpp * nx + 2 * nx * nx);
  b += std::min<int64_t>(C, kServerPrecomputeBatch) * per_pair;
  // Krylov basis and work vectors of the solve, the dot-product partials
  b += ((int64_t)r->max_iter + 8) * nvec * 8 + 1024 * ((int64_t)r->max_iter + 2) * 8;
  // rocBLAS / rocSOLVER work space
  b += (int64_t)64 << 20;
  return b;
}

void run_request(mfs_server* s, hipStream_t stream, Request& q) {
  mfs_ctx* ctx = nullptr;
  mfs_status st = mfs_setup(&ctx, q.P, q.centers.data(), q.radii.data(), q.n_src.data(), q.n_col.data(),
                            q.r_src.data(), &s->prm, stream);
  if (st != MFS_OK) {
    q.status = st;
    q.err = mfs_last_error(nullptr);
    return;
  }
  ctx->pre_batch = kServerPrecomputeBatch;
  auto t0 = clk::now();
  st = mfs_precompute_pairs(ctx, q.problem, nullptr);
  q.info.ms_precompute = ms_between(t0, clk::now());
  if (st == MFS_OK) {
    q.out.assign(3 * (size_t)q.P, 0.0);
    mfs_solve_info si{};
    st = mfs_gmres_solve(ctx, q.problem, q.precision, 1, q.given.data(), q.out.data(), nullptr, q.tol, q.max_iter,
                         &si);
    si.resid_hist = nullptr;
    si.hist_cap = si.hist_len = 0;
    q.info.solve = si;
  }
  if (st != MFS_OK) q.err = mfs_last_error(ctx);
  q.status = st;
  mfs_destroy(ctx);
}

void worker_loop(mfs_server* s, int slot) {
  (void)hipSetDevice(s->device);
  hipStream_t stream = s->streams[slot];
  for (;;) {
    std::shared_ptr<Request> q;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->stop) return;
        // oldest request that fits in what the budget has left
        for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
          if ((*it)->footprint <= s->budget - s->in_use) {
            q = *it;
            s->queue.erase(it);
            break;
          }
        if (q) break;
        s->cv_work.wait(lk);
      }
      s->in_use += q->footprint;
      q->t_admit = clk::now();
    }
    run_request(s, stream, *q);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->in_use -= q->footprint;
      q->t_done = clk::now();
      q->info.ms_queue = ms_between(q->t_submit, q->t_admit);
      q->info.ms_service = ms_between(q->t_admit, q->t_done);
      q->info.ms_total = ms_between(q->t_submit, q->t_done);
      q->info.footprint_bytes = q->footprint;
      q->done = true;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

mfs_status mfs_server_create(mfs_server** srv, size_t hbm_budget_bytes, int32_t max_slots, const mfs_params* prm) {
  if (!srv) return MFS_ERR_ARG;
  *srv = nullptr;
  if (max_slots < 1 || max_slots > 64) return MFS_ERR_ARG;
  auto* s = new mfs_server();
  if (prm)
    s->prm = *prm;
  else
    mfs_default_params(&s->prm);
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return MFS_ERR_DEVICE;
  }
  if (hbm_budget_bytes == 0) {
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete s;
      return MFS_ERR_DEVICE;
    }
    hbm_budget_bytes = (size_t)(0.8 * (double)free_b);
  }
  s->budget = (int64_t)hbm_budget_bytes;
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return MFS_ERR_DEVICE;
    }
    s->streams.push_back(st);
  }
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back(worker_loop, s, i);
  *srv = s;
  return MFS_OK;
}

mfs_status mfs_server_footprint(const mfs_server* srv, const mfs_request* req, int64_t* bytes) {
  if (!srv || !bytes) return MFS_ERR_ARG;
  int64_t C = 0;
  std::string err;
  mfs_status st = check_request(srv, req, &C, &err);
  if (st != MFS_OK) return st;
  *bytes = footprint_of(srv, req, C);
  return MFS_OK;
}

mfs_status mfs_server_submit(mfs_server* s, const mfs_request* r, int64_t* ticket) {
  if (!s || !ticket) return MFS_ERR_ARG;
  int64_t C = 0;
  std::string err;
  mfs_status st = check_request(s, r, &C, &err);
  std::lock_guard<std::mutex> lk(s->mu);
  if (st != MFS_OK) return srv_fail(s, st, err);
  if (s->stop) return srv_fail(s, MFS_ERR_STATE, "server is shutting down");
  auto q = std::make_shared<Request>();
  q->P = r->P;
  q->centers.assign(r->centers, r->centers + 2 * (size_t)r->P);
  q->radii.assign(r->radii, r->radii + r->P);
  q->r_src.assign(r->r_src, r->r_src + r->P);
  q->n_src.assign(r->n_src, r->n_src + r->P);
  q->n_col.assign(r->n_col, r->n_col + r->P);
  q->given.assign(r->given, r->given + 3 * (size_t)r->P);
  q->problem = r->problem;
  q->precision = r->precision;
  q->tol = r->tol;
  q->max_iter = r->max_iter;
  q->footprint = footprint_of(s, r, C);
  if (q->footprint > s->budget)
    return srv_fail(s, MFS_ERR_ARG,
                    "request footprint " + std::to_string(q->footprint) + " B exceeds the budget " +
                        std::to_string(s->budget) + " B");
  q->ticket = s->next_ticket++;
  q->t_submit = clk::now();
  s->tickets[q->ticket] = q;
  s->queue.push_back(q);
  *ticket = q->ticket;
  s->cv_work.notify_one();
  return MFS_OK;
}

mfs_status mfs_server_wait(mfs_server* s, int64_t ticket, double* out, mfs_ticket_info* info, int32_t timeout_ms) {
  if (!s || !out) return MFS_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return srv_fail(s, MFS_ERR_ARG, "unknown ticket " + std::to_string(ticket));
  std::shared_ptr<Request> q = it->second;
  auto ready = [&] { return q->done; };
  if (timeout_ms < 0)
    s->cv_done.wait(lk, ready);
  else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
    return srv_fail(s, MFS_ERR_STATE, "ticket " + std::to_string(ticket) + " not done within the timeout");
  s->tickets.erase(ticket);
  if (q->status == MFS_OK || q->status == MFS_ERR_NOCONV) std::memcpy(out, q->out.data(), sizeof(double) * q->out.size());
  if (info) *info = q->info;
  if (q->status != MFS_OK) s->last_err = "ticket " + std::to_string(ticket) + ": " + q->err;
  return q->status;
}

const char* mfs_server_last_error(const mfs_server* s) { return s ? s->last_err.c_str() : "null server"; }

mfs_status mfs_server_destroy(mfs_server* s) {
  if (!s) return MFS_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  delete s;
  return MFS_OK;
}

}  // extern "C"
