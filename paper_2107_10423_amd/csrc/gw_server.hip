// Request server (include/gw.h, "serving"): first-come-first-served
// admission by device-memory footprint, one HIP stream per pipeline slot,
// each admitted request run through exactly the gw_setup / gw_qp path with
// its context capped at its reserved footprint.  Inputs are validated and
// copied into pinned host memory (a reused pool) on the submitting thread, so
// a slot's upload is one DMA that overlaps the other slots' kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/gw.h"

size_t footprint_bytes(int n_mo, int n_occ, int n_aux, int n_rows, int n_states, int G,
                       int pi_prec, int wc_prec, size_t work_budget, int minres_batch);
int validate_inputs(int n_mo, int n_occ, int n_aux, const double* eps, const double* B_ov,
                    int n_rows, const int* row_ids, const double* B_rows, bool check_arrays);
long copy_check_finite(double* dst, const double* src, long n);
int setup_validated(gw_ctx** out, int n_mo, int n_occ, int n_aux, const double* eps,
                    const double* B_ov, int n_rows, const int* row_ids, const double* B_rows,
                    const gw_opts* opts);

namespace {

using clk = std::chrono::steady_clock;

// Pinned host buffers, kept for reuse in power-of-two size classes (from 64
// MiB) up to a total cap; a request that finds no pinned buffer within the cap
// keeps pageable memory.
struct PinnedPool {
  std::mutex mu;
  std::multimap<size_t, void*> free_bufs;
  size_t total = 0, cap = 0;
  static size_t size_class(size_t b) {
    size_t s = 64ull << 20;
    while (s < b) s <<= 1;
    return s;
  }
  void* acquire(size_t bytes, size_t* got) {
    const size_t want = size_class(bytes);
    std::lock_guard<std::mutex> lk(mu);
    auto it = free_bufs.lower_bound(want);
    if (it != free_bufs.end() && it->first <= 2 * want) {
      void* p = it->second;
      *got = it->first;
      free_bufs.erase(it);
      return p;
    }
    while (total + want > cap && !free_bufs.empty()) {  // make room: drop the largest free buffer
      auto last = std::prev(free_bufs.end());
      hipHostFree(last->second);
      total -= last->first;
      free_bufs.erase(last);
    }
    if (total + want > cap) return nullptr;
    void* p = nullptr;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) return nullptr;
    total += want;
    *got = want;
    return p;
  }
  void release(void* p, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu);
    free_bufs.emplace(bytes, p);
  }
  ~PinnedPool() {
    for (auto& kv : free_bufs) hipHostFree(kv.second);
  }
};

struct Req {
  unsigned long long ticket = 0;
  int n_mo = 0, n_occ = 0, n_aux = 0, n_rows = 0;
  std::vector<double> eps, dsig_x;
  // B_ov [n_aux][n_occ n_virt] then B_rows [n_rows][n_mo][n_aux]: pinned pool
  // memory (pinned_bytes > 0) or the pageable fallback
  double* B = nullptr;
  size_t pinned_bytes = 0;
  std::vector<double> B_pageable;
  std::vector<int> row_ids, states;
  size_t footprint = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int slot = -1;
  int rc = 0;
  std::vector<double> E, S, Z;
  std::vector<int> status;
  bool done = false;
};

}  // namespace

struct gw_server {
  gw_server_opts opts{};
  PinnedPool pinned;
  std::vector<double> xi, w;
  size_t budget = 0, reserved = 0, peak_reserved = 0;
  int active = 0, peak_active = 0;
  unsigned long long next_ticket = 1, submitted = 0, completed = 0, failed = 0;
  std::deque<Req*> pending;
  std::map<unsigned long long, Req*> all;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  clk::time_point t0 = clk::now();
  int device = 0;

  double now() const { return std::chrono::duration<double>(clk::now() - t0).count(); }

  void run_slot(int slot) {
    hipSetDevice(device);
    for (;;) {
      Req* r = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          return stop || (!pending.empty() && reserved + pending.front()->footprint <= budget);
        });
        if (stop && pending.empty()) return;
        if (pending.empty() || reserved + pending.front()->footprint > budget) continue;
        r = pending.front();
        pending.pop_front();
        reserved += r->footprint;
        peak_reserved = std::max(peak_reserved, reserved);
        active++;
        peak_active = std::max(peak_active, active);
        r->t_admit = now();
        r->slot = slot;
      }
      process(r, slot);
      {
        std::lock_guard<std::mutex> lk(mu);
        reserved -= r->footprint;
        active--;
        r->t_done = now();
        r->done = true;
        completed++;
        if (r->rc) failed++;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }

  void process(Req* r, int slot) {
    gw_opts o{};
    o.pi_prec = opts.pi_prec;
    o.wc_prec = opts.wc_prec;
    o.minres_max_iter = opts.minres_max_iter;
    o.minres_rtol = opts.minres_rtol;
    o.qp_tol = opts.qp_tol;
    o.qp_max_iter = opts.qp_max_iter;
    o.dsig_x = r->dsig_x.empty() ? nullptr : r->dsig_x.data();
    o.stream = streams[slot];
    o.mem_budget_bytes = r->footprint;
    o.work_budget_bytes = opts.work_budget_bytes;
    gw_ctx* c = nullptr;
    const size_t nov = (size_t)r->n_occ * (r->n_mo - r->n_occ);
    int rc = setup_validated(&c, r->n_mo, r->n_occ, r->n_aux, r->eps.data(), r->B, r->n_rows,
                             r->row_ids.data(), r->B + nov * r->n_aux, &o);
    // the device holds its copies now (setup synchronises its stream)
    if (r->pinned_bytes) pinned.release(r->B, r->pinned_bytes);
    r->B = nullptr;
    r->pinned_bytes = 0;
    std::vector<double>().swap(r->B_pageable);
    const int n = (int)r->states.size();
    r->E.assign(n, 0.0);
    r->S.assign(n, 0.0);
    r->Z.assign(n, 0.0);
    r->status.assign(n, 0);
    if (rc == 0) {
      gw_grid g{(int)xi.size(), xi.data(), w.data()};
      rc = gw_qp(c, n, r->states.data(), &g, r->E.data(), r->S.data(), r->Z.data(),
                 r->status.data());
    }
    gw_free(c);
    r->rc = rc;
  }
};

extern "C" {

int gw_server_create(gw_server** out, const gw_server_opts* opts) {
  if (!out || !opts || opts->grid_n < 1 || !opts->grid_xi || !opts->grid_w) return GW_EINVAL;
  if (opts->pi_prec < 0 || opts->pi_prec > 2 ||
      (opts->wc_prec != GW_PI_FP64 && opts->wc_prec != GW_PI_BF16X3))
    return GW_EINVAL;
  *out = nullptr;
  gw_server* s = new gw_server();
  s->opts = *opts;
  s->xi.assign(opts->grid_xi, opts->grid_xi + opts->grid_n);
  s->w.assign(opts->grid_w, opts->grid_w + opts->grid_n);
  s->opts.grid_xi = nullptr;
  s->opts.grid_w = nullptr;
  if (s->opts.work_budget_bytes == 0) s->opts.work_budget_bytes = 2ull << 30;
  int ns = opts->n_streams > 0 ? opts->n_streams : 2;
  if (ns > 4) ns = 4;
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return GW_EDEVICE;
  }
  size_t free_b = 0, total_b = 0;
  if (opts->mem_budget_bytes) {
    s->budget = opts->mem_budget_bytes;
  } else {
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete s;
      return GW_EDEVICE;
    }
    s->budget = free_b / 10 * 8;
  }
  s->pinned.cap = 64ull << 30;
  for (int i = 0; i < ns; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) hipStreamDestroy(x);
      delete s;
      return GW_EDEVICE;
    }
    s->streams.push_back(st);
  }
  for (int i = 0; i < ns; ++i) s->workers.emplace_back([s, i] { s->run_slot(i); });
  *out = s;
  return 0;
}

int gw_server_submit(gw_server* s, const gw_request* q, unsigned long long* ticket) {
  if (!s || !q || !ticket) return GW_EINVAL;
  if (q->n_mo < 2 || q->n_occ < 1 || q->n_occ >= q->n_mo || q->n_aux < 1 || q->n_rows < 1 ||
      q->n_states < 1 || !q->eps || !q->B_ov || !q->row_ids || !q->B_rows || !q->states)
    return GW_EINVAL;
  if (int rc = validate_inputs(q->n_mo, q->n_occ, q->n_aux, q->eps, q->B_ov, q->n_rows,
                               q->row_ids, q->B_rows, false))
    return rc;
  Req* r = new Req();
  r->n_mo = q->n_mo;
  r->n_occ = q->n_occ;
  r->n_aux = q->n_aux;
  r->n_rows = q->n_rows;
  const size_t nov = (size_t)q->n_occ * (q->n_mo - q->n_occ);
  const size_t n_bov = nov * q->n_aux, n_brows = (size_t)q->n_rows * q->n_mo * q->n_aux;
  r->eps.assign(q->eps, q->eps + q->n_mo);
  r->B = (double*)s->pinned.acquire((n_bov + n_brows) * sizeof(double), &r->pinned_bytes);
  if (!r->B) {
    r->pinned_bytes = 0;
    r->B_pageable.resize(n_bov + n_brows);
    r->B = r->B_pageable.data();
  }
  // copy and check finiteness in one pass
  const long bad_ov = copy_check_finite(r->B, q->B_ov, (long)n_bov);
  const long bad_rows = bad_ov >= 0 ? -1 : copy_check_finite(r->B + n_bov, q->B_rows, (long)n_brows);
  if (bad_ov >= 0 || bad_rows >= 0) {
    if (r->pinned_bytes) s->pinned.release(r->B, r->pinned_bytes);
    delete r;
    return GW_EINVAL;
  }
  r->row_ids.assign(q->row_ids, q->row_ids + q->n_rows);
  r->states.assign(q->states, q->states + q->n_states);
  if (q->dsig_x) r->dsig_x.assign(q->dsig_x, q->dsig_x + q->n_mo);
  gw_opts o{};
  o.pi_prec = s->opts.pi_prec;
  o.work_budget_bytes = s->opts.work_budget_bytes;
  r->footprint = footprint_bytes(q->n_mo, q->n_occ, q->n_aux, q->n_rows, q->n_states,
                                 (int)s->xi.size(), s->opts.pi_prec, s->opts.wc_prec,
                                 s->opts.work_budget_bytes, 256);
  if (r->footprint > s->budget) {
    if (r->pinned_bytes) s->pinned.release(r->B, r->pinned_bytes);
    delete r;
    return GW_ENOMEM;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = s->now();
    s->pending.push_back(r);
    s->all[r->ticket] = r;
    s->submitted++;
    *ticket = r->ticket;
  }
  s->cv_work.notify_all();
  return 0;
}

int gw_server_poll(gw_server* s, unsigned long long ticket, double* E_qp, double* sigma_c,
                   double* Z, int* status, gw_request_info* info) {
  if (!s) return GW_EINVAL;
  Req* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return GW_EINVAL;
    r = it->second;
    if (!r->done) return 1;
    s->all.erase(it);
  }
  const size_t n = r->states.size();
  if (E_qp) std::copy(r->E.begin(), r->E.end(), E_qp);
  if (sigma_c) std::copy(r->S.begin(), r->S.end(), sigma_c);
  if (Z) std::copy(r->Z.begin(), r->Z.end(), Z);
  if (status) std::copy(r->status.begin(), r->status.end(), status);
  if (info) {
    info->rc = r->rc;
    info->footprint_bytes = r->footprint;
    info->t_submit = r->t_submit;
    info->t_admit = r->t_admit;
    info->t_done = r->t_done;
    info->slot = r->slot;
  }
  (void)n;
  delete r;
  return 0;
}

int gw_server_drain(gw_server* s) {
  if (!s) return GW_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending.empty() && s->active == 0; });
  return 0;
}

int gw_server_get_stats(gw_server* s, gw_server_stats* out) {
  if (!s || !out) return GW_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->budget_bytes = s->budget;
  out->reserved_bytes = s->reserved;
  out->peak_reserved_bytes = s->peak_reserved;
  out->active = s->active;
  out->peak_active = s->peak_active;
  return 0;
}

double gw_server_clock(gw_server* s) { return s ? s->now() : 0.0; }

void gw_server_destroy(gw_server* s) {
  if (!s) return;
  gw_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers) t.join();
  for (hipStream_t st : s->streams) hipStreamDestroy(st);
  for (auto& kv : s->all) delete kv.second;
  delete s;
}

}  // extern "C"
