// Request server (include/gw.h, "serving"): first-come-first-served
// admission by device-memory footprint, one HIP stream per pipeline slot,
// each admitted request run through exactly the gw_setup / gw_qp path with
// its context capped at its reserved footprint.  Inputs are validated and
// copied into pinned host memory (a reused pool) on the submitting thread, so
// a slot's upload is one DMA that overlaps the other slots' kernels.
//
// Small requests are batched by padded shape: the slot that admits one takes
// every pending request of that shape along (continuous batching: whatever
// has arrived by then), runs their stage A as one grouped launch sequence
// replayed from the shape's captured graph, and queues them for their
// quasiparticle stages, which any free slot picks up before admitting new
// work.  Contexts draw their device and pinned blocks from a server-wide
// cache, so requests of recurring shapes reuse memory instead of calling
// hipMalloc / hipFree.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/gw.h"
#include "gw_internal.h"

size_t footprint_bytes(int n_mo, int n_occ, int n_aux, int n_rows, int n_states, int G,
                       int pi_prec, int wc_prec, size_t work_budget, int minres_batch);
struct gw_devcache;
struct gw_group;
int setup_cached(gw_ctx** out, int n_mo, int n_occ, int n_aux, const double* eps,
                 const double* B_ov, int n_rows, const int* row_ids, const double* B_rows,
                 const gw_opts* opts, gw_devcache* cache);
int group_create(gw_group** out, int Np, int Kp, int Rp, const gw_grid* grid, int n_max,
                 int pi_prec, int wc_prec, gw_devcache* cache, bool graphs);
void group_free(gw_group* g);
size_t group_bytes(int Np, int Kp, int Rp, int grid_n, int n, int pi_prec, int wc_prec);
int group_run(gw_group* g, gw_ctx* const* m, int n, int* rc);
void group_stats(const gw_group* g, long* batches, long* items, long* replays);
int ctx_set_stream(gw_ctx* c, hipStream_t st);
void padded_shape(int n_mo, int n_occ, int n_aux, int n_rows, int* Np, int* Kp, int* Rp);
gw_devcache* devcache_create(size_t cap);
void devcache_destroy(gw_devcache* c);
void devcache_stats(gw_devcache* c, long* mallocs, long* hits, long* frees, size_t* live,
                    size_t* cached);
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

// Requests of one padded shape batched together: the group (its workspace and
// captured graphs) is created by the first batch and kept until the server is
// destroyed; its workspace is reserved from the budget for that long.
struct ShapeGroup {
  int Np = 0, Kp = 0, Rp = 0, n_max = 1;
  size_t bytes = 0;
  bool usable = true;        // false: the workspace did not fit, requests run alone
  std::mutex mu;             // one batch at a time
  gw_group* g = nullptr;
};

struct Req {
  unsigned long long ticket = 0;
  ShapeGroup* group = nullptr;   // set when the request may be batched
  gw_ctx* ctx = nullptr;         // between a batch's stage A and the QP stage
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
  gw_devcache* cache = nullptr;
  std::map<std::array<int, 3>, ShapeGroup*> groups;
  std::deque<Req*> qp_ready;     // stage A done (batched), waiting for a pipeline
  long batches = 0, batched = 0;
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

  // caller holds mu
  void admit(Req* r, int slot) {
    reserved += r->footprint;
    peak_reserved = std::max(peak_reserved, reserved);
    active++;
    peak_active = std::max(peak_active, active);
    r->t_admit = now();
    r->slot = slot;
  }

  void complete(Req* r) {
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

  void run_slot(int slot) {
    if (!gw::audit_mode()) hipSetDevice(device);
    for (;;) {
      Req* r = nullptr;
      bool qp_stage = false;
      std::vector<Req*> batch;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] {
          return stop || !qp_ready.empty() ||
                 (!pending.empty() && reserved + pending.front()->footprint <= budget);
        });
        if (!qp_ready.empty()) {
          r = qp_ready.front();
          qp_ready.pop_front();
          qp_stage = true;
        } else if (stop && pending.empty()) {
          return;
        } else if (pending.empty() || reserved + pending.front()->footprint > budget) {
          continue;
        } else {
          r = pending.front();
          pending.pop_front();
          admit(r, slot);
          ShapeGroup* sg = r->group;
          if (sg && sg->usable) {
            // every pending request of the same shape that fits joins the batch
            batch.push_back(r);
            for (auto it = pending.begin();
                 it != pending.end() && (int)batch.size() < sg->n_max;) {
              Req* q = *it;
              if (q->group == sg && reserved + q->footprint <= budget) {
                admit(q, slot);
                batch.push_back(q);
                it = pending.erase(it);
              } else {
                ++it;
              }
            }
          }
        }
      }
      if (qp_stage) {
        qp(r, slot);
        complete(r);
      } else if (batch.size() < 2) {
        // nothing to share a launch with: the solo path, which needs no
        // group workspace and no captured graph
        process(r, slot);
        complete(r);
      } else {
        run_batch(batch, slot);
      }
    }
  }

  gw_opts ctx_opts(const Req* r, int slot) const {
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
    return o;
  }

  // context of a request on the slot's stream; the pinned input copy is
  // released once the device holds it (setup synchronises its stream)
  int make_ctx(Req* r, int slot) {
    gw_opts o = ctx_opts(r, slot);
    const size_t nov = (size_t)r->n_occ * (r->n_mo - r->n_occ);
    int rc = setup_cached(&r->ctx, r->n_mo, r->n_occ, r->n_aux, r->eps.data(), r->B, r->n_rows,
                          r->row_ids.data(), r->B + nov * r->n_aux, &o, cache);
    if (r->pinned_bytes) pinned.release(r->B, r->pinned_bytes);
    r->B = nullptr;
    r->pinned_bytes = 0;
    std::vector<double>().swap(r->B_pageable);
    const int n = (int)r->states.size();
    r->E.assign(n, 0.0);
    r->S.assign(n, 0.0);
    r->Z.assign(n, 0.0);
    r->status.assign(n, 0);
    return rc;
  }

  // quasiparticle stage (and stage A, unless a batch already built it)
  void qp(Req* r, int slot) {
    int rc = ctx_set_stream(r->ctx, streams[slot]);
    if (rc == 0) {
      gw_grid g{(int)xi.size(), xi.data(), w.data()};
      rc = gw_qp(r->ctx, (int)r->states.size(), r->states.data(), &g, r->E.data(), r->S.data(),
                 r->Z.data(), r->status.data());
    }
    gw_free(r->ctx);
    r->ctx = nullptr;
    r->rc = rc;
  }

  void process(Req* r, int slot) {
    const int rc = make_ctx(r, slot);
    if (rc != 0) {
      gw_free(r->ctx);
      r->ctx = nullptr;
      r->rc = rc;
      return;
    }
    qp(r, slot);
  }

  // stage A of a batch of one shape in one grouped launch sequence; the
  // members then wait in qp_ready for their quasiparticle stages
  void run_batch(std::vector<Req*>& batch, int slot) {
    ShapeGroup* sg = batch[0]->group;
    std::vector<Req*> ok;
    for (Req* r : batch) {
      const int rc = make_ctx(r, slot);
      if (rc != 0) {
        gw_free(r->ctx);
        r->ctx = nullptr;
        r->rc = rc;
        complete(r);
      } else {
        ok.push_back(r);
      }
    }
    if (ok.empty()) return;
    std::vector<gw_ctx*> ctxs;
    for (Req* r : ok) ctxs.push_back(r->ctx);
    std::vector<int> rcs(ok.size(), 0);
    int rc = 0;
    {
      std::lock_guard<std::mutex> lk(sg->mu);
      if (!sg->g) {
        gw_grid g{(int)xi.size(), xi.data(), w.data()};
        rc = group_create(&sg->g, sg->Np, sg->Kp, sg->Rp, &g, sg->n_max, opts.pi_prec,
                          opts.wc_prec, cache, true);
      }
      if (rc == 0) rc = group_run(sg->g, ctxs.data(), (int)ctxs.size(), rcs.data());
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      if (rc == 0) {
        batches++;
        batched += (long)ok.size();
      }
      for (size_t j = 0; j < ok.size(); ++j) {
        // a failed group leaves the member's stage A to its own gw_qp call
        if (rc != 0 || rcs[j] == 0) qp_ready.push_back(ok[j]);
      }
    }
    for (size_t j = 0; j < ok.size(); ++j) {
      if (rc == 0 && rcs[j] != 0) {
        gw_free(ok[j]->ctx);
        ok[j]->ctx = nullptr;
        ok[j]->rc = rcs[j];
        complete(ok[j]);
      }
    }
    cv_work.notify_all();
  }

  // the shape group of a small request (created, with its workspace reserved,
  // on first use); caller holds mu
  ShapeGroup* group_for(const Req* r) {
    if (opts.batch_max_aux < 0) return nullptr;
    const int lim = opts.batch_max_aux > 0 ? opts.batch_max_aux : 768;
    int Np, Kp, Rp;
    padded_shape(r->n_mo, r->n_occ, r->n_aux, r->n_rows, &Np, &Kp, &Rp);
    if (Np > lim) return nullptr;
    auto key = std::array<int, 3>{Np, Kp, Rp};
    auto it = groups.find(key);
    if (it != groups.end()) return it->second;
    ShapeGroup* sg = new ShapeGroup();
    sg->Np = Np;
    sg->Kp = Kp;
    sg->Rp = Rp;
    // batch size: as many requests as 2 GiB of grouped workspace holds, 1..8
    const size_t one = group_bytes(Np, Kp, Rp, (int)xi.size(), 1, opts.pi_prec, opts.wc_prec);
    sg->n_max = (int)std::max<size_t>(1, std::min<size_t>(8, (2ull << 30) / std::max<size_t>(one, 1)));
    sg->bytes = one * sg->n_max;
    if (reserved + sg->bytes > budget / 4) {
      sg->usable = false;
    } else {
      reserved += sg->bytes;   // held until the server is destroyed
      peak_reserved = std::max(peak_reserved, reserved);
    }
    groups[key] = sg;
    return sg;
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
  // launch-audit mode (no GPU): contexts walk their launch guards only, on
  // null streams, and the budget is the stated one or 64 GiB
  const bool audit = gw::audit_mode();
  if (!audit && hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return GW_EDEVICE;
  }
  size_t free_b = 0, total_b = 0;
  if (opts->mem_budget_bytes) {
    s->budget = opts->mem_budget_bytes;
  } else if (audit) {
    s->budget = 64ull << 30;
  } else {
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      delete s;
      return GW_EDEVICE;
    }
    s->budget = free_b / 10 * 8;
  }
  s->pinned.cap = 64ull << 30;
  for (int i = 0; i < ns; ++i) {
    hipStream_t st = nullptr;
    if (!audit && hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) hipStreamDestroy(x);
      delete s;
      return GW_EDEVICE;
    }
    s->streams.push_back(st);
  }
  s->cache = devcache_create(s->budget);
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
                                 s->opts.work_budget_bytes, 0);   // the contexts' default batch
  if (r->footprint > s->budget) {
    if (r->pinned_bytes) s->pinned.release(r->B, r->pinned_bytes);
    delete r;
    return GW_ENOMEM;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->group = s->group_for(r);
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
  s->cv_done.wait(lk, [&] { return s->pending.empty() && s->qp_ready.empty() && s->active == 0; });
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
  out->batches = s->batches;
  out->batched_requests = s->batched;
  long replays = 0;
  for (auto& kv : s->groups) {
    std::lock_guard<std::mutex> gl(kv.second->mu);
    if (kv.second->g) {
      long b, it, rp;
      group_stats(kv.second->g, &b, &it, &rp);
      replays += rp;
    }
  }
  out->graph_replays = replays;
  size_t live = 0;
  devcache_stats(s->cache, &out->device_mallocs, &out->cache_hits, &out->device_frees, &live,
                 &out->cached_bytes);
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
  for (auto& kv : s->groups) {
    if (kv.second->g) group_free(kv.second->g);
    delete kv.second;
  }
  for (hipStream_t st : s->streams)
    if (st) hipStreamDestroy(st);
  for (auto& kv : s->all) delete kv.second;
  devcache_destroy(s->cache);
  delete s;
}

}  // extern "C"
