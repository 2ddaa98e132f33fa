// Request server (continuous batching of scattering solves on one device).
//
// Worker threads ("slots"), each with its own HIP stream, take queued
// requests first-fit in arrival order under a device-memory budget: a
// request is admitted when its estimated footprint fits beside the running
// requests and the resident scatterers (unused residents are evicted, least
// recently used first), or alone on an idle server.  A request's work is the
// whole path -- mesh, CBF build, fill fused with the projection (panels
// sized to the request's share of the budget), CMP-GMRES, monostatic RCS --
// issued on its slot's stream, so requests admitted together overlap on the
// device.  Requests with the same nonzero key share one resident mesh, CBF
// set and Z_r: the first builds them, later ones only solve.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "cbf.h"

namespace cbfm {

namespace {

// Scratch for the fill + projection row panels of one request (a panel of
// one cell may exceed it).
constexpr size_t kPanelBudget = (size_t)1 << 30;

struct Resident {
  cbfm_mesh mesh = nullptr;
  cbfm_cbf cbf = nullptr;
  DevBuf Zr;
  int64_t n = 0;
  size_t bytes = 0;     // estimated resident footprint (accounting)
  int users = 0;        // admitted requests using it
  uint64_t last_use = 0;
  bool ready = false, failed = false;
  std::string err;
  ~Resident() {
    if (cbf) cbfm_cbf_free(cbf);
    if (mesh) cbfm_mesh_free(mesh);
  }
};

struct Job {
  int64_t ticket = 0;
  std::vector<double> xyz, gen, inc;
  std::vector<int32_t> tri, eb;
  int64_t nv = 0, nt = 0, nrhs = 0;
  int32_t nblocks = 1, n_gen = 0, precision = CBFM_FP64, max_iter = 0, restart = 0, inner_fp32 = 0;
  cbfm_medium med{};
  double delta = 0, tol = 1e-6;
  uint64_t key = 0;
  size_t transient = 0, resident = 0;  // estimated bytes
  bool builder = false;                // builds the resident entry of its key
  // results
  std::vector<double> rcs;
  std::vector<int32_t> iters;
  double t_submit = 0, t_start = 0, t_end = 0;
  cbfm_status status = CBFM_OK;
  std::string err;
  bool done = false;
};

// Estimated device bytes: (transient, resident) parts of a request.
std::pair<size_t, size_t> estimate(int64_t nt, const std::vector<int32_t>& eb, int32_t nblocks, int32_t S,
                                   int64_t nrhs, int32_t restart, int precision, size_t panel_budget) {
  const double ne = 1.5 * (double)nt;
  std::vector<double> N(std::max(1, nblocks), 0.0);
  if (eb.empty())
    N[0] = ne;
  else
    for (int32_t b : eb)
      if (b >= 0 && b < nblocks) N[b] += 1.0;
  double Nmax = 0, NL = 0;
  for (double x : N) {
    Nmax = std::max(Nmax, x);
    NL += std::min<double>(x, S);
  }
  const double nb = (double)N.size(), n = 2.0 * NL, z = 16.0;
  const double esz = precision == CBFM_FP64 ? 16.0 : 8.0;
  const double cell_local = 27 * 4 * Nmax * Nmax * z;  // one cell's triangle-local self block
  const double build = nb * 4 * Nmax * Nmax * z + nb * 2 * Nmax * S * z +
                       std::max(cell_local, std::min(nb * cell_local, (double)(1 << 30))) +
                       6 * nb * S * Nmax * z + 2 * nb * Nmax * Nmax * z + 2 * S * ne * z;
  const double cell_panel = 27 * 2 * Nmax * (double)nt * esz + 3 * Nmax * ne * z + 4 * Nmax * NL * z;
  const double panel = std::max<double>(cell_panel, (double)panel_budget);
  const double m = restart > 0 ? std::min<double>(restart, n) : std::min<double>(n, 1000);
  // Krylov basis, H and R, the operator, vectors, and the per-column
  // arrays (g, cs, sn and the two dot products)
  const double solve = (m + 1) * nrhs * n * z + 2 * nrhs * (m + 1) * m * z + n * n * z +
                       8 * nrhs * std::max(n, 2 * ne) * z + 5 * nrhs * (m + 1) * z;
  const double resident = n * n * z + NL * NL * z + 2 * ne * S * z + 2048.0 * nt;
  return {(size_t)(std::max(build, panel) + solve), (size_t)resident};
}

}  // namespace
}  // namespace cbfm

using namespace cbfm;

struct cbfm_server_s {
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_ready;
  std::deque<Job*> queue;
  std::map<int64_t, std::unique_ptr<Job>> jobs;
  std::map<uint64_t, std::unique_ptr<Resident>> residents;
  std::vector<std::thread> workers;
  size_t budget = 0, in_use = 0, resident_bytes = 0, peak = 0, panel_budget = 0;
  int running = 0, max_running = 0, device = 0;
  uint64_t tick = 0;
  int64_t next_ticket = 1;
  bool stop = false;
  std::chrono::steady_clock::time_point t0;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

  // Under mu: evict unused residents (least recently used first, never the
  // one of key `keep`) until `need` more bytes fit, or none is left to evict.
  bool make_room(size_t need, uint64_t keep) {
    while (in_use + resident_bytes + need > budget) {
      auto victim = residents.end();
      for (auto it = residents.begin(); it != residents.end(); ++it)
        if (it->second->users == 0 && it->second->ready && (keep == 0 || it->first != keep) &&
            (victim == residents.end() || it->second->last_use < victim->second->last_use))
          victim = it;
      if (victim == residents.end()) return false;
      resident_bytes -= victim->second->bytes;
      residents.erase(victim);
    }
    return true;
  }

  // Under mu: first request in arrival order that may start now.
  Job* admit() {
    for (auto it = queue.begin(); it != queue.end(); ++it) {
      Job* j = *it;
      const bool shared = j->key != 0 && residents.count(j->key);
      // a keyless request holds its own mesh, CBFs and Z_r while it runs; a
      // keyed one adds them unless its key is already resident
      const size_t need = j->transient + (j->key == 0 || !shared ? j->resident : 0);
      // (the resident a keyed request will use is not evicted for it)
      if (!make_room(need, shared ? j->key : 0) && running > 0) continue;
      queue.erase(it);
      in_use += j->transient;
      if (j->key != 0) {
        if (!shared) {
          auto r = std::make_unique<Resident>();
          r->bytes = j->resident;
          resident_bytes += r->bytes;
          residents.emplace(j->key, std::move(r));
          j->builder = true;
        }
        residents[j->key]->users += 1;
      } else {
        in_use += j->resident;
      }
      running += 1;
      max_running = std::max(max_running, running);
      peak = std::max(peak, in_use + resident_bytes);
      return j;
    }
    return nullptr;
  }

  void run(Job* j, hipStream_t s);
  void worker();
};

// Mesh, CBFs and Z_r of a request (into `r`), on stream s.
static void build_scatterer(cbfm_server_s* srv, Job* j, Resident* r, hipStream_t s) {
  auto chk = [](cbfm_status st) {
    if (st != CBFM_OK) throw Error{st, cbfm_last_error()};
  };
  chk(cbfm_mesh_load(j->xyz.data(), j->nv, j->tri.data(), j->nt, j->eb.empty() ? nullptr : j->eb.data(), j->nblocks,
                     &r->mesh));
  cbfm_cbf_params cp{j->gen.data(), j->n_gen, j->delta, 0};
  chk(cbfm_build_cbf(r->mesh, &j->med, &cp, s, &r->cbf));
  int64_t n = 0;
  chk(cbfm_cbf_info(r->cbf, &n, nullptr, nullptr));
  r->n = n;
  r->Zr.alloc((size_t)n * n * sizeof(double2));
  project_dev(r->mesh, make_media(&j->med), r->cbf, j->precision, r->Zr.as<double2>(), n, s, srv->panel_budget);
  CBFM_HIP(hipStreamSynchronize(s));
}

void cbfm_server_s::run(Job* j, hipStream_t s) {
  Resident local;
  Resident* r = &local;
  try {
    if (j->key != 0) {
      std::unique_lock<std::mutex> lk(mu);
      r = residents.at(j->key).get();
      if (!j->builder) {
        cv_ready.wait(lk, [&] { return r->ready || r->failed; });
        if (r->failed) throw Error{CBFM_E_STATE, "shared scatterer failed: " + r->err};
      }
    }
    if (j->key == 0 || j->builder) {
      try {
        build_scatterer(this, j, r, s);
      } catch (const Error& e) {
        if (j->key != 0) {
          std::lock_guard<std::mutex> lk(mu);
          r->failed = true;
          r->err = e.msg;
          cv_ready.notify_all();
        }
        throw;
      }
      if (j->key != 0) {
        std::lock_guard<std::mutex> lk(mu);
        r->ready = true;
        cv_ready.notify_all();
      }
    }
    cbfm_solver_params sp{};
    sp.tol = j->tol;
    sp.max_iter = j->max_iter > 0 ? j->max_iter : 3000;
    sp.restart = j->restart > 0 ? j->restart : (int32_t)std::min<int64_t>(r->n, 1000);
    sp.use_cmp = 1;
    sp.inner_fp32 = j->inner_fp32 ? 1 : 0;
    j->rcs.assign(j->nrhs, 0.0);
    j->iters.assign(j->nrhs, 0);
    const cbfm_status st = cbfm_solve(r->mesh, &j->med, r->cbf, r->Zr.p, r->n, j->inc.data(), j->nrhs, &sp, nullptr,
                                      j->iters.data(), nullptr, nullptr, 0, j->rcs.data(), s);
    j->status = st;
    if (st != CBFM_OK) j->err = cbfm_last_error();
  } catch (const Error& e) {
    j->status = e.code;
    j->err = e.msg;
  } catch (const std::exception& e) {
    j->status = CBFM_E_HIP;
    j->err = e.what();
  }
}

void cbfm_server_s::worker() {
  hipStream_t s = nullptr;
  size_t trim_limit = 0;
  const bool ok = hipSetDevice(device) == hipSuccess && hipStreamCreate(&s) == hipSuccess;
  cbfm::async_cmp_on_this_thread(false);  // requests overlap one another already
  for (;;) {
    Job* j = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return (j = admit()) != nullptr || (stop && queue.empty()); });
      if (!j) break;
      j->t_start = now();
    }
    if (ok) {
      run(j, s);
    } else {
      j->status = CBFM_E_HIP;
      j->err = "the worker could not create its HIP stream";
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      j->t_end = now();
      in_use -= j->transient;
      if (j->key != 0) {
        auto it = residents.find(j->key);
        if (it != residents.end()) {
          it->second->users -= 1;
          it->second->last_use = ++tick;
          if (it->second->failed && it->second->users == 0) {
            resident_bytes -= it->second->bytes;
            residents.erase(it);
          }
        }
      } else {
        in_use -= j->resident;
      }
      running -= 1;
      j->done = true;
      // idle cached scratch may hold what the running requests and the
      // residents leave of the budget, no more
      const size_t used = in_use + resident_bytes;
      trim_limit = budget > used ? budget - used : 0;
    }
    scratch_trim_to(trim_limit);
    cv_done.notify_all();
    cv_work.notify_all();
  }
  if (s) {
    // the scratch cache must not keep this stream's handle or events
    (void)hipStreamSynchronize(s);
    scratch_forget_stream(s);
    (void)hipStreamDestroy(s);
  }
}

extern "C" {

cbfm_status cbfm_request_footprint(const cbfm_request* req, int64_t* bytes) {
  return guarded([&] {
    CBFM_REQUIRE(req && bytes, CBFM_E_ARG, "null argument");
    std::vector<int32_t> eb;
    if (req->edge_block) eb.assign(req->edge_block, req->edge_block + (size_t)(3 * req->nt / 2));
    const auto e = estimate(req->nt, eb, req->edge_block ? req->nblocks : 1, req->n_gen, req->nrhs, req->restart,
                            req->precision, kPanelBudget);
    *bytes = (int64_t)(e.first + e.second);
  });
}

cbfm_status cbfm_server_create(int32_t slots, int64_t budget_bytes, cbfm_server* out) {
  return guarded([&] {
    CBFM_REQUIRE(out, CBFM_E_ARG, "null argument");
    CBFM_REQUIRE(slots >= 1 && slots <= 16, CBFM_E_ARG, "slots outside [1, 16]");
    CBFM_REQUIRE(budget_bytes > 0, CBFM_E_ARG, "budget must be positive");
    auto srv = std::make_unique<cbfm_server_s>();
    CBFM_HIP(hipGetDevice(&srv->device));
    srv->budget = (size_t)budget_bytes;
    srv->panel_budget = kPanelBudget;
    srv->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < slots; ++i) srv->workers.emplace_back([p = srv.get()] { p->worker(); });
    *out = srv.release();
  });
}

cbfm_status cbfm_server_submit(cbfm_server srv, const cbfm_request* req, int64_t* ticket) {
  return guarded([&] {
    CBFM_REQUIRE(srv && req && ticket, CBFM_E_ARG, "null argument");
    CBFM_REQUIRE(req->xyz_host && req->tri_host && req->gen_host && req->inc_host, CBFM_E_ARG, "null input array");
    CBFM_REQUIRE(req->nv > 0 && req->nt > 0 && req->n_gen > 0 && req->nrhs > 0, CBFM_E_ARG, "empty input");
    CBFM_REQUIRE(req->tol > 0, CBFM_E_ARG, "tol must be positive");
    CBFM_REQUIRE(req->precision >= CBFM_FP64 && req->precision <= CBFM_MIXED_BF16X3, CBFM_E_ARG, "unknown precision");
    auto j = std::make_unique<Job>();
    j->xyz.assign(req->xyz_host, req->xyz_host + 3 * req->nv);
    j->tri.assign(req->tri_host, req->tri_host + 3 * req->nt);
    if (req->edge_block) j->eb.assign(req->edge_block, req->edge_block + (size_t)(3 * req->nt / 2));
    j->gen.assign(req->gen_host, req->gen_host + 6 * (size_t)req->n_gen);
    j->inc.assign(req->inc_host, req->inc_host + 6 * (size_t)req->nrhs);
    j->nv = req->nv;
    j->nt = req->nt;
    j->nrhs = req->nrhs;
    j->nblocks = req->edge_block ? req->nblocks : 1;
    j->n_gen = req->n_gen;
    j->precision = req->precision;
    j->max_iter = req->max_iter;
    j->restart = req->restart;
    j->inner_fp32 = req->inner_fp32;
    j->med = req->medium;
    j->delta = req->delta_svd;
    j->tol = req->tol;
    j->key = req->scatterer_key;
    const auto e = estimate(j->nt, j->eb, j->nblocks, j->n_gen, j->nrhs, j->restart, j->precision, srv->panel_budget);
    j->transient = e.first;
    j->resident = e.second;
    std::lock_guard<std::mutex> lk(srv->mu);
    CBFM_REQUIRE(!srv->stop, CBFM_E_STATE, "server is stopping");
    j->ticket = srv->next_ticket++;
    j->t_submit = srv->now();
    *ticket = j->ticket;
    srv->queue.push_back(j.get());
    srv->jobs.emplace(j->ticket, std::move(j));
    srv->cv_work.notify_all();
  });
}

cbfm_status cbfm_server_wait(cbfm_server srv, int64_t ticket, double* rcs_host, int32_t* iters_host,
                             double* times_host) {
  std::unique_ptr<Job> j;
  const cbfm_status st = guarded([&] {
    CBFM_REQUIRE(srv, CBFM_E_ARG, "null server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->jobs.find(ticket);
    CBFM_REQUIRE(it != srv->jobs.end(), CBFM_E_ARG, "unknown ticket");
    Job* p = it->second.get();
    srv->cv_done.wait(lk, [&] { return p->done; });
    j = std::move(it->second);
    srv->jobs.erase(it);
  });
  if (st != CBFM_OK) return st;
  if (rcs_host) std::memcpy(rcs_host, j->rcs.data(), j->rcs.size() * sizeof(double));
  if (iters_host) std::memcpy(iters_host, j->iters.data(), j->iters.size() * sizeof(int32_t));
  if (times_host) {
    times_host[0] = j->t_submit;
    times_host[1] = j->t_start;
    times_host[2] = j->t_end;
  }
  if (j->status != CBFM_OK) set_error(j->err);
  return j->status;
}

cbfm_status cbfm_server_stats(cbfm_server srv, int64_t* peak_bytes, int32_t* max_running, int32_t* resident) {
  return guarded([&] {
    CBFM_REQUIRE(srv, CBFM_E_ARG, "null server");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (peak_bytes) *peak_bytes = (int64_t)srv->peak;
    if (max_running) *max_running = srv->max_running;
    if (resident) *resident = (int32_t)srv->residents.size();
  });
}

void cbfm_server_destroy(cbfm_server srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->workers) t.join();
  delete srv;
}

}  // extern "C"
