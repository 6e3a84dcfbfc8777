// Serving: many DD solves (Section 2's fixed-point loop) against one resident
// dataset, with their projections P_D batched across solves.
//
// Two host threads per server.  The scheduler admits queued solves in arrival
// order while their device footprint fits the budget, and advances every
// admitted solve through its DD iterations without blocking: each solve owns a
// HIP stream, its constraint projection P_C runs there in batches of CG
// iterations polled through events.  A solve whose admissible state y is ready
// joins the next projection batch; the projection thread concatenates the
// whitened states of every ready solve (a large mesh may span several
// batches), runs one dd_project over them on its own stream and scatters the
// associations back.  While a batch runs, the other solves keep iterating on
// their streams and queue for the next batch (continuous batching).  Every
// solve's arithmetic is the one of dd_solve, so its result does not depend on
// the mix it ran in.
//
// Device memory.  The server holds a fixed reserve from creation to destroy:
// the batch buffers and the scratch of the largest projection batch (every
// temporary buffer of the batch's projection is carved from it, so the
// projection allocates nothing and never exceeds it).  A solve is charged its
// solver buffers while it is admitted.  A mesh that dd_solve would solve through a cached K^-1
// and whose inverse the dataset does not hold yet is charged that inverse too:
// the inverse is formed on a builder thread (the solve waits, the others go
// on) and stays charged to the server while the dataset's cache keeps it.  A
// solve whose inverse could not fit next to it even on an idle server is run
// by CG instead (the trajectory of dd_solve with DD_SOLVE_CG).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <future>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "scan.h"
#include "solve.h"

namespace dd {

size_t project_scratch_need(const Dataset& D, int mode, int64_t m_max);
dd_status project_reserved(const Dataset& D, const double* states_dev, bool whitened, int64_t m,
                           const int64_t* warm_start_idx_dev, const dd_project_opts* opts,
                           int64_t* idx_out_dev, double* dist_out_dev, ScratchArena* arena,
                           hipStream_t st);

namespace {

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0, Clock::time_point t1) {
  return std::chrono::duration<double, std::milli>(t1 - t0).count();
}

struct Job {
  uint64_t ticket = 0;
  dd_mesh mesh{};
  std::vector<uint8_t> mask;
  std::vector<double> force;
  std::vector<int64_t> init;
  int max_iter = 500;
  double deadline_s = 0.0;
  int64_t footprint = 0;
  int64_t inv_bytes = 0;       // K^-1 the solve would use (0: solved by CG)
  bool use_cg = false;         // run by CG: its K^-1 does not fit the budget
  std::string inv_key;         // mesh and Dirichlet pattern of its K^-1
  int64_t n_mp = 0, n_dof = 0;

  enum Phase { kQueued, kInverse, kCg, kReady, kInBatch, kScalars, kDone };
  Phase phase = kQueued;       // scheduler thread only
  bool done = false;           // results published (guarded by mu): the waiter may free the job
  bool cancel = false;
  dd_status status = DD_OK;
  std::string error;

  std::unique_ptr<DDSolver> S;
  hipStream_t stream = nullptr;
  int it = 0;                  // DD iterations completed
  int64_t pd_next = 0;         // next material point to hand to a projection batch
  int64_t pd_done = 0;         // material points projected in this iteration
  double prev_full = INFINITY;
  int stop_reason = 0;
  int64_t cg_total = 0;
  double cg_res_max = 0.0;

  Clock::time_point t_submit, t_admit, t_ready, t_done;
  // results (host)
  std::vector<double> u, eps, sig, d_half, d_full;
  std::vector<int64_t> idx, changed;
};

struct Chunk {
  Job* job;
  int64_t first, count, at;   // job's material points [first, first+count) at batch offset at
};

}  // namespace

struct Server {
  const Dataset* D = nullptr;
  int device = 0;
  int mode = DD_MIXED_BF16;
  int ann_budget = 0;
  int max_active = 64;
  int64_t max_batch = 65536;
  int64_t max_queue = 4096;
  int64_t budget = 0;

  std::mutex mu;
  std::condition_variable cv_done;     // a job finished
  std::condition_variable cv_work;     // work for the scheduler (submit, cancel, stop)
  std::deque<Job*> queue;              // submitted, not admitted (arrival order)
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  uint64_t next_ticket = 1;
  std::atomic<bool> stop{false};

  // scheduler-thread state
  std::vector<Job*> active;
  int64_t used = 0;
  // K^-1 formed ahead of setup: builds in flight (key -> result, bytes) and the
  // inverses this server formed that the dataset still caches (key -> bytes)
  struct Build {
    std::shared_future<std::pair<dd_status, std::string>> done;
    int64_t bytes;
  };
  std::map<std::string, Build> building;
  std::map<std::string, int64_t> formed;
  int64_t held_bytes();
  std::atomic<int64_t> n_active{0};

  // projection thread
  std::mutex pmu;
  std::condition_variable pcv;
  std::vector<Chunk> batch;            // the batch in flight
  bool batch_posted = false;
  std::atomic<bool> batch_done{false};
  dd_status batch_status = DD_OK;
  std::string batch_error;
  hipStream_t pst = nullptr;
  DevBuf bq, bw, bi, bd;               // batch buffers: states, warm start, idx, dist
  std::unique_ptr<ScratchArena> scratch;   // the batch projection's scratch (its own block)
  int64_t reserve = 0;                 // batch buffers + scratch block, held throughout

  // statistics (under mu)
  Clock::time_point t_create, t_first_submit;
  bool any_submit = false;
  int64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_rejected = 0, n_cancelled = 0;
  int64_t n_batches = 0, n_queries = 0, peak_active = 0, peak_used = 0;
  std::vector<double> lat_proj, lat_solve, lat_queue;

  std::thread sched_thr, proj_thr;

  void scheduler();
  void projector();
  dd_status admit(Job* j);
  dd_status admit_setup(Job* j);
  void finish(Job* j, dd_status st, const std::string& msg);
  bool step(Job* j);
  void launch_batch();
  void complete_batch();
};

// ---------------------------------------------------------------------------
// scheduler thread
// ---------------------------------------------------------------------------
// Bytes of the inverses in flight and of those this server formed that the
// dataset still caches (dropped from the charge once the cache lets them go).
int64_t Server::held_bytes() {
  int64_t b = 0;
  for (const auto& kv : building) b += kv.second.bytes;
  for (auto it = formed.begin(); it != formed.end();) {
    dd_mesh m;
    std::memcpy(&m, it->first.data(), sizeof(m));
    const uint8_t* mask = reinterpret_cast<const uint8_t*>(it->first.data() + sizeof(m));
    if (DDSolver::inverse_cached(*D, m, mask)) {
      b += it->second;
      ++it;
    } else {
      it = formed.erase(it);
    }
  }
  return b;
}

dd_status Server::admit(Job* j) {
  DD_HIP(hipStreamCreateWithFlags(&j->stream, hipStreamNonBlocking));
  if (j->inv_bytes > 0 && !j->use_cg && !DDSolver::inverse_cached(*D, j->mesh, j->mask.data())) {
    // form K^-1 on a builder thread (or wait for the build of the same
    // inverse already in flight); the solve waits in kInverse
    if (!building.count(j->inv_key)) {
      const Dataset* ds = D;
      const int dev = device;
      const dd_mesh mesh = j->mesh;
      std::vector<uint8_t> mask = j->mask;
      auto fut = std::async(std::launch::async, [ds, dev, mesh, mask]() {
        std::pair<dd_status, std::string> r{DD_OK, std::string()};
        hipStream_t s = nullptr;
        if (hipSetDevice(dev) != hipSuccess ||
            hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
          r.first = set_error(DD_ERR_DEVICE, "K^-1 builder: no stream");
        } else {
          r.first = DDSolver::prepare_inverse(*ds, mesh, mask.data(), s);
          (void)hipStreamDestroy(s);
        }
        if (r.first != DD_OK) r.second = dd_last_error();
        return r;
      });
      building[j->inv_key] = Build{fut.share(), j->inv_bytes};
    }
    j->phase = Job::kInverse;
    return DD_OK;
  }
  return admit_setup(j);
}

dd_status Server::admit_setup(Job* j) {
  j->S.reset(new DDSolver());
  dd_solve_opts o{};
  o.mode = mode;
  o.ann_budget = ann_budget;
  o.flags = DD_SOLVE_NO_GRAPH | (j->use_cg ? DD_SOLVE_CG : 0);
  DD_TRY(j->S->setup(*D, j->mesh, j->mask.data(), j->force.data(), &o, j->stream));
  DD_TRY(j->S->set_assignment(j->init.data()));
  DD_TRY(j->S->async_init());
  DD_TRY(j->S->pc_begin());
  DD_TRY(j->S->cg_batch());
  j->phase = Job::kCg;
  return DD_OK;
}

void Server::finish(Job* j, dd_status st, const std::string& msg) {
  if (j->stream) (void)hipStreamSynchronize(j->stream);
  if (st == DD_OK || st == DD_ERR_NOT_CONVERGED) {
    j->u.resize(j->n_dof);
    j->idx.resize(j->n_mp);
    j->eps.resize(6 * j->n_mp);
    j->sig.resize(6 * j->n_mp);
    dd_status f = j->S->fetch_results(j->u.data(), j->idx.data(), j->eps.data(), j->sig.data());
    if (f != DD_OK) {
      st = f;
    }
  }
  std::string err = (st == DD_OK) ? std::string() : (msg.empty() ? std::string(dd_last_error()) : msg);
  if (j->S) j->S.reset();
  if (j->stream) (void)hipStreamDestroy(j->stream);
  j->stream = nullptr;
  used -= j->footprint;
  std::lock_guard<std::mutex> lk(mu);
  j->status = st;
  j->error = err;
  j->t_done = Clock::now();
  j->phase = Job::kDone;   // published (done) once the scheduler has let go of the job
  if (st == DD_OK || st == DD_ERR_NOT_CONVERGED) {
    ++n_completed;
    lat_solve.push_back(ms_since(j->t_submit, j->t_done));
  } else if (st == DD_ERR_CANCELLED) {
    ++n_cancelled;
  } else {
    ++n_failed;
  }
}

// Advances one admitted job as far as it can go without waiting.  Returns true
// if anything changed.
bool Server::step(Job* j) {
  bool cancel;
  {
    std::lock_guard<std::mutex> lk(mu);
    cancel = j->cancel;
  }
  if (!cancel && j->deadline_s > 0 && ms_since(j->t_submit, Clock::now()) > 1e3 * j->deadline_s)
    cancel = true;
  if (cancel && j->phase != Job::kInBatch) {
    finish(j, DD_ERR_CANCELLED, "solve cancelled");
    return true;
  }
  if (j->phase == Job::kInverse) {
    // the build was swept when it ended; setup() then finds the inverse cached
    // (or, after a failed build, forms it itself and reports its error)
    if (building.count(j->inv_key)) return false;
    const dd_status st = admit_setup(j);
    if (st != DD_OK) finish(j, st, "");
    return true;
  }
  DDSolver& S = *j->S;
  dd_status st = DD_OK;
  switch (j->phase) {
    case Job::kCg: {
      if (hipEventQuery(S.ev_cg) != hipSuccess) return false;
      if (!S.cg_finished()) {
        st = S.cg_batch();
      } else {
        st = S.pc_end();
        if (st == DD_OK) {
          j->cg_total += S.cg_last_iters[0] + S.cg_last_iters[1];
          j->cg_res_max = std::max({j->cg_res_max, S.cg_last_res[0], S.cg_last_res[1]});
          j->phase = Job::kReady;
          j->pd_next = 0;
          j->pd_done = 0;
          j->t_ready = Clock::now();
        }
      }
      break;
    }
    case Job::kScalars: {
      if (hipEventQuery(S.ev_scal) != hipSuccess) return false;
      double sc[3];
      int bad = 0;
      S.scalars_end(sc, &bad);
      if (bad) {
        finish(j, DD_ERR_DEVICE, "dd_solve: the admissible state became non-finite");
        return true;
      }
      j->it += 1;
      j->d_half.push_back(sc[0]);
      j->d_full.push_back(sc[1]);
      j->changed.push_back((int64_t)sc[2]);
      const bool approximate = (walk_mode(mode) && ann_budget > 0);
      if (sc[2] == 0.0) {
        j->stop_reason = 1;
      } else if (approximate && j->it > 1 && !(sc[1] < j->prev_full)) {
        j->stop_reason = 2;
      }
      j->prev_full = sc[1];
      if (j->stop_reason != 0) {
        finish(j, DD_OK, "");
        return true;
      }
      if (j->it >= j->max_iter) {
        finish(j, DD_ERR_NOT_CONVERGED, "dd_solve reached max_iter");
        return true;
      }
      st = S.pc_begin();
      if (st == DD_OK) st = S.cg_batch();
      if (st == DD_OK) j->phase = Job::kCg;
      break;
    }
    default:
      return false;
  }
  if (st != DD_OK) {
    finish(j, st, "");
  }
  return true;
}

// Packs the oldest ready solves (whole or in part) into one batch and posts it.
void Server::launch_batch() {
  std::vector<Job*> ready;
  for (Job* j : active)
    if ((j->phase == Job::kReady || j->phase == Job::kInBatch) && j->pd_next < j->n_mp) ready.push_back(j);
  if (ready.empty()) return;
  std::stable_sort(ready.begin(), ready.end(),
                   [](const Job* a, const Job* b) { return a->t_ready < b->t_ready; });
  std::vector<Chunk> b;
  int64_t at = 0;
  for (Job* j : ready) {
    if (at >= max_batch) break;
    const int64_t n = std::min(j->n_mp - j->pd_next, max_batch - at);
    b.push_back(Chunk{j, j->pd_next, n, at});
    j->pd_next += n;
    j->phase = Job::kInBatch;
    at += n;
  }
  {
    std::lock_guard<std::mutex> lk(pmu);
    batch = std::move(b);
    batch_done = false;
    batch_posted = true;
  }
  pcv.notify_one();
}

void Server::complete_batch() {
  std::vector<Chunk> b;
  dd_status bst;
  std::string berr;
  {
    std::lock_guard<std::mutex> lk(pmu);
    b = std::move(batch);
    batch.clear();
    batch_posted = false;
    bst = batch_status;
    berr = batch_error;
  }
  int64_t q = 0;
  for (const Chunk& c : b) q += c.count;
  {
    std::lock_guard<std::mutex> lk(mu);
    ++n_batches;
    n_queries += q;
  }
  const auto now = Clock::now();
  for (const Chunk& c : b) {
    Job* j = c.job;
    if (j->phase == Job::kDone) continue;
    if (bst != DD_OK) {
      finish(j, bst, berr);
      continue;
    }
    j->pd_done += c.count;
    if (j->pd_done < j->n_mp) {
      j->phase = Job::kReady;   // more of its points wait for the next batch
      continue;
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      lat_proj.push_back(ms_since(j->t_ready, now));
    }
    dd_status st = j->S->scalars_begin();
    if (st != DD_OK) {
      finish(j, st, "");
      continue;
    }
    j->phase = Job::kScalars;
  }
}

void Server::scheduler() {
  (void)hipSetDevice(device);
  for (;;) {
    bool progress = false;
    // finished K^-1 builds: charged while the dataset caches the inverse
    for (auto it = building.begin(); it != building.end();) {
      if (it->second.done.wait_for(std::chrono::seconds(0)) == std::future_status::ready) {
        if (it->second.done.get().first == DD_OK) formed[it->first] = it->second.bytes;
        it = building.erase(it);
        progress = true;
      } else {
        ++it;
      }
    }
    // admission: arrival order, as long as the footprint fits
    {
      std::unique_lock<std::mutex> lk(mu);
      if (stop) break;
      // cancelled while queued
      for (auto it = queue.begin(); it != queue.end();) {
        Job* j = *it;
        if (j->cancel) {
          j->status = DD_ERR_CANCELLED;
          j->error = "solve cancelled";
          j->phase = Job::kDone;
          j->done = true;
          j->t_done = Clock::now();
          ++n_cancelled;
          it = queue.erase(it);
          cv_done.notify_all();
          progress = true;
        } else {
          ++it;
        }
      }
      while (!queue.empty() && (int)active.size() < max_active) {
        Job* j = queue.front();
        // the K^-1 this solve would form: charged from admission on; one that
        // cannot fit next to the solve even on an idle server means CG
        int64_t extra = 0;
        if (j->inv_bytes > 0 && !j->use_cg && !building.count(j->inv_key) &&
            !DDSolver::inverse_cached(*D, j->mesh, j->mask.data())) {
          if (reserve + j->footprint + j->inv_bytes > budget)
            j->use_cg = true;
          else
            extra = j->inv_bytes;
        }
        const int64_t held = held_bytes();
        if (reserve + used + held + j->footprint + extra > budget) break;
        queue.pop_front();
        j->t_admit = Clock::now();
        lat_queue.push_back(ms_since(j->t_submit, j->t_admit));
        used += j->footprint;
        active.push_back(j);
        peak_active = std::max<int64_t>(peak_active, (int64_t)active.size());
        lk.unlock();
        dd_status st = admit(j);
        if (st != DD_OK) finish(j, st, "");
        lk.lock();
        peak_used = std::max(peak_used, reserve + used + held_bytes());
        progress = true;
      }
    }
    for (Job* j : active)
      if (j->phase != Job::kDone) progress |= step(j);
    if (batch_posted && batch_done.load()) {
      complete_batch();
      progress = true;
    }
    if (!batch_posted) launch_batch();
    // drop finished jobs from the active set, then publish them: a waiter may
    // free a published job at once, so the scheduler must not touch it again
    {
      std::vector<Job*> keep, gone;
      for (Job* j : active) (j->phase == Job::kDone ? gone : keep).push_back(j);
      if (!gone.empty()) {
        active.swap(keep);
        std::lock_guard<std::mutex> lk(mu);
        for (Job* j : gone) j->done = true;
        cv_done.notify_all();
        progress = true;
      }
    }
    n_active = (int64_t)active.size();
    if (!progress) {
      std::unique_lock<std::mutex> lk(mu);
      if (stop) break;
      if (active.empty() && queue.empty())
        cv_work.wait_for(lk, std::chrono::milliseconds(50));
      else
        cv_work.wait_for(lk, std::chrono::microseconds(50));
    }
  }
  // shutdown: wait for the projection thread, then cancel what is left
  for (;;) {
    if (!batch_posted) break;
    if (batch_done.load()) {
      complete_batch();
      break;
    }
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
  for (Job* j : active)
    if (j->phase != Job::kDone) finish(j, DD_ERR_CANCELLED, "server destroyed");
  std::lock_guard<std::mutex> lk(mu);
  for (Job* j : active) j->done = true;
  active.clear();
  for (Job* j : queue) {
    j->status = DD_ERR_CANCELLED;
    j->error = "server destroyed";
    j->phase = Job::kDone;
    j->done = true;
    ++n_cancelled;
  }
  queue.clear();
  cv_done.notify_all();
}

// ---------------------------------------------------------------------------
// projection thread
// ---------------------------------------------------------------------------
void Server::projector() {
  (void)hipSetDevice(device);
  for (;;) {
    std::vector<Chunk> b;
    {
      std::unique_lock<std::mutex> lk(pmu);
      pcv.wait(lk, [&] { return (batch_posted && !batch_done.load()) || stop; });
      if (stop && !(batch_posted && !batch_done.load())) return;
      b = batch;
    }
    dd_status st = DD_OK;
    int64_t total = 0;
    for (const Chunk& c : b) {
      DDSolver& S = *c.job->S;
      if (st == DD_OK && hipStreamWaitEvent(pst, S.ev_ready, 0) != hipSuccess) st = DD_ERR_DEVICE;
      if (st == DD_OK &&
          hipMemcpyAsync(bq.as<double>() + 12 * c.at, S.d_yw.as<double>() + 12 * c.first,
                         sizeof(double) * 12 * c.count, hipMemcpyDeviceToDevice, pst) != hipSuccess)
        st = DD_ERR_DEVICE;
      if (st == DD_OK &&
          hipMemcpyAsync(bw.as<int64_t>() + c.at, S.d_idx.as<int64_t>() + c.first,
                         sizeof(int64_t) * c.count, hipMemcpyDeviceToDevice, pst) != hipSuccess)
        st = DD_ERR_DEVICE;
      total = std::max(total, c.at + c.count);
    }
    std::string err;
    if (st == DD_OK) {
      dd_project_opts o{};
      o.mode = mode;
      o.ann_budget = ann_budget;
      st = project_reserved(*D, bq.as<double>(), true, total, bw.as<int64_t>(), &o,
                            bi.as<int64_t>(), bd.as<double>(), scratch.get(), pst);
    }
    if (st == DD_OK) {
      for (const Chunk& c : b) {
        DDSolver& S = *c.job->S;
        if (hipMemcpyAsync(S.d_idx_new.as<int64_t>() + c.first, bi.as<int64_t>() + c.at,
                           sizeof(int64_t) * c.count, hipMemcpyDeviceToDevice, pst) != hipSuccess ||
            hipMemcpyAsync(S.d_dist.as<double>() + c.first, bd.as<double>() + c.at,
                           sizeof(double) * c.count, hipMemcpyDeviceToDevice, pst) != hipSuccess) {
          st = DD_ERR_DEVICE;
          break;
        }
      }
    }
    if (hipStreamSynchronize(pst) != hipSuccess && st == DD_OK) st = DD_ERR_DEVICE;
    if (st != DD_OK) err = dd_last_error();
    {
      std::lock_guard<std::mutex> lk(pmu);
      batch_status = st;
      batch_error = err;
    }
    batch_done = true;
    cv_work.notify_one();
  }
}

}  // namespace dd

struct dd_server {
  dd::Server s;
};

namespace {

dd_status check_request(const dd::Dataset& D, const dd_solve_request* r) {
  using dd::set_error;
  if (!r) return set_error(DD_ERR_ARG, "request is NULL");
  const dd_mesh& m = r->mesh;
  if (m.nx < 1 || m.ny < 1 || m.nz < 1 || !(m.lx > 0) || !(m.ly > 0) || !(m.lz > 0))
    return set_error(DD_ERR_ARG, "mesh needs nx, ny, nz >= 1 and positive edge lengths");
  if ((int64_t)m.nx * m.ny * m.nz > (1 << 24)) return set_error(DD_ERR_TOO_LARGE, "mesh too large");
  if (!r->dirichlet_mask || !r->nodal_force || !r->init_idx)
    return set_error(DD_ERR_ARG, "request needs mask, force and init_idx");
  if (r->max_iter < 0 || r->deadline_s < 0 || r->reserved != 0)
    return set_error(DD_ERR_ARG, "request: max_iter and deadline must be >= 0, reserved 0");
  const int64_t nd = 3 * (int64_t)(m.nx + 1) * (m.ny + 1) * (m.nz + 1);
  const int64_t nm = 8 * (int64_t)m.nx * m.ny * m.nz;
  for (int64_t i = 0; i < nd; ++i)
    if (!std::isfinite(r->nodal_force[i])) return set_error(DD_ERR_ARG, "non-finite nodal force");
  for (int64_t e = 0; e < nm; ++e)
    if (r->init_idx[e] < 0 || r->init_idx[e] >= D.N) return set_error(DD_ERR_ARG, "init_idx out of range");
  return DD_OK;
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double r = p / 100.0 * (double)(v.size() - 1);
  const size_t lo = (size_t)r;
  const size_t hi = std::min(lo + 1, v.size() - 1);
  return v[lo] + (r - (double)lo) * (v[hi] - v[lo]);
}

}  // namespace

extern "C" dd_status dd_server_create(const dd_dataset* ds, size_t hbm_budget_bytes,
                                      const dd_server_opts* opts, dd_server** out) {
  using namespace dd;
  if (!out) return set_error(DD_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!ds) return set_error(DD_ERR_ARG, "dataset is NULL");
  const Dataset& D = ds->d;
  int mode = DD_MIXED_BF16;
  if (opts && opts->mode >= 0) mode = opts->mode;
  if (opts && (opts->max_active < 0 || opts->max_batch < 0 || opts->ann_budget < 0 ||
               opts->max_queue < 0 || opts->reserved != 0))
    return set_error(DD_ERR_ARG, "dd_server_opts: negative field or reserved != 0");
  const bool ok = (mode == DD_EXACT_FP64 && (D.packs & DD_PACK_FP64)) ||
                  (mode == DD_DIRECT_FP64 && (D.packs & DD_PACK_FP64)) ||
                  (mode == DD_MIXED_FP32 && (D.packs & DD_PACK_FP32)) ||
                  (mode == DD_MIXED_BF16 && (D.packs & DD_PACK_BF16)) ||
                  (mode == DD_MIXED_FP16 && (D.packs & DD_PACK_FP16)) ||
                  (mode == DD_ANN && (D.packs & DD_PACK_ANN)) ||
                  (mode == DD_KMEANS && (D.packs & DD_PACK_KMEANS));
  if (!ok) return set_error(DD_ERR_UNSUPPORTED, "dataset lacks the pack of the server's mode");
  std::unique_ptr<dd_server> h(new (std::nothrow) dd_server());
  if (!h) return set_error(DD_ERR_OOM, "host allocation failed");
  Server& s = h->s;
  s.D = &D;
  s.device = D.device;
  s.mode = mode;
  s.ann_budget = opts ? opts->ann_budget : 0;
  if (opts && opts->max_active > 0) s.max_active = opts->max_active;
  if (opts && opts->max_batch > 0) s.max_batch = opts->max_batch;
  if (opts && opts->max_queue > 0) s.max_queue = opts->max_queue;
  DD_HIP(hipSetDevice(D.device));
  if (hbm_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    DD_HIP(hipMemGetInfo(&fr, &tot));
    hbm_budget_bytes = fr / 2;
  }
  s.budget = (int64_t)std::min<size_t>(hbm_budget_bytes, (size_t)INT64_MAX);
  // the fixed reserve: batch buffers and the scratch of a full batch's projection
  const size_t scratch_bytes = project_scratch_need(D, mode, s.max_batch);
  s.reserve = (int64_t)(scratch_bytes + (sizeof(double) * 12 + 3 * sizeof(int64_t)) * (size_t)s.max_batch);
  if (s.reserve > s.budget)
    return set_error(DD_ERR_TOO_LARGE, "the server's fixed reserve (" + std::to_string(s.reserve) +
                                           " bytes: batch buffers and projection scratch for " +
                                           std::to_string(s.max_batch) +
                                           " states) exceeds the budget; lower max_batch");
  DD_TRY(s.bq.alloc(sizeof(double) * 12 * (size_t)s.max_batch));
  DD_TRY(s.bw.alloc(sizeof(int64_t) * (size_t)s.max_batch));
  DD_TRY(s.bi.alloc(sizeof(int64_t) * (size_t)s.max_batch));
  DD_TRY(s.bd.alloc(sizeof(double) * (size_t)s.max_batch));
  s.scratch.reset(new ScratchArena);
  DD_HIP(hipEventCreateWithFlags(&s.scratch->done, hipEventDisableTiming));
  DD_HIP(hipHostMalloc((void**)&s.scratch->pinned, sizeof(uint32_t) * kArenaPinnedWords,
                       hipHostMallocDefault));
  DD_HIP(hipMalloc(&s.scratch->block, scratch_bytes));
  s.scratch->bytes = scratch_bytes;
  s.peak_used = s.reserve;
  DD_HIP(hipStreamCreateWithFlags(&s.pst, hipStreamNonBlocking));
  s.t_create = Clock::now();
  s.sched_thr = std::thread([&s] { s.scheduler(); });
  s.proj_thr = std::thread([&s] { s.projector(); });
  *out = h.release();
  return DD_OK;
}

extern "C" dd_status dd_server_destroy(dd_server* h) {
  using namespace dd;
  if (!h) return DD_OK;
  Server& s = h->s;
  {
    std::lock_guard<std::mutex> lk(s.mu);
    s.stop = true;
  }
  s.cv_work.notify_all();
  if (s.sched_thr.joinable()) s.sched_thr.join();
  {
    std::lock_guard<std::mutex> lk(s.pmu);   // the projector re-checks its predicate
  }
  s.pcv.notify_all();
  if (s.proj_thr.joinable()) s.proj_thr.join();
  if (s.pst) (void)hipStreamDestroy(s.pst);
  delete h;
  return DD_OK;
}

extern "C" dd_status dd_server_submit(dd_server* h, const dd_solve_request* r, uint64_t* ticket) {
  using namespace dd;
  if (!h || !ticket) return set_error(DD_ERR_ARG, "server or ticket is NULL");
  Server& s = h->s;
  DD_TRY(check_request(*s.D, r));
  std::unique_ptr<Job> j(new Job());
  j->mesh = r->mesh;
  j->n_dof = 3 * (int64_t)(r->mesh.nx + 1) * (r->mesh.ny + 1) * (r->mesh.nz + 1);
  j->n_mp = 8 * (int64_t)r->mesh.nx * r->mesh.ny * r->mesh.nz;
  j->mask.assign(r->dirichlet_mask, r->dirichlet_mask + j->n_dof);
  j->force.assign(r->nodal_force, r->nodal_force + j->n_dof);
  j->init.assign(r->init_idx, r->init_idx + j->n_mp);
  j->max_iter = r->max_iter > 0 ? r->max_iter : 500;
  j->deadline_s = r->deadline_s;
  j->footprint = DDSolver::footprint_bytes(r->mesh);
  j->inv_bytes = DDSolver::inverse_bytes(r->mesh);
  {
    dd_mesh key_mesh;
    std::memset(&key_mesh, 0, sizeof(key_mesh));   // no padding bytes of the caller's struct
    key_mesh.nx = r->mesh.nx;
    key_mesh.ny = r->mesh.ny;
    key_mesh.nz = r->mesh.nz;
    key_mesh.lx = r->mesh.lx;
    key_mesh.ly = r->mesh.ly;
    key_mesh.lz = r->mesh.lz;
    j->mesh = key_mesh;
    j->inv_key.assign(reinterpret_cast<const char*>(&key_mesh), sizeof(key_mesh));
    j->inv_key.append(reinterpret_cast<const char*>(j->mask.data()), j->mask.size());
  }
  std::lock_guard<std::mutex> lk(s.mu);
  if (s.stop) return set_error(DD_ERR_CANCELLED, "server is shutting down");
  if (s.reserve + j->footprint > s.budget) {
    ++s.n_rejected;
    return set_error(DD_ERR_TOO_LARGE, "solve needs " + std::to_string(j->footprint) +
                                           " device bytes, more than the server budget " +
                                           std::to_string(s.budget));
  }
  if ((int64_t)s.queue.size() >= s.max_queue) {
    ++s.n_rejected;
    return set_error(DD_ERR_TOO_LARGE, "server queue is full");
  }
  j->ticket = s.next_ticket++;
  j->t_submit = Clock::now();
  if (!s.any_submit) {
    s.any_submit = true;
    s.t_first_submit = j->t_submit;
  }
  ++s.n_submitted;
  *ticket = j->ticket;
  s.queue.push_back(j.get());
  s.jobs[j->ticket] = std::move(j);
  s.cv_work.notify_one();
  return DD_OK;
}

extern "C" dd_status dd_server_wait(dd_server* h, uint64_t ticket, dd_solve_result* res,
                                    double timeout_s) {
  using namespace dd;
  if (!h) return set_error(DD_ERR_ARG, "server is NULL");
  Server& s = h->s;
  std::unique_lock<std::mutex> lk(s.mu);
  auto it = s.jobs.find(ticket);
  if (it == s.jobs.end()) return set_error(DD_ERR_ARG, "unknown ticket");
  Job* j = it->second.get();
  auto done = [&] { return j->done; };
  if (timeout_s < 0) {
    s.cv_done.wait(lk, done);
  } else if (!s.cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) {
    return set_error(DD_ERR_TIMEOUT, "solve not finished within the timeout");
  }
  std::unique_ptr<Job> own = std::move(it->second);
  s.jobs.erase(it);
  lk.unlock();
  if (res) {
    const int n = (int)j->d_half.size();
    const int cap = std::min(n, std::max(res->history_capacity, 0));
    if (!j->u.empty()) {
      if (res->u) std::memcpy(res->u, j->u.data(), sizeof(double) * j->u.size());
      if (res->idx) std::memcpy(res->idx, j->idx.data(), sizeof(int64_t) * j->idx.size());
      if (res->eps) std::memcpy(res->eps, j->eps.data(), sizeof(double) * j->eps.size());
      if (res->sig) std::memcpy(res->sig, j->sig.data(), sizeof(double) * j->sig.size());
    }
    for (int i = 0; i < cap; ++i) {
      if (res->d_half) res->d_half[i] = j->d_half[i];
      if (res->d_full) res->d_full[i] = j->d_full[i];
      if (res->changed) res->changed[i] = j->changed[i];
    }
    res->iterations = n;
    res->converged = j->stop_reason == 1 ? 1 : 0;
    res->stop_reason = j->stop_reason;
    res->skipped = 0;
    res->cg_iterations = j->cg_total;
    res->cg_max_residual = j->cg_res_max;
    res->elapsed_ms = ms_since(j->t_submit, j->t_done);
    res->project_ms = 0.0;
  }
  if (j->status != DD_OK) return set_error(j->status, j->error);
  return DD_OK;
}

extern "C" dd_status dd_server_cancel(dd_server* h, uint64_t ticket) {
  using namespace dd;
  if (!h) return set_error(DD_ERR_ARG, "server is NULL");
  Server& s = h->s;
  std::lock_guard<std::mutex> lk(s.mu);
  auto it = s.jobs.find(ticket);
  if (it == s.jobs.end()) return set_error(DD_ERR_ARG, "unknown ticket");
  it->second->cancel = true;
  s.cv_work.notify_one();
  return DD_OK;
}

extern "C" dd_status dd_server_stats(const dd_server* h, dd_server_statistics* out) {
  using namespace dd;
  if (!h || !out) return set_error(DD_ERR_ARG, "server or stats is NULL");
  // reading the counters takes the server's lock; nothing else changes
  Server& s = const_cast<dd_server*>(h)->s;
  std::lock_guard<std::mutex> lk(s.mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s.n_submitted;
  out->completed = s.n_completed;
  out->failed = s.n_failed;
  out->rejected = s.n_rejected;
  out->cancelled = s.n_cancelled;
  out->queued = (int64_t)s.queue.size();
  out->active = s.n_active.load();
  out->batches = s.n_batches;
  out->queries = s.n_queries;
  out->peak_active = s.peak_active;
  out->peak_bytes = s.peak_used;
  out->budget_bytes = s.budget;
  out->reserve_bytes = s.reserve;
  out->proj_p50_ms = percentile(s.lat_proj, 50);
  out->proj_p99_ms = percentile(s.lat_proj, 99);
  out->solve_p50_ms = percentile(s.lat_solve, 50);
  out->solve_p99_ms = percentile(s.lat_solve, 99);
  out->queue_p50_ms = percentile(s.lat_queue, 50);
  out->queue_p99_ms = percentile(s.lat_queue, 99);
  const double el = s.any_submit ? ms_since(s.t_first_submit, Clock::now()) / 1e3 : 0.0;
  out->elapsed_s = el;
  out->queries_per_s = el > 0 ? (double)s.n_queries / el : 0.0;
  return DD_OK;
}
