// Serving loop: independent ground-state requests (each an EARCG solve of
// its own crystal) are admitted while the sum of their estimated device
// footprints stays within a budget and a slot is free; each admitted request
// runs on its own HIP stream from its own host thread, so the kernels of
// different requests overlap on the GPU, and it keeps its frames, density,
// directions and Krylov blocks resident until it finishes.  A finished
// request frees its memory and slot, which admits the next queued request
// that fits (requests are taken in arrival order, a large one does not block
// smaller ones behind it).  Each request's result depends only on its own
// inputs: no reduction crosses requests.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "ops.h"

using namespace eahp;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  eahp_system_desc desc{};
  std::vector<double> frac, Z, kfrac, kweight, sym_trans;
  std::vector<int> sym_rot;
  eahp_solve_params prm{};
  std::vector<z64> psi;  // initial frame, then the result
  size_t est = 0;
  int state = 0;  // 0 queued, 1 running, 2 done, 3 failed
  int status = EAHP_OK;
  std::string err;
  eahp_stats stats{};
  double t_submit = 0, t_start = 0, t_done = 0;
};

}  // namespace

struct eahp_server {
  int device = 0;
  size_t budget = 0;
  int max_slots = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<uint64_t, Request*> all;
  size_t used = 0;
  int active = 0;
  uint64_t next = 1;
  bool stop = false;
  std::thread sched;
  // one joinable thread per admitted request; a finished request puts its
  // ticket into `finished` and the scheduler joins the thread (outside the
  // lock), so no request thread outlives wait_all or destroy
  std::map<uint64_t, std::thread> workers;
  std::vector<uint64_t> finished;
};

namespace {

void run_request(eahp_server* sv, Request* rq) {
  int rc = EAHP_OK;
  std::string err;
  hipStream_t st = nullptr;
  eahp_ctx* ctx = nullptr;
  eahp_problem* pb = nullptr;
  void* dpsi = nullptr;
  const size_t fb = sizeof(z64) * rq->psi.size();
  auto check = [&](int r) {
    if (r != EAHP_OK && rc == EAHP_OK) {
      rc = r;
      err = eahp_last_error();
    }
    return r == EAHP_OK || r == EAHP_ENOCONV;
  };
  if (hipSetDevice(sv->device) != hipSuccess || hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
    rc = EAHP_EDEVICE;
    err = "stream creation failed";
  }
  if (rc == EAHP_OK && check(eahp_ctx_create(sv->device, st, &ctx)) && check(eahp_problem_create(ctx, &rq->desc, &pb))) {
    if (hipMalloc(&dpsi, fb) != hipSuccess || hipMemcpyAsync(dpsi, rq->psi.data(), fb, hipMemcpyHostToDevice, st) !=
                                                  hipSuccess) {
      rc = EAHP_ENOMEM;
      err = "frame allocation failed";
    } else {
      const int r = eahp_solve(pb, dpsi, &rq->prm, &rq->stats);
      if (r != EAHP_OK && r != EAHP_ENOCONV) check(r);
      else rq->status = r;
      if (rc == EAHP_OK &&
          (hipMemcpyAsync(rq->psi.data(), dpsi, fb, hipMemcpyDeviceToHost, st) != hipSuccess ||
           hipStreamSynchronize(st) != hipSuccess)) {
        rc = EAHP_EDEVICE;
        err = "result copy failed";
      }
    }
  }
  if (st) (void)hipStreamSynchronize(st);
  if (dpsi) (void)hipFree(dpsi);
  if (pb) eahp_problem_destroy(pb);
  if (ctx) eahp_ctx_destroy(ctx);
  if (st) (void)hipStreamDestroy(st);
  std::lock_guard<std::mutex> lk(sv->mu);
  rq->t_done = now_s();
  sv->finished.push_back(rq->ticket);
  if (rc != EAHP_OK) {
    rq->status = rc;
    rq->err = err;
    rq->state = 3;
  } else {
    rq->state = 2;
  }
  sv->used -= rq->est;
  --sv->active;
  sv->cv.notify_all();
}

void scheduler(eahp_server* sv) {
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    // join the threads of finished requests (they may still be releasing the
    // lock and their per-thread state), without holding the lock
    if (!sv->finished.empty()) {
      std::vector<std::thread> done;
      for (uint64_t id : sv->finished) {
        auto it = sv->workers.find(id);
        if (it != sv->workers.end()) {
          done.push_back(std::move(it->second));
          sv->workers.erase(it);
        }
      }
      sv->finished.clear();
      lk.unlock();
      for (auto& t : done) t.join();
      lk.lock();
      sv->cv.notify_all();
      continue;
    }
    // admit the first queued request that fits
    Request* pick = nullptr;
    if (sv->active < sv->max_slots) {
      for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it)
        if (sv->used + (*it)->est <= sv->budget || sv->active == 0) {
          pick = *it;
          sv->queue.erase(it);
          break;
        }
    }
    if (pick) {
      pick->state = 1;
      pick->t_start = now_s();
      sv->used += pick->est;
      ++sv->active;
      sv->workers.emplace(pick->ticket, std::thread(run_request, sv, pick));
      continue;
    }
    if (sv->stop && sv->queue.empty() && sv->active == 0 && sv->workers.empty()) return;
    sv->cv.wait(lk);
  }
}

}  // namespace

extern "C" {

int eahp_layout_estimate(const eahp_system_desc* desc, int64_t* npw_per_k, int fft[3], int64_t* bytes) {
  try {
    std::vector<int64_t> npw;
    int n[3], ns;
    size_t b;
    layout_estimate(desc, npw, n, ns, b);
    if (npw_per_k) std::copy(npw.begin(), npw.end(), npw_per_k);
    if (fft) std::copy(n, n + 3, fft);
    if (bytes) *bytes = (int64_t)b;
    return EAHP_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.status;
  } catch (...) {
    g_last_error = "layout estimate failed";
    return EAHP_EINVAL;
  }
}

int eahp_server_create(int device, size_t hbm_budget, int max_slots, eahp_server** out) {
  if (!out || max_slots < 1 || hbm_budget == 0) return EAHP_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return EAHP_EINVAL;
  auto* sv = new eahp_server;
  sv->device = device;
  sv->budget = hbm_budget;
  sv->max_slots = max_slots;
  sv->sched = std::thread(scheduler, sv);
  *out = sv;
  return EAHP_OK;
}

int eahp_server_submit(eahp_server* sv, const eahp_system_desc* desc, const eahp_solve_params* prm,
                       const void* psi0_host, uint64_t* ticket) {
  if (!sv || !desc || !prm || !psi0_host || !ticket) return EAHP_EINVAL;
  auto* rq = new Request;
  try {
    rq->desc = *desc;
    rq->frac.assign(desc->frac, desc->frac + 3 * desc->natoms);
    rq->Z.assign(desc->Z, desc->Z + desc->natoms);
    rq->kfrac.assign(desc->kfrac, desc->kfrac + 3 * desc->nk);
    rq->kweight.assign(desc->kweight, desc->kweight + desc->nk);
    rq->desc.frac = rq->frac.data();
    rq->desc.Z = rq->Z.data();
    rq->desc.kfrac = rq->kfrac.data();
    rq->desc.kweight = rq->kweight.data();
    if (desc->nsym > 1 && desc->sym_rot && desc->sym_trans) {
      rq->sym_rot.assign(desc->sym_rot, desc->sym_rot + 9 * (size_t)desc->nsym);
      rq->sym_trans.assign(desc->sym_trans, desc->sym_trans + 3 * (size_t)desc->nsym);
      rq->desc.sym_rot = rq->sym_rot.data();
      rq->desc.sym_trans = rq->sym_trans.data();
    }
    rq->prm = *prm;
    std::vector<int64_t> npw;
    int n[3], ns;
    layout_estimate(&rq->desc, npw, n, ns, rq->est);
    int64_t ntot = 0;
    for (int64_t v : npw) ntot += v;
    rq->psi.resize((size_t)ntot * desc->p);
    std::memcpy(rq->psi.data(), psi0_host, sizeof(z64) * rq->psi.size());
  } catch (const Error& e) {
    g_last_error = e.msg;
    delete rq;
    return e.status;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  rq->ticket = sv->next++;
  rq->t_submit = now_s();
  sv->all[rq->ticket] = rq;
  sv->queue.push_back(rq);
  *ticket = rq->ticket;
  sv->cv.notify_all();
  return EAHP_OK;
}

int eahp_server_poll(eahp_server* sv, uint64_t ticket, int* state, eahp_stats* stats, double* latency_s,
                     double* queued_s) {
  if (!sv) return EAHP_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return EAHP_EINVAL;
  Request* rq = it->second;
  if (state) *state = rq->state;
  if (rq->state >= 2) {
    if (stats) *stats = rq->stats;
    if (latency_s) *latency_s = rq->t_done - rq->t_submit;
    if (queued_s) *queued_s = rq->t_start - rq->t_submit;
    if (rq->state == 3) g_last_error = rq->err;
    return rq->status;
  }
  return EAHP_OK;
}

int eahp_server_result(eahp_server* sv, uint64_t ticket, void* psi_host) {
  if (!sv || !psi_host) return EAHP_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end() || it->second->state < 2) return EAHP_EINVAL;
  Request* rq = it->second;
  if (rq->state == 3) {
    g_last_error = rq->err;
    return rq->status;
  }
  std::memcpy(psi_host, rq->psi.data(), sizeof(z64) * rq->psi.size());
  delete rq;
  sv->all.erase(it);
  return EAHP_OK;
}

int eahp_server_wait_all(eahp_server* sv) {
  if (!sv) return EAHP_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  // also until the scheduler has joined every finished request's thread
  sv->cv.wait(lk, [&] { return sv->queue.empty() && sv->active == 0 && sv->workers.empty(); });
  return EAHP_OK;
}

void eahp_server_destroy(eahp_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv.notify_all();
  }
  sv->sched.join();
  for (auto& kv : sv->all) delete kv.second;
  delete sv;
}

}  // extern "C"
