// Serving loop for scan jobs: continuous batching of whole PIC runs on one
// device.  Built only on the public C ABI (pic_create / pic_load_tables /
// pic_step_many / pic_emission_stats / pic_destroy) plus hipMemGetInfo.
//
// Jobs wait in a FIFO.  Each scheduling round
//   1. admits waiting jobs, in arrival order, while a resident slot is free
//      and the device reports enough free memory for the job's context
//      (pic_memory_required) on top of the configured reserve;
//   2. advances every resident job by up to quantum_steps steps in one
//      pic_step_many call (per step, one batched launch of each kernel of the
//      step covers every resident job; uneven jobs simply drop out of the
//      later steps of the round);
//   3. waits for the device, retires the jobs that reached their step count
//      (statistics read back, context freed unless kept) and stamps their
//      completion time.
// A job's particles, fields and photons stay on the device from admission to
// retirement.  Its result does not depend on the other jobs in the round:
// every chunk and field node is updated exactly as pic_step would.
#include <chrono>
#include <cstddef>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>
#include <hip/hip_runtime.h>
#include "../../include/pic.h"

namespace {

struct Job {
  uint64_t id = 0;
  pic_config cfg{};
  int32_t nsteps = 0;
  int32_t done = 0;
  pic_tables t{};
  bool has_tables = false;
  std::vector<double> h, lnxi, ncs, sig, br;
  double t_submit = 0, t_admit = -1, t_finish = -1;
  uint64_t bytes = 0;
  pic_ctx* ctx = nullptr;
  int32_t status = PIC_OK;
  pic_stats stats{};
};

double now_s(const std::chrono::steady_clock::time_point& t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct pic_server {
  pic_server_config sc{};
  std::chrono::steady_clock::time_point t0;
  pic_batch* batch = nullptr;
  std::mutex mu;                              // guards queue, err, next_id
  std::deque<std::unique_ptr<Job>> queue;     // waiting, arrival order
  std::vector<std::unique_ptr<Job>> resident; // on the device
  std::vector<std::unique_ptr<Job>> done;     // finished, not yet polled
  std::vector<std::unique_ptr<Job>> kept;     // polled, context kept for read-back
  uint64_t next_id = 1;
  std::string err;
  ~pic_server() {
    for (auto& j : resident) pic_destroy(j->ctx);
    for (auto& j : done) pic_destroy(j->ctx);
    for (auto& j : kept) pic_destroy(j->ctx);
    pic_batch_destroy(batch);
  }
};

namespace {

void retire(pic_server* s, std::unique_ptr<Job>& j, int32_t status) {
  j->t_finish = now_s(s->t0);
  if (j->ctx) {
    pic_stats st{};
    const pic_status r = pic_emission_stats(j->ctx, &st);
    if (r == PIC_OK || r == PIC_ERR_OVERFLOW) j->stats = st;
    if (status == PIC_OK) status = r;
    if (!s->sc.keep_finished) {
      pic_destroy(j->ctx);
      j->ctx = nullptr;
    }
  }
  j->status = status;
  s->done.push_back(std::move(j));
}

// Admission: FIFO, while a slot is free and the job fits the free memory.
void admit(pic_server* s) {
  for (;;) {
    std::unique_ptr<Job> j;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->queue.empty() || (int32_t)s->resident.size() >= s->sc.max_jobs) return;
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) return;
      Job& head = *s->queue.front();
      const uint64_t need = head.bytes + s->sc.hbm_reserve_bytes;
      if (need > (uint64_t)tot) {  // can never fit: fail it now
        j = std::move(s->queue.front());
        s->queue.pop_front();
        j->t_admit = now_s(s->t0);
        retire(s, j, PIC_ERR_NOMEM);
        continue;
      }
      if (need > (uint64_t)fr) return;  // wait for running jobs to free memory
      j = std::move(s->queue.front());
      s->queue.pop_front();
    }
    j->cfg.stream = s->sc.stream;
    j->t_admit = now_s(s->t0);
    pic_status r = pic_create(&j->cfg, &j->ctx);
    if (r == PIC_ERR_NOMEM && !s->resident.empty()) {  // fragmentation: retry after a retirement
      std::lock_guard<std::mutex> lk(s->mu);
      j->t_admit = -1;
      s->queue.push_front(std::move(j));
      return;
    }
    if (r == PIC_OK && j->has_tables) r = pic_load_tables(j->ctx, &j->t);
    if (r != PIC_OK) {
      retire(s, j, r);
      continue;
    }
    j->h.clear(); j->lnxi.clear(); j->ncs.clear(); j->sig.clear(); j->br.clear();
    j->h.shrink_to_fit(); j->lnxi.shrink_to_fit(); j->ncs.shrink_to_fit();
    j->sig.shrink_to_fit(); j->br.shrink_to_fit();
    s->resident.push_back(std::move(j));
  }
}

}  // namespace

extern "C" {

pic_status pic_device_memory(uint64_t* free_bytes, uint64_t* total_bytes) {
  if (!free_bytes || !total_bytes) return PIC_ERR_INVALID;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return PIC_ERR_DEVICE;
  *free_bytes = fr;
  *total_bytes = tot;
  return PIC_OK;
}

pic_status pic_server_create(const pic_server_config* sc, pic_server** out) {
  if (!sc || !out) return PIC_ERR_INVALID;
  *out = nullptr;
  if (sc->abi_version != PIC_ABI_VERSION || sc->max_jobs < 1 || sc->quantum_steps < 1 ||
      sc->keep_finished > 1)
    return PIC_ERR_INVALID;
  pic_server* s = new (std::nothrow) pic_server;
  if (!s) return PIC_ERR_NOMEM;
  s->sc = *sc;
  s->t0 = std::chrono::steady_clock::now();
  const pic_status r = pic_batch_create(sc->stream, &s->batch);
  if (r != PIC_OK) {
    delete s;
    return r;
  }
  *out = s;
  return PIC_OK;
}

void pic_server_destroy(pic_server* s) { delete s; }

double pic_server_clock(const pic_server* s) { return s ? now_s(s->t0) : 0.0; }

const char* pic_server_last_error(const pic_server* s) { return s ? s->err.c_str() : ""; }

pic_status pic_server_submit(pic_server* s, const pic_config* cfg, const pic_tables* t,
                             int32_t nsteps, double t_arrival, uint64_t* job) {
  if (!s || !cfg || !job || nsteps < 0) return PIC_ERR_INVALID;
  if (cfg->flags & (PIC_BW | PIC_BH)) {  // a job carries emission tables only
    std::lock_guard<std::mutex> lk(s->mu);
    s->err = "pair production is not served (jobs carry no pair tables)";
    return PIC_ERR_INVALID;
  }
  std::unique_ptr<Job> j(new (std::nothrow) Job);
  if (!j) return PIC_ERR_NOMEM;
  j->cfg = *cfg;
  j->nsteps = nsteps;
  const pic_status r = pic_memory_required(cfg, &j->bytes);
  if (r != PIC_OK) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->err = pic_last_error(nullptr);
    return r;
  }
  if (t) {  // deep copy: the caller may free its arrays on return
    if (t->n_eta < 1 || t->n_xi < 1 || t->n_T < 1 || t->n_y < 1 || !t->h || !t->ln_xi ||
        !t->ncs_cdf || !t->sigma || !t->br_cdf)
      return PIC_ERR_TABLES;
    j->t = *t;
    j->h.assign(t->h, t->h + t->n_eta);
    j->lnxi.assign(t->ln_xi, t->ln_xi + t->n_xi);
    j->ncs.assign(t->ncs_cdf, t->ncs_cdf + (size_t)t->n_eta * t->n_xi);
    j->sig.assign(t->sigma, t->sigma + t->n_T);
    j->br.assign(t->br_cdf, t->br_cdf + (size_t)t->n_T * t->n_y);
    j->t.h = j->h.data();
    j->t.ln_xi = j->lnxi.data();
    j->t.ncs_cdf = j->ncs.data();
    j->t.sigma = j->sig.data();
    j->t.br_cdf = j->br.data();
    j->has_tables = true;
  }
  j->t_submit = t_arrival >= 0.0 ? t_arrival : now_s(s->t0);
  std::lock_guard<std::mutex> lk(s->mu);
  j->id = s->next_id++;
  *job = j->id;
  s->queue.push_back(std::move(j));
  return PIC_OK;
}

pic_status pic_server_run(pic_server* s, int32_t* resident, int32_t* queued) {
  if (!s) return PIC_ERR_INVALID;
  admit(s);
  pic_status ret = PIC_OK;
  if (!s->resident.empty()) {
    std::vector<pic_ctx*> ctxs;
    std::vector<int32_t> steps;
    for (auto& j : s->resident) {
      ctxs.push_back(j->ctx);
      const int32_t left = j->nsteps - j->done;
      steps.push_back(left < s->sc.quantum_steps ? left : s->sc.quantum_steps);
    }
    pic_status r = pic_step_many(s->batch, ctxs.data(), steps.data(), (int32_t)ctxs.size());
    if (r == PIC_OK) {
      const hipError_t e = hipStreamSynchronize((hipStream_t)s->sc.stream);
      if (e != hipSuccess) r = PIC_ERR_DEVICE;
    }
    if (r != PIC_OK) {
      s->err = pic_batch_last_error(s->batch);
      ret = r;
      // a failed round leaves every resident run in an unknown state
      for (auto& j : s->resident) retire(s, j, r);
      s->resident.clear();
    } else {
      std::vector<std::unique_ptr<Job>> still;
      for (size_t k = 0; k < s->resident.size(); ++k) {
        std::unique_ptr<Job>& j = s->resident[k];
        j->done += steps[k];
        if (j->done >= j->nsteps) retire(s, j, PIC_OK);
        else still.push_back(std::move(j));
      }
      s->resident.swap(still);
    }
  }
  if (resident) *resident = (int32_t)s->resident.size();
  if (queued) {
    std::lock_guard<std::mutex> lk(s->mu);
    *queued = (int32_t)s->queue.size();
  }
  return ret;
}

pic_status pic_server_poll(pic_server* s, pic_job_result* out, int32_t max, int32_t* n) {
  if (!s || !n || max < 0 || (max > 0 && !out)) return PIC_ERR_INVALID;
  int32_t k = 0;
  std::vector<std::unique_ptr<Job>> rest;
  for (auto& j : s->done) {
    if (k >= max) {
      rest.push_back(std::move(j));
      continue;
    }
    pic_job_result r{};
    r.job = j->id;
    r.status = j->status;
    r.steps = j->nsteps;
    r.t_submit = j->t_submit;
    r.t_admit = j->t_admit;
    r.t_finish = j->t_finish;
    r.device_bytes = j->bytes;
    r.stats = j->stats;
    out[k++] = r;
    if (j->ctx) s->kept.push_back(std::move(j));
  }
  s->done.swap(rest);
  *n = k;
  return PIC_OK;
}

pic_status pic_server_job_ctx(pic_server* s, uint64_t job, pic_ctx** ctx) {
  if (!s || !ctx) return PIC_ERR_INVALID;
  for (auto& j : s->kept)
    if (j->id == job) {
      *ctx = j->ctx;
      return PIC_OK;
    }
  for (auto& j : s->done)
    if (j->id == job && j->ctx) {
      *ctx = j->ctx;
      return PIC_OK;
    }
  return PIC_ERR_STATE;
}

pic_status pic_server_release(pic_server* s, uint64_t job) {
  if (!s) return PIC_ERR_INVALID;
  for (size_t k = 0; k < s->kept.size(); ++k)
    if (s->kept[k]->id == job) {
      pic_destroy(s->kept[k]->ctx);
      s->kept.erase(s->kept.begin() + (std::ptrdiff_t)k);
      return PIC_OK;
    }
  for (auto& j : s->done)
    if (j->id == job && j->ctx) {
      pic_destroy(j->ctx);
      j->ctx = nullptr;
      return PIC_OK;
    }
  return PIC_ERR_STATE;
}

}  // extern "C"
