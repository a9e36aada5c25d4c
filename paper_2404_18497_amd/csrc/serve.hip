// Serving loop: resident MPHFs, build and query requests admitted under an HBM budget, several HIP
// streams in flight, continuous batching of queries (one multi-request launch) and of builds (one
// batched build).  Scheduling never changes a result: every launch and batched build produces
// exactly what the request would produce alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "phobic_internal.h"

namespace phobic {
namespace {

struct Req {
  uint64_t id = 0, mphf = 0, n = 0;
  uint32_t kind = PHOBIC_REQ_BUILD;
  const uint64_t* keys = nullptr;
  uint64_t* out = nullptr;
  uint64_t reserve = 0;  // builds: admitted memory estimate
  double submit = 0, start = 0, done = 0;
  uint32_t batch = 1;
  phobic_status status = PHOBIC_OK;
};

struct Resident {
  phobic_mphf* h = nullptr;   // null while building
  bool failed = false;
  uint64_t bytes = 0;
  uint32_t users = 0;         // queued or running queries
  bool release_pending = false;
};

uint64_t build_estimate(uint64_t n) { return 32 * n + (64ULL << 20); }

}  // namespace
}  // namespace phobic

struct phobic_server {
  phobic_server_config cfg{};
  phobic_params prm{};
  int device = 0;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable work_cv, done_cv;
  std::deque<phobic::Req*> pending;     // arrival order
  std::deque<phobic::Req*> completed;
  std::map<uint64_t, phobic::Resident> mphfs;
  uint64_t next_id = 1;
  uint64_t resident_bytes = 0, reserved_bytes = 0, peak_bytes = 0;
  uint64_t query_launches = 0, build_launches = 0, ncompleted = 0;
  uint32_t running = 0;
  bool stop = false;
  std::vector<std::thread> workers;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  void note_peak() { peak_bytes = std::max(peak_bytes, resident_bytes + reserved_bytes); }

  // Picks the next batch of work for a worker (lock held).  Queries first, in arrival order, up to
  // max_query_batch whose MPHF is ready; otherwise builds in arrival order that fit the budget,
  // unless the worker is one of the query_workers kept for queries only.
  std::vector<phobic::Req*> pick(bool queries_only) {
    std::vector<phobic::Req*> got;
    for (auto it = pending.begin(); it != pending.end() && got.size() < cfg.max_query_batch;) {
      phobic::Req* r = *it;
      if (r->kind == PHOBIC_REQ_QUERY) {
        auto m = mphfs.find(r->mphf);
        if (m != mphfs.end() && (m->second.h || m->second.failed)) {
          got.push_back(r);
          it = pending.erase(it);
          continue;
        }
      }
      ++it;
    }
    if (!got.empty() || queries_only) return got;
    for (auto it = pending.begin(); it != pending.end() && got.size() < cfg.max_build_batch;) {
      phobic::Req* r = *it;
      if (r->kind == PHOBIC_REQ_BUILD) {
        if (resident_bytes + reserved_bytes + r->reserve <= cfg.hbm_budget_bytes) {
          reserved_bytes += r->reserve;
          note_peak();
          got.push_back(r);
          it = pending.erase(it);
          continue;
        }
        break;  // builds are admitted in arrival order
      }
      ++it;
    }
    return got;
  }

  void run_queries(std::vector<phobic::Req*>& rs, hipStream_t st) {
    std::vector<const phobic_mphf*> hs;
    std::vector<const uint64_t*> ks;
    std::vector<uint64_t> ns;
    std::vector<uint64_t*> outs;
    std::vector<phobic::Req*> live;
    {
      std::lock_guard<std::mutex> lock(mu);
      for (auto r : rs) {
        auto& m = mphfs[r->mphf];
        if (!m.h) {
          r->status = PHOBIC_E_INVALID;  // its build failed
          continue;
        }
        hs.push_back(m.h);
        ks.push_back(r->keys);
        ns.push_back(r->n);
        outs.push_back(r->out);
        live.push_back(r);
      }
      query_launches++;
    }
    phobic_status s = phobic_query_multi_u64(hs.data(), ks.data(), ns.data(), outs.data(), (uint32_t)hs.size(), st);
    if (s == PHOBIC_OK && hipStreamSynchronize(st) != hipSuccess) s = PHOBIC_E_DEVICE;
    for (auto r : live) r->status = s;
  }

  void run_builds(std::vector<phobic::Req*>& rs, hipStream_t st) {
    std::vector<phobic_mphf*> made(rs.size(), nullptr);
    phobic_status s;
    if (rs.size() == 1) {
      s = phobic_build_u64(rs[0]->keys, rs[0]->n, &prm, st, &made[0]);
      rs[0]->status = s;
    } else {
      std::vector<const uint64_t*> ks;
      std::vector<uint64_t> ns;
      for (auto r : rs) {
        ks.push_back(r->keys);
        ns.push_back(r->n);
      }
      s = phobic_build_batch_u64(ks.data(), ns.data(), (uint32_t)rs.size(), &prm, st, made.data());
      if (s != PHOBIC_OK) {
        // a batch fails as a whole; build the members alone so each gets its own status
        for (size_t i = 0; i < rs.size(); i++) rs[i]->status = phobic_build_u64(ks[i], ns[i], &prm, st, &made[i]);
      } else {
        for (auto r : rs) r->status = PHOBIC_OK;
      }
    }
    std::lock_guard<std::mutex> lock(mu);
    build_launches++;
    for (size_t i = 0; i < rs.size(); i++) {
      auto& m = mphfs[rs[i]->mphf];
      reserved_bytes -= rs[i]->reserve;
      if (made[i]) {
        m.h = made[i];
        m.bytes = phobic_size_bits(made[i]) / 8;
        resident_bytes += m.bytes;
      } else {
        m.failed = true;
      }
    }
    note_peak();
  }

  void worker_main(uint32_t index) {
    const bool queries_only = index < cfg.query_workers;
    (void)hipSetDevice(device);
    hipStream_t st = nullptr;
    (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    for (;;) {
      std::vector<phobic::Req*> batch;
      {
        std::unique_lock<std::mutex> lock(mu);
        for (;;) {
          batch = pick(queries_only);
          if (!batch.empty() || (stop && pending.empty())) break;
          if (stop && queries_only) break;  // the other workers finish or fail what is left
          if (stop && running == 0) {  // shutting down and nothing can progress: fail what is left
            const double t = now();
            for (auto r : pending) {
              r->status = PHOBIC_E_OOM;
              r->start = r->done = t;
              if (r->kind == PHOBIC_REQ_QUERY && mphfs[r->mphf].users) mphfs[r->mphf].users--;
              completed.push_back(r);
              ncompleted++;
            }
            pending.clear();
            done_cv.notify_all();
            break;
          }
          work_cv.wait(lock);
        }
        if (batch.empty()) break;
        running++;
        const double t = now();
        for (auto r : batch) {
          r->start = t;
          r->batch = (uint32_t)batch.size();
        }
      }
      if (batch[0]->kind == PHOBIC_REQ_QUERY)
        run_queries(batch, st);
      else
        run_builds(batch, st);
      {
        std::lock_guard<std::mutex> lock(mu);
        const double t = now();
        for (auto r : batch) {
          r->done = t;
          if (r->kind == PHOBIC_REQ_QUERY) {
            auto& m = mphfs[r->mphf];
            if (m.users) m.users--;
            if (m.release_pending && m.users == 0) free_resident(r->mphf);
          }
          completed.push_back(r);
          ncompleted++;
        }
        running--;
      }
      work_cv.notify_all();
      done_cv.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
  }

  void free_resident(uint64_t id) {  // lock held
    auto it = mphfs.find(id);
    if (it == mphfs.end()) return;
    if (it->second.h) {
      resident_bytes -= it->second.bytes;
      phobic_free(it->second.h);
    }
    mphfs.erase(it);
  }
};

using namespace phobic;

extern "C" phobic_status phobic_server_create(const phobic_server_config* cfg, const phobic_params* params,
                                              phobic_server** out) {
  if (!out || !cfg || !params) return fail(PHOBIC_E_INVALID, "null argument");
  *out = nullptr;
  uint32_t B;
  phobic_status vs = validate_params(params, &B);
  if (vs != PHOBIC_OK) return vs;
  if (cfg->workers < 1 || cfg->workers > 64 || cfg->max_query_batch < 1 || cfg->max_build_batch < 1 ||
      cfg->hbm_budget_bytes == 0 || cfg->query_workers >= cfg->workers)
    return fail(PHOBIC_E_INVALID,
                "workers in [1, 64], query_workers < workers, batches >= 1 and a nonzero budget are required");
  auto s = new (std::nothrow) phobic_server();
  if (!s) return fail(PHOBIC_E_OOM, "host allocation");
  s->cfg = *cfg;
  s->prm = *params;
  s->prm.flags &= ~PHOBIC_FLAG_KEEP_PILOTS;
  s->t0 = std::chrono::steady_clock::now();
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(PHOBIC_E_DEVICE, "no HIP device");
  }
  for (uint32_t w = 0; w < cfg->workers; w++) s->workers.emplace_back([s, w] { s->worker_main(w); });
  *out = s;
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_server_submit_build(phobic_server* s, const uint64_t* d_keys, uint64_t n,
                                                    uint64_t* request_id) {
  if (!s || !request_id || (n && !d_keys)) return fail(PHOBIC_E_INVALID, "null argument");
  auto r = new Req();
  r->kind = PHOBIC_REQ_BUILD;
  r->keys = d_keys;
  r->n = n;
  r->reserve = build_estimate(n);
  {
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) {
      delete r;
      return fail(PHOBIC_E_INVALID, "server is shutting down");
    }
    r->id = r->mphf = s->next_id++;
    r->submit = s->now();
    *request_id = r->id;
    s->mphfs[r->id] = Resident{};
    if (r->reserve > s->cfg.hbm_budget_bytes) {  // can never be admitted
      r->status = PHOBIC_E_OOM;
      r->start = r->done = r->submit;
      s->mphfs[r->id].failed = true;
      s->completed.push_back(r);
      s->ncompleted++;
      s->done_cv.notify_all();
      return PHOBIC_OK;
    }
    s->pending.push_back(r);
  }
  s->work_cv.notify_all();
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_server_submit_query(phobic_server* s, uint64_t mphf_id, const uint64_t* d_keys,
                                                    uint64_t n, uint64_t* d_pos, uint64_t* request_id) {
  if (!s || !request_id || (n && (!d_keys || !d_pos))) return fail(PHOBIC_E_INVALID, "null argument");
  auto r = new Req();
  r->kind = PHOBIC_REQ_QUERY;
  r->mphf = mphf_id;
  r->keys = d_keys;
  r->out = d_pos;
  r->n = n;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    auto m = s->mphfs.find(mphf_id);
    if (s->stop || m == s->mphfs.end() || m->second.release_pending) {
      delete r;
      return fail(PHOBIC_E_INVALID, "unknown or released MPHF " + std::to_string(mphf_id));
    }
    if (m->second.failed) {
      delete r;
      return fail(PHOBIC_E_INVALID, "the build of MPHF " + std::to_string(mphf_id) + " failed");
    }
    m->second.users++;
    r->id = s->next_id++;
    r->submit = s->now();
    *request_id = r->id;
    s->pending.push_back(r);
  }
  s->work_cv.notify_all();
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_server_poll(phobic_server* s, phobic_request_result* out, uint32_t cap, uint32_t* got,
                                            uint32_t wait_ms) {
  if (!s || !got || (cap && !out)) return fail(PHOBIC_E_INVALID, "null argument");
  *got = 0;
  std::unique_lock<std::mutex> lock(s->mu);
  if (s->completed.empty() && wait_ms)
    s->done_cv.wait_for(lock, std::chrono::milliseconds(wait_ms), [s] { return !s->completed.empty(); });
  while (*got < cap && !s->completed.empty()) {
    Req* r = s->completed.front();
    s->completed.pop_front();
    phobic_request_result& o = out[(*got)++];
    o.request_id = r->id;
    o.mphf_id = r->mphf;
    o.n = r->n;
    o.status = r->status;
    o.kind = r->kind;
    o.batch = r->batch;
    o.reserved = 0;
    o.submit_s = r->submit;
    o.start_s = r->start;
    o.done_s = r->done;
    delete r;
  }
  return PHOBIC_OK;
}

extern "C" const phobic_mphf* phobic_server_mphf(phobic_server* s, uint64_t mphf_id) {
  if (!s) return nullptr;
  std::lock_guard<std::mutex> lock(s->mu);
  auto m = s->mphfs.find(mphf_id);
  return m == s->mphfs.end() ? nullptr : m->second.h;
}

extern "C" phobic_status phobic_server_release(phobic_server* s, uint64_t mphf_id) {
  if (!s) return fail(PHOBIC_E_INVALID, "null server");
  std::lock_guard<std::mutex> lock(s->mu);
  auto m = s->mphfs.find(mphf_id);
  if (m == s->mphfs.end()) return fail(PHOBIC_E_INVALID, "unknown MPHF " + std::to_string(mphf_id));
  if (!m->second.h && !m->second.failed) return fail(PHOBIC_E_INVALID, "MPHF is still being built");
  if (m->second.users) {
    m->second.release_pending = true;
    return PHOBIC_OK;
  }
  s->free_resident(mphf_id);
  return PHOBIC_OK;
}

extern "C" phobic_status phobic_server_get_stats(phobic_server* s, phobic_server_stats* out) {
  if (!s || !out) return fail(PHOBIC_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lock(s->mu);
  uint64_t res = 0;
  for (auto& kv : s->mphfs) res += kv.second.h ? 1 : 0;
  out->resident_mphfs = res;
  out->resident_bytes = s->resident_bytes;
  out->reserved_bytes = s->reserved_bytes;
  out->peak_bytes = s->peak_bytes;
  out->query_launches = s->query_launches;
  out->build_launches = s->build_launches;
  out->completed = s->ncompleted;
  out->pending = s->pending.size() + s->running;
  return PHOBIC_OK;
}

extern "C" double phobic_server_now(phobic_server* s) { return s ? s->now() : 0.0; }

extern "C" void phobic_server_destroy(phobic_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lock(s->mu);
    s->stop = true;
  }
  s->work_cv.notify_all();
  for (auto& t : s->workers) t.join();
  for (auto r : s->completed) delete r;
  for (auto& kv : s->mphfs)
    if (kv.second.h) phobic_free(kv.second.h);
  delete s;
}
