// Continuous-batching server for PNK solves on one GPU (include/pnkcc.h,
// "Serving").
//
// max_slots worker threads each own a HIP stream. The scheduler
// (scheduler.hpp) admits queued requests as workers free up and their
// footprints fit in the unused budget; the worker copies the problem to the
// device, solves it on its own stream (so kernels of different requests
// overlap on the GPU) and releases the problem's memory. All device memory
// of a request is allocated and freed stream-ordered on the worker's stream,
// so admitting or retiring one request never synchronises the others.
//
// Finished requests leave their handle (engine with its workspace and
// recorded HIP graphs, solver with its Krylov bases) in a cache keyed by
// shape and precision. A later request of the same key takes it over
// instead of allocating and recording again. Cached handles count against
// the memory budget; when a queued request does not fit, the least recently
// used ones are freed first.

#include <chrono>
#include <cstring>
#include <list>
#include <mutex>
#include <thread>

#include "../../include/pnkcc.h"
#include "api_internal.hpp"
#include "scheduler.hpp"

using namespace pnk;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// One request: its host inputs until the solve has consumed them, then its
// results until they are collected.
struct Job {
  int o = 0, v = 0, naux = 0;
  std::vector<double> f_oo, f_ov, f_vv, L;
  cc_pnk_opts opts;
  cc_info info{};
  std::vector<double> t1, t2;
  std::string err;
  size_t host_bytes() const {
    return sizeof(double) * (f_oo.capacity() + f_ov.capacity() + f_vv.capacity() + L.capacity() + t1.capacity() +
                             t2.capacity());
  }
  void drop_inputs() {
    std::vector<double>().swap(f_oo);
    std::vector<double>().swap(f_ov);
    std::vector<double>().swap(f_vv);
    std::vector<double>().swap(L);
  }
};

struct CachedHandle {
  int o = 0, v = 0, naux = 0, lowp = 0;
  size_t bytes = 0;
  std::unique_ptr<Handle> h;
};

}  // namespace

struct cc_server {
  int device = 0;
  int max_slots = 1;
  double t0 = 0;
  std::unique_ptr<Scheduler<Job>> sched;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  std::mutex cache_mu;
  std::list<CachedHandle> cache;  // most recently used first
  size_t cached_bytes = 0;
  uint64_t reuses = 0;
};

namespace {

size_t request_footprint(int o, int v, int naux, const cc_pnk_opts& op) {
  const int lowp = lowp_for(op.jvp_prec);
  const size_t n = (size_t)o + v;
  const size_t problem = sizeof(double) * ((size_t)o * o + (size_t)o * v + (size_t)v * v + (size_t)naux * n * n);
  return workspace_bytes(o, v, naux, lowp, op.m_max, op.inner_restart, 0) + problem + (1u << 20);
}

// Bytes a handle keeps between requests (its engine, solver and vectors).
size_t handle_bytes(const Handle& H) {
  if (!H.eng) return 0;
  const int lp = (H.eng->options().lowp_f32 ? 1 : 0) | (H.eng->options().lowp_bf16 ? 2 : 0);
  return workspace_bytes(H.eng->o(), H.eng->v(), H.eng->naux(), lp, H.sol_m, H.sol_r, H.sol_d, H.sol_cap);
}

std::unique_ptr<Handle> take_cached(cc_server* S, int o, int v, int naux, int lowp, size_t* bytes) {
  std::lock_guard<std::mutex> lk(S->cache_mu);
  for (auto it = S->cache.begin(); it != S->cache.end(); ++it) {
    if (it->o == o && it->v == v && it->naux == naux && it->lowp == lowp) {
      std::unique_ptr<Handle> h = std::move(it->h);
      *bytes = it->bytes;
      S->cached_bytes -= it->bytes;
      S->cache.erase(it);
      ++S->reuses;
      return h;
    }
  }
  return nullptr;
}

// Free the least recently used cached handle; false when none is left.
bool evict_one(cc_server* S) {
  CachedHandle victim;
  {
    std::lock_guard<std::mutex> lk(S->cache_mu);
    if (S->cache.empty()) return false;
    victim = std::move(S->cache.back());
    S->cache.pop_back();
    S->cached_bytes -= victim.bytes;
  }
  victim.h.reset();  // stream-ordered frees on the stream it last ran on
  S->sched->unhold(victim.bytes);
  return true;
}

void worker_main(cc_server* S, int slot) {
  (void)hipSetDevice(S->device);
  hipStream_t stream = S->streams[slot];
  while (Scheduler<Job>::Entry* E = S->sched->take([S] { return evict_one(S); })) {
    Job& R = *E->payload;
    const int lowp = lowp_for(R.opts.jvp_prec);
    size_t cached = 0;
    std::unique_ptr<Handle> Hp = take_cached(S, R.o, R.v, R.naux, lowp, &cached);
    if (Hp) {
      // its memory is part of this request's footprint from here on
      S->sched->unhold(cached);
    } else {
      Hp = std::make_unique<Handle>();
      Hp->device = S->device;
    }
    Handle& H = *Hp;
    H.alloc_stream = stream;
    H.stream_ordered = true;
    cc_status st = CC_OK;
    double *d_oo = nullptr, *d_ov = nullptr, *d_vv = nullptr, *d_L = nullptr, *d_t1 = nullptr, *d_t2 = nullptr;
    const int64_t ov = (int64_t)R.o * R.v, n2 = ov * ov;
    try {
      d_oo = (double*)H.dev_alloc(R.f_oo.size() * sizeof(double));
      d_ov = (double*)H.dev_alloc(R.f_ov.size() * sizeof(double));
      d_vv = (double*)H.dev_alloc(R.f_vv.size() * sizeof(double));
      d_L = (double*)H.dev_alloc(R.L.size() * sizeof(double));
      d_t1 = (double*)H.dev_alloc(ov * sizeof(double));
      d_t2 = (double*)H.dev_alloc(n2 * sizeof(double));
      PNK_HIP(hipMemcpyAsync(d_oo, R.f_oo.data(), R.f_oo.size() * 8, hipMemcpyHostToDevice, stream));
      PNK_HIP(hipMemcpyAsync(d_ov, R.f_ov.data(), R.f_ov.size() * 8, hipMemcpyHostToDevice, stream));
      PNK_HIP(hipMemcpyAsync(d_vv, R.f_vv.data(), R.f_vv.size() * 8, hipMemcpyHostToDevice, stream));
      PNK_HIP(hipMemcpyAsync(d_L, R.L.data(), R.L.size() * 8, hipMemcpyHostToDevice, stream));
      cc_problem p{R.o, R.v, R.naux, d_oo, d_ov, d_vv, d_L};
      st = cc_solve_pnk(reinterpret_cast<cc_handle*>(&H), &p, &R.opts, d_t1, d_t2, &R.info, stream);
      if (st == CC_OK || st == CC_NOT_CONVERGED || st == CC_ERR_NAN) {
        R.t1.resize(ov);
        R.t2.resize(n2);
        PNK_HIP(hipMemcpyAsync(R.t1.data(), d_t1, ov * 8, hipMemcpyDeviceToHost, stream));
        PNK_HIP(hipMemcpyAsync(R.t2.data(), d_t2, n2 * 8, hipMemcpyDeviceToHost, stream));
      }
      R.err = H.err;
    } catch (const std::exception& e) {
      R.err = e.what();
      st = CC_ERR_HIP;
    }
    for (double* p : {d_oo, d_ov, d_vv, d_L, d_t1, d_t2}) H.dev_free(p);
    (void)hipStreamSynchronize(stream);  // results on the host, inputs consumed
    size_t keep = 0;
    const size_t hb = handle_bytes(H);
    if ((st == CC_OK || st == CC_NOT_CONVERGED || st == CC_ERR_NAN) && hb <= E->footprint) {
      keep = hb;
      std::lock_guard<std::mutex> lk(S->cache_mu);
      CachedHandle c;
      c.o = R.o; c.v = R.v; c.naux = R.naux; c.lowp = lowp;
      c.bytes = keep;
      c.h = std::move(Hp);
      S->cache.push_front(std::move(c));
      S->cached_bytes += keep;
    } else {
      Hp.reset();  // a failed handle is not reused
      (void)hipStreamSynchronize(stream);
    }
    S->sched->complete(E, (int)st, [](Job& j) { j.drop_inputs(); }, keep);
  }
}

}  // namespace

extern "C" {

cc_status cc_server_create(cc_server** out, int device, size_t mem_budget, int max_slots) {
  if (!out || max_slots < 1 || max_slots > 64) return CC_ERR_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
    (void)hipGetLastError();
    return CC_ERR_HIP;
  }
  if (hipSetDevice(device) != hipSuccess) return CC_ERR_HIP;
  if (mem_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return CC_ERR_HIP;
    mem_budget = (size_t)(0.9 * (double)fr);
  }
  // keep freed stream-ordered memory cached in the pool
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  (void)hipGetLastError();
  cc_server* S = new (std::nothrow) cc_server();
  if (!S) return CC_ERR_OOM;
  S->device = device;
  S->max_slots = max_slots;
  S->t0 = now_s();
  const double t0 = S->t0;
  // a request can be passed over by smaller ones at most twice per slot
  S->sched = std::make_unique<Scheduler<Job>>(
      mem_budget, 2 * max_slots, [t0] { return now_s() - t0; }, [](const Job& j) { return j.host_bytes(); });
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
      delete S;
      return CC_ERR_HIP;
    }
    S->streams.push_back(st);
  }
  for (int i = 0; i < max_slots; ++i) S->workers.emplace_back(worker_main, S, i);
  *out = S;
  return CC_OK;
}

cc_status cc_server_submit(cc_server* S, const cc_problem* p, const cc_pnk_opts* opts, uint64_t* req_id) {
  if (!S || !p || !req_id) return CC_ERR_ARG;
  try {
    check_problem(p);
    cc_pnk_opts o;
    cc_pnk_opts_default(&o);
    if (opts) o = *opts;
    check_pnk_opts(o);
    auto R = std::make_unique<Job>();
    R->o = p->nocc;
    R->v = p->nvir;
    R->naux = p->naux;
    R->opts = o;
    const size_t n = (size_t)R->o + R->v;
    const size_t footprint = request_footprint(R->o, R->v, R->naux, o);
    R->f_oo.assign(p->f_oo, p->f_oo + (size_t)R->o * R->o);
    R->f_ov.assign(p->f_ov, p->f_ov + (size_t)R->o * R->v);
    R->f_vv.assign(p->f_vv, p->f_vv + (size_t)R->v * R->v);
    R->L.assign(p->L, p->L + (size_t)R->naux * n * n);
    if (!S->sched->submit(std::move(R), footprint, req_id)) return CC_ERR_REJECTED;
  } catch (const ArgError&) {
    return CC_ERR_ARG;
  } catch (const std::bad_alloc&) {
    return CC_ERR_OOM;
  }
  return CC_OK;
}

cc_status cc_server_poll(cc_server* S, uint64_t req_id, int* done, cc_info* info, double* t1_host, double* t2_host) {
  if (!S || !done) return CC_ERR_ARG;
  int status = CC_OK;
  const int r = S->sched->release(req_id, [&](Scheduler<Job>::Entry& e) {
    const Job& R = *e.payload;
    if (info) *info = R.info;
    if (t1_host && !R.t1.empty()) std::memcpy(t1_host, R.t1.data(), R.t1.size() * 8);
    if (t2_host && !R.t2.empty()) std::memcpy(t2_host, R.t2.data(), R.t2.size() * 8);
    status = e.status;
  });
  if (r < 0) return CC_ERR_ARG;
  *done = r;
  return r ? (cc_status)status : CC_OK;
}

cc_status cc_server_drain(cc_server* S) {
  if (!S) return CC_ERR_ARG;
  S->sched->drain();
  return CC_OK;
}

cc_status cc_server_get_stats(cc_server* S, cc_server_stats* st) {
  if (!S || !st) return CC_ERR_ARG;
  const auto s = S->sched->stats();
  st->queued = s.queued;
  st->running = s.running;
  st->finished = s.finished;
  st->rejected = s.rejected;
  st->bytes_in_use = s.bytes_in_use;
  st->peak_bytes = s.peak_bytes;
  st->budget = s.budget;
  st->max_slots = S->max_slots;
  st->peak_running = s.peak_running;
  st->host_bytes_held = s.held_payload_bytes;
  st->requests_held = s.entries;
  std::lock_guard<std::mutex> lk(S->cache_mu);
  st->cached_bytes = S->cached_bytes;
  st->cached_handles = S->cache.size();
  st->handle_reuses = S->reuses;
  return CC_OK;
}

cc_status cc_server_request_times(cc_server* S, uint64_t req_id, double* t_submit, double* t_admit,
                                  double* t_finish) {
  if (!S) return CC_ERR_ARG;
  Scheduler<Job>::Times t;
  if (!S->sched->times(req_id, &t)) return CC_ERR_ARG;
  if (t_submit) *t_submit = t.t_submit;
  if (t_admit) *t_admit = t.t_admit;
  if (t_finish) *t_finish = t.t_finish;
  return CC_OK;
}

void cc_server_destroy(cc_server* S) {
  if (!S) return;
  S->sched->stop();
  for (auto& t : S->workers) t.join();
  {
    std::lock_guard<std::mutex> lk(S->cache_mu);
    S->cache.clear();  // stream-ordered frees on the workers' streams
  }
  for (hipStream_t st : S->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  delete S;
}

}  // extern "C"
