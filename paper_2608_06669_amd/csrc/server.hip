// Continuous-batching server for PNK solves on one GPU (include/pnkcc.h,
// "Serving").
//
// max_slots worker threads each own a HIP stream. The scheduler admits the
// oldest queued request as soon as a worker is idle and the request's
// footprint fits in the unused budget; the worker copies the problem to the
// device, solves it on its own stream (so kernels of different requests
// overlap on the GPU) and releases the memory. All device memory of a
// request is allocated and freed stream-ordered on the worker's stream, so
// admitting or retiring one request never synchronises the others.

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "../../include/pnkcc.h"
#include "api_internal.hpp"

using namespace pnk;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t id = 0;
  int o = 0, v = 0, naux = 0;
  std::vector<double> f_oo, f_ov, f_vv, L;
  cc_pnk_opts opts;
  size_t footprint = 0;
  enum State { Queued, Running, Done } state = Queued;
  cc_status status = CC_OK;
  cc_info info{};
  std::vector<double> t1, t2;
  double t_submit = 0, t_admit = 0, t_finish = 0;
  std::string err;
};

}  // namespace

struct cc_server {
  int device = 0;
  size_t budget = 0;
  int max_slots = 1;
  double t0 = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_id = 1;
  size_t in_use = 0, peak = 0;
  int running = 0, peak_running = 0;
  uint64_t finished = 0, rejected = 0;
  bool stop = false;
  std::vector<std::thread> workers;
};

namespace {

size_t request_footprint(int o, int v, int naux, const cc_pnk_opts& op) {
  const int lowp = op.jvp_prec == CC_FP32 ? 1 : (op.jvp_prec == CC_BF16 ? 2 : 0);
  const size_t n = (size_t)o + v;
  const size_t problem = sizeof(double) * ((size_t)o * o + (size_t)o * v + (size_t)v * v + (size_t)naux * n * n);
  return workspace_bytes(o, v, naux, lowp, op.m_max, op.inner_restart, 0) + problem + (1u << 20);
}

void worker_main(cc_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t stream = nullptr;
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) return;
  while (true) {
    Request* R = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] {
        if (S->stop) return true;
        if (S->queue.empty()) return false;
        const Request* head = S->reqs[S->queue.front()].get();
        return S->in_use + head->footprint <= S->budget;
      });
      if (S->stop) break;
      R = S->reqs[S->queue.front()].get();
      S->queue.pop_front();
      S->in_use += R->footprint;
      S->peak = std::max(S->peak, S->in_use);
      ++S->running;
      S->peak_running = std::max(S->peak_running, S->running);
      R->state = Request::Running;
      R->t_admit = now_s() - S->t0;
    }
    // solve on this worker's stream
    auto Hp = std::make_unique<Handle>();
    Handle& H = *Hp;
    H.device = S->device;
    H.alloc_stream = stream;
    H.stream_ordered = true;
    cc_status st = CC_OK;
    double *d_oo = nullptr, *d_ov = nullptr, *d_vv = nullptr, *d_L = nullptr, *d_t1 = nullptr, *d_t2 = nullptr;
    const int64_t ov = (int64_t)R->o * R->v, n2 = ov * ov;
    try {
      d_oo = (double*)H.dev_alloc(R->f_oo.size() * sizeof(double));
      d_ov = (double*)H.dev_alloc(R->f_ov.size() * sizeof(double));
      d_vv = (double*)H.dev_alloc(R->f_vv.size() * sizeof(double));
      d_L = (double*)H.dev_alloc(R->L.size() * sizeof(double));
      d_t1 = (double*)H.dev_alloc(ov * sizeof(double));
      d_t2 = (double*)H.dev_alloc(n2 * sizeof(double));
      PNK_HIP(hipMemcpyAsync(d_oo, R->f_oo.data(), R->f_oo.size() * 8, hipMemcpyHostToDevice, stream));
      PNK_HIP(hipMemcpyAsync(d_ov, R->f_ov.data(), R->f_ov.size() * 8, hipMemcpyHostToDevice, stream));
      PNK_HIP(hipMemcpyAsync(d_vv, R->f_vv.data(), R->f_vv.size() * 8, hipMemcpyHostToDevice, stream));
      PNK_HIP(hipMemcpyAsync(d_L, R->L.data(), R->L.size() * 8, hipMemcpyHostToDevice, stream));
      cc_problem p{R->o, R->v, R->naux, d_oo, d_ov, d_vv, d_L};
      st = cc_solve_pnk(reinterpret_cast<cc_handle*>(&H), &p, &R->opts, d_t1, d_t2, &R->info, stream);
      if (st == CC_OK || st == CC_NOT_CONVERGED || st == CC_ERR_NAN) {
        R->t1.resize(ov);
        R->t2.resize(n2);
        PNK_HIP(hipMemcpyAsync(R->t1.data(), d_t1, ov * 8, hipMemcpyDeviceToHost, stream));
        PNK_HIP(hipMemcpyAsync(R->t2.data(), d_t2, n2 * 8, hipMemcpyDeviceToHost, stream));
      }
      R->err = H.err;
    } catch (const std::exception& e) {
      R->err = e.what();
      st = CC_ERR_HIP;
    }
    for (double* p : {d_oo, d_ov, d_vv, d_L, d_t1, d_t2}) H.dev_free(p);
    Hp.reset();  // stream-ordered release of the workspace
    (void)hipStreamSynchronize(stream);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      R->status = st;
      R->state = Request::Done;
      R->t_finish = now_s() - S->t0;
      S->in_use -= R->footprint;
      --S->running;
      ++S->finished;
    }
    S->cv.notify_all();
  }
  (void)hipStreamDestroy(stream);
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
  S->budget = mem_budget;
  S->max_slots = max_slots;
  S->t0 = now_s();
  for (int i = 0; i < max_slots; ++i) S->workers.emplace_back(worker_main, S);
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
    auto R = std::make_unique<Request>();
    R->o = p->nocc;
    R->v = p->nvir;
    R->naux = p->naux;
    R->opts = o;
    const size_t n = (size_t)R->o + R->v;
    R->f_oo.assign(p->f_oo, p->f_oo + (size_t)R->o * R->o);
    R->f_ov.assign(p->f_ov, p->f_ov + (size_t)R->o * R->v);
    R->f_vv.assign(p->f_vv, p->f_vv + (size_t)R->v * R->v);
    R->L.assign(p->L, p->L + (size_t)R->naux * n * n);
    R->footprint = request_footprint(R->o, R->v, R->naux, o);
    std::lock_guard<std::mutex> lk(S->mu);
    if (R->footprint > S->budget) {
      ++S->rejected;
      return CC_ERR_REJECTED;
    }
    R->id = S->next_id++;
    R->t_submit = now_s() - S->t0;
    *req_id = R->id;
    S->queue.push_back(R->id);
    S->reqs[R->id] = std::move(R);
  } catch (const ArgError&) {
    return CC_ERR_ARG;
  } catch (const std::bad_alloc&) {
    return CC_ERR_OOM;
  }
  S->cv.notify_all();
  return CC_OK;
}

cc_status cc_server_poll(cc_server* S, uint64_t req_id, int* done, cc_info* info, double* t1_host, double* t2_host) {
  if (!S || !done) return CC_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(req_id);
  if (it == S->reqs.end()) return CC_ERR_ARG;
  Request* R = it->second.get();
  *done = R->state == Request::Done;
  if (!*done) return CC_OK;
  if (info) *info = R->info;
  if (t1_host && !R->t1.empty()) std::memcpy(t1_host, R->t1.data(), R->t1.size() * 8);
  if (t2_host && !R->t2.empty()) std::memcpy(t2_host, R->t2.data(), R->t2.size() * 8);
  R->t1.clear();
  R->t1.shrink_to_fit();
  R->t2.clear();
  R->t2.shrink_to_fit();
  return R->status;
}

cc_status cc_server_drain(cc_server* S) {
  if (!S) return CC_ERR_ARG;
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv.wait(lk, [&] { return S->queue.empty() && S->running == 0; });
  return CC_OK;
}

cc_status cc_server_get_stats(cc_server* S, cc_server_stats* st) {
  if (!S || !st) return CC_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  st->queued = S->queue.size();
  st->running = (uint64_t)S->running;
  st->finished = S->finished;
  st->rejected = S->rejected;
  st->bytes_in_use = S->in_use;
  st->peak_bytes = S->peak;
  st->budget = S->budget;
  st->max_slots = S->max_slots;
  st->peak_running = S->peak_running;
  return CC_OK;
}

cc_status cc_server_request_times(cc_server* S, uint64_t req_id, double* t_submit, double* t_admit,
                                  double* t_finish) {
  if (!S) return CC_ERR_ARG;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(req_id);
  if (it == S->reqs.end()) return CC_ERR_ARG;
  if (t_submit) *t_submit = it->second->t_submit;
  if (t_admit) *t_admit = it->second->t_admit;
  if (t_finish) *t_finish = it->second->t_finish;
  return CC_OK;
}

void cc_server_destroy(cc_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  for (auto& t : S->workers) t.join();
  delete S;
}

}  // extern "C"
