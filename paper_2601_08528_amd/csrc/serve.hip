// Serving runtime: a host dispatcher thread that keeps the index on the
// device and runs a stream of search / insert / delete requests of uneven
// sizes with continuous batching (the real-time coordination of SVFusion,
// Sec. 4.4: several search streams plus one update stream, queries of varying
// batch size running concurrently).
//
//  - Search requests are coalesced in arrival order into device batches of
//    up to max_batch queries (requests with the same k and beam share a
//    batch); each batch runs on one of `streams` search streams with its own
//    device and pinned buffers, so batches admitted while others are on the
//    GPU overlap with them.  A batch is admitted when a stream slot is free
//    and its buffers fit in the HBM budget; buffers are released when the
//    batch retires.
//  - Mutations are applied one at a time in arrival order on the update
//    stream.  An insert is prepared (vectors stored beyond n_slots, batched
//    search, forward prune, reverse-edge prune into staged rows) by a worker
//    thread while search batches keep running, because preparation only reads
//    what searches read; its commit waits for in-flight search batches to
//    retire, writes the rows and alive bits, and advances the epoch.  A
//    delete (bitset marks and repair) runs with no search batch in flight.
//  - A search sees the epoch committed when its batch was launched: exactly
//    the state a search issued alone at that moment would see, so results
//    are independent of the other requests in the mix.  To read its own
//    writes a client waits for the insert's ticket before searching.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "index_internal.hpp"

using Clock = std::chrono::steady_clock;

namespace svf {

struct ServeReq {
  uint64_t ticket = 0;
  int kind = 0;  // 0 search, 1 insert, 2 delete
  int64_t n = 0;
  int k = 0, beam = 0;
  std::vector<float> vin;
  std::vector<int32_t> iin;
  int32_t* out_ids = nullptr;
  float* out_d = nullptr;
  Clock::time_point t_submit, t_launch, t_done;
  int status = 1;  // 1 pending, else an SVF status
  int64_t epoch = 0, batch_q = 0;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  int64_t cap = 0;           // queries the buffers hold
  int k = 0;
  size_t bytes = 0;          // device bytes charged to the budget
  float* hq = nullptr;       // pinned staging
  int32_t* hid = nullptr;
  float* hd = nullptr;
  float* dq = nullptr;       // device
  int32_t* did = nullptr;
  float* dd = nullptr;
  uint64_t* dkey = nullptr;
  std::vector<ServeReq*> reqs;
  int64_t nq = 0;
  int bk = 0;                // k of the batch in flight (row length of the outputs)
};

struct Server {
  svf_index* ix = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_submit, cv_done;
  std::deque<ServeReq*> searches, mutations;
  std::unordered_map<uint64_t, std::unique_ptr<ServeReq>> reqs;
  bool stopping = false;
  uint64_t next_ticket = 1;
  std::vector<Slot> slots;
  int64_t max_batch = 0;
  int64_t budget = 0, in_use = 0;
  int64_t epoch = 0;
  // insert in preparation
  std::thread worker;
  std::atomic<int> prep_state{0};  // 0 idle, 1 running, 2 prepared
  int prep_rc = 0;
  svf_detail::PendingInsert pend;
  ServeReq* prep_req = nullptr;
  int64_t prep_done = 0;           // vectors of prep_req already committed
  float* prep_dev = nullptr;       // device copy of the request's vectors
};

namespace {

size_t slot_bytes(const svf_index* ix, int64_t nq, int k) {
  return (size_t)nq * ((size_t)ix->dim * 4 + (size_t)k * 8 + 8) + 4096;
}

void free_slot_buffers(Slot& s) {
  if (s.hq) (void)hipHostFree(s.hq);
  if (s.hid) (void)hipHostFree(s.hid);
  if (s.hd) (void)hipHostFree(s.hd);
  if (s.dq) (void)hipFree(s.dq);
  if (s.did) (void)hipFree(s.did);
  if (s.dd) (void)hipFree(s.dd);
  if (s.dkey) (void)hipFree(s.dkey);
  s.hq = nullptr; s.hid = nullptr; s.hd = nullptr;
  s.dq = nullptr; s.did = nullptr; s.dd = nullptr; s.dkey = nullptr;
  s.cap = 0;
  s.k = 0;
}

// Buffers for nq queries of k results (kept between batches, regrown on demand).
hipError_t size_slot(const svf_index* ix, Slot& s, int64_t nq, int k) {
  if (nq <= s.cap && k <= s.k) return hipSuccess;
  free_slot_buffers(s);
  const int64_t c = nq;
  const int kk = k;
  hipError_t e;
  if ((e = hipHostMalloc((void**)&s.hq, c * ix->dim * 4, 0)) != hipSuccess) return e;
  if ((e = hipHostMalloc((void**)&s.hid, c * kk * 4, 0)) != hipSuccess) return e;
  if ((e = hipHostMalloc((void**)&s.hd, c * kk * 4, 0)) != hipSuccess) return e;
  if ((e = hipMalloc(&s.dq, c * ix->dim * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&s.did, c * kk * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&s.dd, c * kk * 4)) != hipSuccess) return e;
  if ((e = hipMalloc(&s.dkey, c * 8)) != hipSuccess) return e;
  s.cap = c;
  s.k = kk;
  return hipSuccess;
}

void finish(Server* sv, ServeReq* r, int status) {
  r->status = status;
  r->t_done = Clock::now();
  if (r->kind != 0) r->epoch = sv->epoch;   // a search keeps its launch epoch
}

// Retire finished search batches (caller holds sv->mu).  A batch still
// running is not an error: its status must not stay behind as the thread's
// last HIP error.  A batch whose stream failed ends its requests with
// SVF_E_DEVICE instead of waiting for ever.
void retire(Server* sv) {
  for (Slot& s : sv->slots) {
    if (!s.busy) continue;
    const hipError_t q = hipEventQuery(s.ev);
    if (q == hipErrorNotReady) {
      (void)hipGetLastError();
      continue;
    }
    const int status = q == hipSuccess ? SVF_OK : SVF_E_DEVICE;
    int64_t off = 0;
    for (ServeReq* r : s.reqs) {
      if (status == SVF_OK) {
        std::memcpy(r->out_ids, s.hid + off * s.bk, (size_t)r->n * r->k * 4);
        std::memcpy(r->out_d, s.hd + off * s.bk, (size_t)r->n * r->k * 4);
      }
      off += r->n;
      finish(sv, r, status);
    }
    s.reqs.clear();
    s.busy = false;
    sv->in_use -= (int64_t)s.bytes;
    s.bytes = 0;
    sv->cv_done.notify_all();
  }
}

bool any_busy(const Server* sv) {
  for (const Slot& s : sv->slots)
    if (s.busy) return true;
  return false;
}

// Launch one coalesced batch from the head of the search queue, if a slot and
// the budget allow.  Returns true when something was launched.
bool launch_batch(Server* sv) {
  if (sv->searches.empty()) return false;
  Slot* slot = nullptr;
  for (Slot& s : sv->slots)
    if (!s.busy) { slot = &s; break; }
  if (!slot) return false;
  svf_index* ix = sv->ix;
  ServeReq* head = sv->searches.front();
  // coalesce consecutive requests with the same k and beam
  std::vector<ServeReq*> take;
  int64_t nq = 0;
  for (ServeReq* r : sv->searches) {
    if (r->k != head->k || r->beam != head->beam) break;
    if (!take.empty() && nq + r->n > sv->max_batch) break;
    take.push_back(r);
    nq += r->n;
  }
  const size_t bytes = slot_bytes(ix, nq, head->k);
  if ((int64_t)bytes > sv->budget) {      // can never fit: refuse the head
    sv->searches.pop_front();
    finish(sv, head, SVF_E_NOMEM);
    sv->cv_done.notify_all();
    return true;
  }
  if (sv->in_use + (int64_t)bytes > sv->budget) return false;   // wait for memory
  if (size_slot(ix, *slot, nq, head->k) != hipSuccess) {
    sv->searches.pop_front();
    finish(sv, head, SVF_E_NOMEM);
    sv->cv_done.notify_all();
    return true;
  }
  for (size_t i = 0; i < take.size(); ++i) sv->searches.pop_front();
  int64_t off = 0;
  const auto now = Clock::now();
  for (ServeReq* r : take) {
    std::memcpy(slot->hq + off * ix->dim, r->vin.data(), (size_t)r->n * ix->dim * 4);
    off += r->n;
    r->t_launch = now;
    r->batch_q = nq;
    r->epoch = sv->epoch;
  }
  const int k = head->k;
  hipStream_t st = slot->st;
  bool ok = hipMemcpyAsync(slot->dq, slot->hq, nq * ix->dim * 4, hipMemcpyHostToDevice, st) == hipSuccess;
  if (ix->n_slots == 0) {
    ok = ok && svf::launch_fill_u32(slot->did, nq * k, 0xffffffffu, st) == hipSuccess;
    ok = ok && svf::launch_fill_u32(slot->dd, nq * k, 0x7f800000u, st) == hipSuccess;
  } else {
    svf::SearchArgs a = svf_detail::base_args(ix);
    svf_detail::set_beam(a, ix, head->beam);
    a.k = k;
    a.queries = slot->dq;
    a.qstride = ix->dim;
    a.nq = (int)nq;
    a.out_ids = slot->did;
    a.out_d = slot->dd;
    ok = ok && svf::launch_query_keys(slot->dq, ix->dim, nullptr, ix->dim, a.nq, ix->opt.seed,
                                      slot->dkey, st) == hipSuccess;
    a.qkey = slot->dkey;
    ok = ok && svf::launch_search(a, ix->veclp_prec, st) == hipSuccess;
  }
  ok = ok && hipMemcpyAsync(slot->hid, slot->did, nq * k * 4, hipMemcpyDeviceToHost, st) == hipSuccess;
  ok = ok && hipMemcpyAsync(slot->hd, slot->dd, nq * k * 4, hipMemcpyDeviceToHost, st) == hipSuccess;
  ok = ok && hipEventRecord(slot->ev, st) == hipSuccess;
  if (!ok) {
    for (ServeReq* r : take) finish(sv, r, SVF_E_DEVICE);
    sv->cv_done.notify_all();
    return true;
  }
  slot->reqs = std::move(take);
  slot->nq = nq;
  slot->bk = k;
  slot->busy = true;
  slot->bytes = bytes;
  sv->in_use += (int64_t)bytes;
  return true;
}

// Wait (dropping the lock) until no search batch is in flight.
void drain(Server* sv, std::unique_lock<std::mutex>& lk) {
  while (any_busy(sv)) {
    lk.unlock();
    for (Slot& s : sv->slots)
      if (s.busy) (void)hipEventSynchronize(s.ev);
    lk.lock();
    retire(sv);
  }
}

void start_prepare(Server* sv) {
  ServeReq* r = sv->prep_req;
  svf_index* ix = sv->ix;
  const int64_t b = std::min<int64_t>(ix->opt.insert_batch_max, r->n - sv->prep_done);
  const float* src = sv->prep_dev + sv->prep_done * ix->dim;
  sv->prep_state = 1;
  if (sv->worker.joinable()) sv->worker.join();
  sv->worker = std::thread([sv, src, b]() {
    sv->prep_rc = svf_detail::insert_prepare(sv->ix, src, b, &sv->pend);
    sv->prep_state = 2;
    sv->cv_submit.notify_all();
  });
}

// Begin the mutation at the head of the mutation queue (caller holds mu).
void begin_mutation(Server* sv, std::unique_lock<std::mutex>& lk) {
  ServeReq* r = sv->mutations.front();
  svf_index* ix = sv->ix;
  if (r->kind == 2) {                      // delete: exclusive
    sv->mutations.pop_front();
    drain(sv, lk);
    r->t_launch = Clock::now();
    const int rc = svf_detail::delete_ids(ix, r->iin.data(), r->n);
    if (rc == SVF_OK) ++sv->epoch;
    finish(sv, r, rc);
    sv->cv_done.notify_all();
    return;
  }
  // insert: grow capacity with no search in flight, then prepare beside them
  sv->mutations.pop_front();
  r->t_launch = Clock::now();
  if (ix->n_slots == 0 || ix->n_slots + r->n > ix->cap) {
    drain(sv, lk);
    int rc = svf_detail::reserve(ix, ix->n_slots + r->n + (ix->n_slots + r->n) / 2);
    if (rc) { finish(sv, r, rc); sv->cv_done.notify_all(); return; }
  }
  if (sv->prep_dev) (void)hipFree(sv->prep_dev);
  sv->prep_dev = nullptr;
  if (hipMalloc(&sv->prep_dev, (size_t)r->n * ix->dim * 4) != hipSuccess ||
      hipMemcpy(sv->prep_dev, r->vin.data(), (size_t)r->n * ix->dim * 4, hipMemcpyHostToDevice) != hipSuccess) {
    finish(sv, r, SVF_E_NOMEM);
    sv->cv_done.notify_all();
    return;
  }
  sv->prep_req = r;
  sv->prep_done = 0;
  if (ix->n_slots == 0) {
    // an empty index builds exclusively (seed rule, then growing batches)
    drain(sv, lk);
    int rc = SVF_OK;
    int64_t done = 0;
    while (rc == SVF_OK && done < r->n) {
      int64_t b = ix->n_slots == 0 ? std::min<int64_t>(r->n, 4 * ix->R)
                                   : std::min<int64_t>({(int64_t)ix->opt.insert_batch_max, r->n - done,
                                                        (ix->n_alive + 7) / 8});
      svf_detail::PendingInsert p;
      rc = svf_detail::insert_prepare(ix, sv->prep_dev + done * ix->dim, b, &p);
      if (rc == SVF_OK) rc = svf_detail::insert_commit(ix, &p);
      done += b;
    }
    if (rc == SVF_OK) {
      for (int64_t i = 0; i < r->n; ++i) r->out_ids[i] = (int32_t)i;
      ++sv->epoch;
    }
    finish(sv, r, rc);
    sv->prep_req = nullptr;
    sv->cv_done.notify_all();
    return;
  }
  start_prepare(sv);
}

// A prepared insert batch: fence, commit, continue or finish (caller holds mu).
void commit_prepared(Server* sv, std::unique_lock<std::mutex>& lk) {
  if (sv->worker.joinable()) sv->worker.join();
  ServeReq* r = sv->prep_req;
  svf_index* ix = sv->ix;
  int rc = sv->prep_rc;
  if (rc == SVF_OK) {
    drain(sv, lk);
    rc = svf_detail::insert_commit(ix, &sv->pend);
  }
  sv->prep_state = 0;
  if (rc == SVF_OK) {
    for (int64_t i = 0; i < sv->pend.b; ++i)
      r->out_ids[sv->prep_done + i] = (int32_t)(sv->pend.n0 + i);
    sv->prep_done += sv->pend.b;
    ++sv->epoch;
    if (sv->prep_done < r->n) {
      start_prepare(sv);
      return;
    }
  }
  finish(sv, r, rc);
  sv->prep_req = nullptr;
  sv->cv_done.notify_all();
}

void dispatcher(Server* sv) {
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    retire(sv);
    bool progressed = false;
    if (sv->prep_state == 2) {
      commit_prepared(sv, lk);
      progressed = true;
    }
    if (sv->prep_state == 0 && !sv->prep_req && sv->ix->bg.active && sv->ix->bg.done) {
      // a background consolidation has finished: merge it like a commit
      drain(sv, lk);
      if (svf_detail::bg_merge(sv->ix) == SVF_OK) ++sv->epoch;
      progressed = true;
    }
    if (sv->prep_state == 0 && !sv->prep_req && !sv->mutations.empty()) {
      begin_mutation(sv, lk);
      progressed = true;
    }
    while (launch_batch(sv)) progressed = true;
    const bool idle = sv->searches.empty() && sv->mutations.empty() && !any_busy(sv) &&
                      sv->prep_state == 0 && !sv->prep_req;
    if (sv->stopping && idle) break;
    if (progressed) continue;
    if (any_busy(sv) || sv->prep_state == 1) {
      // poll the device without holding the lock
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      sv->cv_submit.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
  if (sv->worker.joinable()) sv->worker.join();
}

int submit(svf_index* ix, std::unique_ptr<ServeReq> r, uint64_t* ticket) {
  Server* sv = ix->server;
  if (!sv) return svf_detail::fail(SVF_E_BUSY, "the serving loop is not running");
  std::lock_guard<std::mutex> g(sv->mu);
  if (sv->stopping) return svf_detail::fail(SVF_E_BUSY, "the serving loop is stopping");
  r->ticket = sv->next_ticket++;
  r->t_submit = Clock::now();
  ServeReq* p = r.get();
  if (ticket) *ticket = p->ticket;
  sv->reqs.emplace(p->ticket, std::move(r));
  if (p->kind == 0) sv->searches.push_back(p);
  else sv->mutations.push_back(p);
  sv->cv_submit.notify_all();
  return SVF_OK;
}

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace
}  // namespace svf

using svf_detail::fail;

void svf_detail::serve_shutdown(svf_index* ix) {
  svf::Server* sv = ix->server;
  if (!sv) return;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stopping = true;
    sv->cv_submit.notify_all();
  }
  if (sv->th.joinable()) sv->th.join();
  for (svf::Slot& s : sv->slots) {
    if (s.st) (void)hipStreamSynchronize(s.st);
    svf::free_slot_buffers(s);
    if (s.ev) (void)hipEventDestroy(s.ev);
    if (s.st) (void)hipStreamDestroy(s.st);
  }
  if (sv->prep_dev) (void)hipFree(sv->prep_dev);
  ix->server = nullptr;
  delete sv;
}

extern "C" {

int svf_serve_start(svf_index* ix, int32_t streams, int64_t max_batch, int64_t hbm_budget) {
  if (!ix) return fail(SVF_E_INVAL, "null index");
  if (streams < 1 || streams > 16) return fail(SVF_E_INVAL, "streams in [1, 16]");
  if (max_batch < 1 || max_batch > (1 << 20)) return fail(SVF_E_INVAL, "max_batch in [1, 2^20]");
  if (hbm_budget < 0) return fail(SVF_E_INVAL, "hbm_budget >= 0");
  std::lock_guard<std::mutex> g(ix->mu);
  if (ix->server) return fail(SVF_E_BUSY, "already serving");
  if (ix->opt.use_model) return fail(SVF_E_INVAL, "serving runs the plain or reduced-precision form");
  auto* sv = new (std::nothrow) svf::Server();
  if (!sv) return fail(SVF_E_NOMEM, "host allocation");
  sv->ix = ix;
  sv->max_batch = max_batch;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
  const int64_t avail = (int64_t)(free_b * 0.8);
  sv->budget = hbm_budget > 0 ? std::min<int64_t>(hbm_budget, avail > 0 ? avail : hbm_budget) : avail;
  sv->slots.resize(streams);
  for (svf::Slot& s : sv->slots) {
    if (hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.ev, hipEventDisableTiming) != hipSuccess) {
      ix->server = sv;
      svf_detail::serve_shutdown(ix);
      return fail(SVF_E_DEVICE, "stream setup");
    }
  }
  ix->server = sv;
  sv->th = std::thread(svf::dispatcher, sv);
  return SVF_OK;
}

int svf_serve_stop(svf_index* ix) {
  if (!ix) return fail(SVF_E_INVAL, "null index");
  if (!ix->server) return fail(SVF_E_BUSY, "not serving");
  svf_detail::serve_shutdown(ix);
  return SVF_OK;
}

int svf_submit_search(svf_index* ix, const float* queries, int64_t nq, int32_t k, int32_t beam,
                      int32_t* out_ids, float* out_dists, uint64_t* ticket) {
  int rc = svf_detail::check_search_args(ix, nq, k, beam);
  if (rc) return rc;
  if (nq < 1 || !queries || !out_ids || !out_dists) return fail(SVF_E_INVAL, "bad buffer");
  if (!svf_detail::all_finite(queries, nq * ix->dim)) return fail(SVF_E_INVAL, "non-finite query value");
  auto r = std::make_unique<svf::ServeReq>();
  r->kind = 0;
  r->n = nq;
  r->k = k;
  r->beam = beam;
  r->vin.assign(queries, queries + nq * ix->dim);
  r->out_ids = out_ids;
  r->out_d = out_dists;
  return svf::submit(ix, std::move(r), ticket);
}

int svf_submit_insert(svf_index* ix, const float* vecs, int64_t n, int32_t* out_ids, uint64_t* ticket) {
  if (!ix || n < 1 || !vecs || !out_ids) return fail(SVF_E_INVAL, "bad argument");
  if (!svf_detail::all_finite(vecs, n * ix->dim)) return fail(SVF_E_INVAL, "non-finite vector value");
  auto r = std::make_unique<svf::ServeReq>();
  r->kind = 1;
  r->n = n;
  r->vin.assign(vecs, vecs + n * ix->dim);
  r->out_ids = out_ids;
  return svf::submit(ix, std::move(r), ticket);
}

int svf_submit_delete(svf_index* ix, const int32_t* ids, int64_t n, uint64_t* ticket) {
  if (!ix || n < 1 || !ids) return fail(SVF_E_INVAL, "bad argument");
  auto r = std::make_unique<svf::ServeReq>();
  r->kind = 2;
  r->n = n;
  r->iin.assign(ids, ids + n);
  return svf::submit(ix, std::move(r), ticket);
}

int svf_wait(svf_index* ix, uint64_t ticket, double timeout_s, svf_request_info* info) {
  if (!ix) return fail(SVF_E_INVAL, "null index");
  svf::Server* sv = ix->server;
  if (!sv) return fail(SVF_E_BUSY, "not serving");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(SVF_E_NOTFOUND, "unknown ticket");
  svf::ServeReq* r = it->second.get();
  const auto deadline = Clock::now() + std::chrono::duration<double>(timeout_s);
  while (r->status == 1) {
    if (timeout_s >= 0 && Clock::now() >= deadline) return fail(SVF_E_BUSY, "timed out");
    sv->cv_done.wait_for(lk, std::chrono::milliseconds(2));
  }
  const int st = r->status;
  if (info) {
    info->status = st;
    info->queue_ms = svf::ms_between(r->t_submit, r->t_launch);
    info->total_ms = svf::ms_between(r->t_submit, r->t_done);
    info->batch_queries = r->batch_q;
    info->epoch = r->epoch;
  }
  sv->reqs.erase(it);
  if (st != SVF_OK) return fail(st, "request failed");
  return SVF_OK;
}

}  // extern "C"
