// Serving runtime: a native request loop for private-inference linear operators.
//
// Clients submit matmul_cp requests (their own keys, a registered weight matrix, encrypted
// inputs resident in HBM, caller-owned output buffers).  A worker thread owns the context:
//   - admission: a request is admitted when the plan (diagonal plaintexts of its weight at
//     its padded length L') is resident or can be generated within the plan-cache budget;
//     least-recently-used plans that no admitted request uses are evicted to make room;
//     requests are taken in arrival order, or (policy 1) those whose plan is resident first,
//     then the oldest together with every queued request on the plan generated for it, with
//     a request older than max_wait_ms always first;
//   - continuous batching: every admitted request joins the next batch; a batch runs as one
//     blb_batch_matmul_cp (plus per-request mask-and-share) on one of several streams, so
//     requests that arrive while earlier batches are on the GPU are admitted and launched
//     while those batches still run;
//   - completion is detected with events; latency = completion - submission (host clock).
// Results do not depend on the batch a request lands in (exact modular arithmetic).
#include <hip/hip_runtime.h>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "blb_internal.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Weights {
  std::vector<double> W;
  double* W_dev = nullptr;  // device copy (plans are generated from it without a host copy)
  int d_in = 0, d_out = 0, level = 0;
  int cplx = 0;  // complex-slot output packing (two column blocks per output ciphertext)
};

struct PlanEntry {
  blb_plan* plan = nullptr;
  size_t bytes = 0;
  size_t off = 0;  // position in the plan arena
  int users = 0;   // admitted requests (and the generation itself while pending)
  double last_use = 0;
  bool pending = false;  // generation enqueued, not yet complete
  hipEvent_t ready = nullptr;
};

// First-fit allocator over one device allocation made when the server starts: plans are
// carved out of it and returned to it on eviction, so the cache never calls hipMalloc /
// hipFree (which cost about a millisecond per GB at plan sizes of tens of GB).
struct Arena {
  uint64_t* base = nullptr;
  size_t cap = 0;
  std::map<size_t, size_t> free_;  // offset -> size, coalesced
  static constexpr size_t kAlign = 4096;
  static size_t round(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }
  bool alloc(size_t bytes, size_t* off) {
    const size_t b = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= b) {
        *off = it->first;
        const size_t rest = it->second - b, at = it->first + b;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t bytes) {
    size_t b = round(bytes);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + b == next->first) {
      b += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += b;
        return;
      }
    }
    free_[off] = b;
  }
};

struct Request {
  int64_t id;
  const blb_keys* keys;
  int weight_id;
  int L, Lp;
  int level;  // input level (its weight's); a batch holds requests of one level
  std::vector<blb_ct> X;
  blb_ct* Y;  // caller's array
  int n_out;
  uint64_t mask_seed;
  uint64_t* share;
  int target_level;
  double t_submit = 0, t_done = 0;
  int state = 0;  // 0 queued, 1 running, 2 done, < 0 error code
  PlanEntry* pe = nullptr;
  bool seen = false;  // plan residency recorded (plan hit: ready when first considered)
};

struct Batch {
  std::vector<Request*> reqs;
  hipEvent_t done = nullptr;
  int stream = 0;
};

int ceil_log2i(int64_t v) {
  int r = 0;
  while ((1ll << r) < v) ++r;
  return r;
}

}  // namespace

struct blb_server {
  blb_ctx* c;
  int p50 = 0;  // plaintext format of the cached plans (the context's knob at creation)
  blb_server_config cfg;
  std::vector<hipStream_t> streams;
  std::map<int, Weights> weights;
  std::map<std::pair<int, int>, PlanEntry> plans;  // (weight id, L') -> plan
  std::atomic<size_t> plan_bytes{0};
  Arena arena;
  // asynchronous plan generation (policy 1): up to kGenDepth generations queued on their own
  // stream (stream order keeps the device overflow flag of each one separate)
  static constexpr int kGenDepth = 2;
  hipStream_t gen_stream = nullptr;
  int* gen_flag = nullptr;  // pinned [kGenDepth]: each generation's overflow flag
  struct Gen {
    PlanEntry* pe;
    std::pair<int, int> key;
    double t0;
    int slot;
  };
  std::deque<Gen> gens;  // in stream order
  std::map<std::pair<int, int>, int> bad_plans;  // keys whose plan cannot be built -> error
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::map<int64_t, Request*> all;
  std::deque<Batch> running;
  int64_t next_id = 1;
  bool stop = false;
  std::thread worker;
  // statistics
  // statistics written by the worker and read by blb_server_stats: atomics; the others
  // change under `mu`
  std::atomic<int64_t> hits{0}, misses{0}, batches{0}, gen_ns{0};
  // scheduling diagnostics: plan generations deferred for lack of a free arena range or of
  // device memory for their temporaries, plan bytes generated, batch launches retried after
  // ENOMEM, and the time the worker held queued requests with nothing on the GPU for them
  // (no batch running, no generation in flight)
  std::atomic<int64_t> defer_room{0}, defer_mem{0}, gen_bytes{0}, launch_retries{0}, stall_ns{0};
  int64_t rejected = 0, completed = 0, failed = 0;
  std::vector<double> latencies;
};

namespace {

// carve `need` bytes out of the plan arena, evicting least-recently-used plans that no
// admitted request uses until a contiguous range is free; false if that is impossible now
bool make_room(blb_server* S, size_t need, size_t* off) {
  while (!S->arena.alloc(need, off)) {
    auto victim = S->plans.end();
    for (auto it = S->plans.begin(); it != S->plans.end(); ++it)
      if (it->second.users == 0 && (victim == S->plans.end() || it->second.last_use < victim->second.last_use)) victim = it;
    if (victim == S->plans.end()) return false;
    S->plan_bytes -= victim->second.bytes;
    blb_plan_destroy(victim->second.plan);
    S->arena.release(victim->second.off, victim->second.bytes);
    S->plans.erase(victim);
  }
  return true;
}

bool plan_ready(blb_server* S, const Request* r) {
  auto it = S->plans.find(std::make_pair(r->weight_id, r->Lp));
  return it != S->plans.end() && !it->second.pending;
}

// admit a request whose plan is resident and ready: 1; else 0.  A request counts as a plan
// hit when its plan was ready the first time it was considered.
int admit_ready(blb_server* S, Request* r) {
  auto it = S->plans.find(std::make_pair(r->weight_id, r->Lp));
  const bool ready = it != S->plans.end() && !it->second.pending;
  if (!r->seen) {
    r->seen = true;
    if (ready) ++S->hits;
  }
  if (!ready) return 0;
  it->second.users++;
  it->second.last_use = now_s();
  r->pe = &it->second;
  return 1;
}

// build the plan of r's (weight, L'): synchronously (async = false) or enqueued on the
// generation stream.  1: built / enqueued, 0: no room now, < 0: the request cannot be served.
int generate_plan(blb_server* S, Request* r, bool async) {
  blb_ctx* c = S->c;
  const auto key = std::make_pair(r->weight_id, r->Lp);
  auto bad = S->bad_plans.find(key);
  if (bad != S->bad_plans.end()) return bad->second;
  const Weights* wp;
  {
    std::lock_guard<std::mutex> lk(S->mu);  // registered weights never change (map nodes are stable)
    wp = &S->weights.at(r->weight_id);
  }
  const Weights& w = *wp;
  const size_t need = cp_plan_bytes(c, r->Lp, w.d_in, w.d_out, w.level, w.cplx, S->p50);
  if (Arena::round(need) > S->arena.cap) return BLB_ENOMEM;
  size_t off = 0;
  if (!make_room(S, need, &off)) {  // memory frees up when running batches finish
    ++S->defer_room;
    return 0;
  }
  const double t0 = now_s();
  blb_plan* P = nullptr;
  hipStream_t saved = c->stream;
  if (async) c->stream = S->gen_stream;
  int slot = 0;  // a flag slot no queued generation uses
  if (async)
    for (slot = 0; slot < blb_server::kGenDepth; ++slot) {
      bool used = false;
      for (const auto& g : S->gens) used |= g.slot == slot;
      if (!used) break;
    }
  const int rc = cp_plan_create(c, w.W.data(), w.d_in, w.d_out, r->Lp, w.level, (uint64_t*)((char*)S->arena.base + off), &P,
                                async ? S->gen_flag + slot : nullptr, w.W_dev, 0, 0, w.cplx, S->p50);
  hipEvent_t ev = nullptr;
  if (rc == BLB_OK && async && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) (void)hipEventRecord(ev, c->stream);
  c->stream = saved;
  if (rc) {
    S->arena.release(off, need);
    if (rc == BLB_ENOMEM) {
      ++S->defer_mem;
      return 0;
    }
    S->bad_plans[key] = rc;
    return rc;
  }
  ++S->misses;
  S->gen_bytes += (int64_t)P->bytes;
  PlanEntry& pe = S->plans[key];
  pe.plan = P;
  pe.off = off;
  pe.bytes = P->bytes;
  pe.users = 0;
  pe.last_use = now_s();
  S->plan_bytes += P->bytes;
  if (async) {
    if (!ev) (void)hipStreamSynchronize(S->gen_stream);
    pe.pending = ev != nullptr;
    pe.ready = ev;
    pe.users = pe.pending ? 1 : 0;  // not evictable while being written
    if (pe.pending) S->gens.push_back(blb_server::Gen{&pe, key, t0, slot});
  } else {
    S->gen_ns += (int64_t)((now_s() - t0) * 1e9);
  }
  return 1;
}

// completes the asynchronous generations whose events have fired (in stream order)
void poll_generation(blb_server* S) {
  while (!S->gens.empty() && hipEventQuery(S->gens.front().pe->ready) == hipSuccess) {
    const blb_server::Gen g = S->gens.front();
    S->gens.pop_front();
    PlanEntry* pe = g.pe;
    S->gen_ns += (int64_t)((now_s() - g.t0) * 1e9);
    (void)hipEventDestroy(pe->ready);
    pe->ready = nullptr;
    pe->pending = false;
    pe->users--;
    if (S->gen_flag[g.slot]) {  // encoder overflow: the weights cannot be encoded at this scale
      S->gen_flag[g.slot] = 0;
      S->bad_plans[g.key] = BLB_EINVAL;
      S->plan_bytes -= pe->bytes;
      blb_plan_destroy(pe->plan);
      S->arena.release(pe->off, pe->bytes);
      S->plans.erase(g.key);
    }
  }
}

void finish_batches(blb_server* S, bool block) {
  while (!S->running.empty()) {
    Batch& b = S->running.front();
    if (block) (void)hipEventSynchronize(b.done);
    else if (hipEventQuery(b.done) != hipSuccess) return;
    const double t = now_s();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (Request* r : b.reqs) {
        r->t_done = t;
        r->pe->users--;
        if (r->state != 1) {  // the batch failed at launch: keep its error code
          ++S->failed;
          continue;
        }
        r->state = 2;
        S->latencies.push_back(t - r->t_submit);
        ++S->completed;
      }
    }
    (void)hipEventDestroy(b.done);
    S->running.pop_front();
    S->cv.notify_all();
  }
}

void worker_loop(blb_server* S) {
  blb_ctx* c = S->c;
  (void)hipSetDevice(c->device);
  int next_stream = 0;
  double stall_since = -1;  // start of a stretch with queued requests and nothing on the GPU for them
  for (;;) {
    std::vector<Request*> pending;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait_for(lk, std::chrono::microseconds(200), [&] { return S->stop || !S->queue.empty(); });
      if (S->stop && S->queue.empty() && S->running.empty()) return;
      pending.assign(S->queue.begin(), S->queue.end());
    }
    finish_batches(S, false);
    if (pending.empty()) continue;
    std::vector<Request*> batch;
    std::vector<Request*> rejected;
    auto reject = [&](Request* r, int code) {
      r->state = code;
      rejected.push_back(r);
    };
    if (S->cfg.policy == 1) {
      poll_generation(S);
      Request* oldest = pending.front();
      const bool overdue = (now_s() - oldest->t_submit) * 1e3 > S->cfg.max_wait_ms;
      // An overdue request whose plan is missing has its plan generated first.  When the plan
      // cache has no room for it because batches in flight hold the other plans, no new batch
      // is formed until they finish: otherwise requests on resident plans, arriving all the
      // time, would keep those plans pinned and starve it.
      bool hold = false;
      const auto okey = std::make_pair(oldest->weight_id, oldest->Lp);
      if (overdue && !S->bad_plans.count(okey) && !S->plans.count(okey) && (int)S->gens.size() < blb_server::kGenDepth) {
        const int g = generate_plan(S, oldest, true);
        if (g < 0) reject(oldest, g);
        hold = g == 0;
      }
      // requests whose plan is ready, the oldest first when it is overdue; no new batch while
      // n_streams + 1 are in flight (the worker keeps queueing plan generations meanwhile)
      const bool can_launch = !hold && (int)S->running.size() < (int)S->streams.size() + 1;
      if (can_launch && overdue && admit_ready(S, oldest)) batch.push_back(oldest);
      for (Request* r : pending) {
        if (!can_launch || (int)batch.size() >= S->cfg.max_batch) break;
        if (r == oldest && overdue) continue;
        if (S->bad_plans.count(std::make_pair(r->weight_id, r->Lp))) reject(r, S->bad_plans[std::make_pair(r->weight_id, r->Lp)]);
        else if (!batch.empty() && r->level != batch.front()->level) continue;  // one level per batch
        else if (admit_ready(S, r)) batch.push_back(r);
      }
      // queue the plans of the oldest requests that have none, up to kGenDepth at a time
      for (Request* r : pending) {
        if (hold || (int)S->gens.size() >= blb_server::kGenDepth) break;
        if (std::find(rejected.begin(), rejected.end(), r) != rejected.end()) continue;
        if (S->plans.count(std::make_pair(r->weight_id, r->Lp))) continue;
        const int g = generate_plan(S, r, true);
        if (g < 0) reject(r, g);
        if (g == 0) break;  // no room until running batches finish
      }
    } else {
      // arrival order; a missing plan is built synchronously before its request runs
      for (Request* r : pending) {
        if ((int)batch.size() >= S->cfg.max_batch) break;
        if (!batch.empty() && r->level != batch.front()->level) break;  // one level per batch
        if (!plan_ready(S, r)) {
          r->seen = true;  // a miss
          const int g = generate_plan(S, r, false);
          if (g < 0) {
            reject(r, g);
            continue;
          }
          if (g == 0) break;  // wait for memory
        }
        if (admit_ready(S, r)) batch.push_back(r);
        else break;
      }
    }
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (Request* r : batch) S->queue.erase(std::find(S->queue.begin(), S->queue.end(), r));
      for (Request* r : rejected) {
        S->queue.erase(std::find(S->queue.begin(), S->queue.end(), r));
        r->t_done = now_s();
        ++S->rejected;
      }
    }
    if (!rejected.empty()) S->cv.notify_all();
    const bool stalled = batch.empty() && S->gens.empty() && S->running.empty() && pending.size() > rejected.size();
    if (stalled && stall_since < 0) stall_since = now_s();
    if (!stalled && stall_since >= 0) {
      S->stall_ns += (int64_t)((now_s() - stall_since) * 1e9);
      stall_since = -1;
    }
    if (batch.empty()) {
      if (!S->gens.empty()) std::this_thread::sleep_for(std::chrono::microseconds(50));  // a plan is on its way
      else if (!S->running.empty()) finish_batches(S, true);  // a batch slot or memory frees up
      continue;
    }
    // launch the batch on the next stream
    hipStream_t saved = c->stream;
    c->stream = S->streams[next_stream];
    std::vector<blb_cp_instance> inst;
    for (Request* r : batch) {
      blb_cp_instance I;
      I.keys = r->keys;
      I.plan = r->pe->plan;
      I.X = r->X.data();
      I.n_in = (int)r->X.size();
      I.Y = r->Y;
      I.n_out = r->n_out;
      inst.push_back(I);
      r->state = 1;
    }
    int rc = blb_batch_matmul_cp(c, inst.data(), (int)inst.size());
    if (rc == BLB_ENOMEM) {
      ++S->launch_retries;
      // the batch's temporaries did not fit beside the batches in flight (the call fails before it
      // writes any output): let those finish, give back idle memory and try again, then one
      // request at a time
      finish_batches(S, true);
      (void)blb_ctx_trim(c);
      rc = blb_batch_matmul_cp(c, inst.data(), (int)inst.size());
      if (rc == BLB_ENOMEM && inst.size() > 1) {
        rc = BLB_OK;
        for (size_t q = 0; q < inst.size() && rc == BLB_OK; ++q) rc = blb_batch_matmul_cp(c, &inst[q], 1);
      }
    }
    // mask-and-share per request: a failure marks that request only
    std::vector<int> mrc(batch.size(), BLB_OK);
    for (size_t k = 0; k < batch.size() && rc == BLB_OK; ++k)
      if (batch[k]->share)
        mrc[k] = blb_mask_to_share(c, batch[k]->Y, batch[k]->n_out, batch[k]->mask_seed, batch[k]->target_level, batch[k]->share);
    Batch b;
    b.reqs = batch;
    b.stream = next_stream;
    (void)hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
    (void)hipEventRecord(b.done, c->stream);
    c->stream = saved;
    next_stream = (next_stream + 1) % (int)S->streams.size();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (size_t k = 0; k < batch.size(); ++k)
        if (rc != BLB_OK) batch[k]->state = rc;
        else if (mrc[k] != BLB_OK) batch[k]->state = mrc[k];
    }
    ++S->batches;
    S->running.push_back(b);
    // policy 0 (the synchronous per-op baseline) waits here; policy 1 checks before launching
    if (S->cfg.policy == 0)
      while ((int)S->running.size() >= (int)S->streams.size() + 1) finish_batches(S, true);
  }
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0;
  std::sort(v.begin(), v.end());
  const double idx = p * (v.size() - 1);
  const size_t lo = (size_t)idx, hi = std::min(v.size() - 1, lo + 1);
  return v[lo] + (v[hi] - v[lo]) * (idx - lo);
}

}  // namespace

extern "C" {

int blb_server_create(blb_ctx* c, const blb_server_config* cfg, blb_server** out) {
  if (!c || !cfg || !out || cfg->max_batch < 1 || cfg->max_queue < 1 || cfg->n_streams < 1 || cfg->n_streams > 8 ||
      (cfg->policy != 0 && cfg->policy != 1) || !(cfg->max_wait_ms >= 0))
    return BLB_EINVAL;
  *out = nullptr;
  blb_server* S = new (std::nothrow) blb_server();
  if (!S) return BLB_ENOMEM;
  S->c = c;
  S->p50 = c->plan_p50;
  S->cfg = *cfg;
  // device memory that the stream-ordered pool keeps cached would crowd out the plan arena and
  // the batch workspaces: release it before reserving them
  if (blb_ctx_trim(c) != BLB_OK) {
    delete S;
    return BLB_EDEVICE;
  }
  S->arena.cap = cfg->plan_cache_bytes / Arena::kAlign * Arena::kAlign;
  if (S->arena.cap > 0) {
    if (c->budget && c->dev_bytes + S->arena.cap > c->budget) {
      delete S;
      return BLB_ENOMEM;
    }
    if (hipMalloc((void**)&S->arena.base, S->arena.cap) != hipSuccess) {
      (void)hipGetLastError();
      delete S;
      return BLB_ENOMEM;
    }
    c->dev_bytes += S->arena.cap;
    S->arena.free_[0] = S->arena.cap;
  }
  if (hipStreamCreateWithFlags(&S->gen_stream, hipStreamNonBlocking) != hipSuccess ||
      hipHostMalloc((void**)&S->gen_flag, sizeof(int) * blb_server::kGenDepth, hipHostMallocDefault) != hipSuccess) {
    if (S->gen_stream) (void)hipStreamDestroy(S->gen_stream);
    if (S->arena.base) {
      (void)hipFree(S->arena.base);
      c->dev_bytes -= S->arena.cap;
    }
    delete S;
    return BLB_EDEVICE;
  }
  for (int i = 0; i < blb_server::kGenDepth; ++i) S->gen_flag[i] = 0;
  for (int i = 0; i < cfg->n_streams; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t t : S->streams) (void)hipStreamDestroy(t);
      (void)hipStreamDestroy(S->gen_stream);
      (void)hipHostFree(S->gen_flag);
      if (S->arena.base) {
        (void)hipFree(S->arena.base);
        c->dev_bytes -= S->arena.cap;
      }
      delete S;
      return BLB_EDEVICE;
    }
    S->streams.push_back(s);
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) return BLB_EDEVICE;
  S->worker = std::thread(worker_loop, S);
  *out = S;
  return BLB_OK;
}

}  // extern "C"

static int add_weights(blb_server* S, int weight_id, const double* W, int d_in, int d_out, int level, int cplx) {
  if (!S || !W || d_in < 1 || d_out < 1 || level < 1 || level >= S->c->n_q) return BLB_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->weights.count(weight_id)) return BLB_EINVAL;  // a registered weight id is immutable
  const size_t bytes = (size_t)d_in * d_out * 8;
  double* dev = nullptr;
  if (hipMalloc((void**)&dev, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return BLB_ENOMEM;
  }
  if (hipMemcpy(dev, W, bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(dev);
    return BLB_EDEVICE;
  }
  Weights& w = S->weights[weight_id];
  w.W_dev = dev;
  w.W.assign(W, W + (size_t)d_in * d_out);
  w.d_in = d_in;
  w.d_out = d_out;
  w.level = level;
  w.cplx = cplx;
  return BLB_OK;
}

extern "C" {

int blb_server_add_weights(blb_server* S, int weight_id, const double* W, int d_in, int d_out, int level) {
  return add_weights(S, weight_id, W, d_in, d_out, level, 0);
}

int blb_server_add_weights_cplx(blb_server* S, int weight_id, const double* W, int d_in, int d_out, int level) {
  return add_weights(S, weight_id, W, d_in, d_out, level, 1);
}

int blb_server_submit(blb_server* S, const blb_keys* keys, int weight_id, int L, const blb_ct* X, int n_in, blb_ct* Y, int n_out,
                      uint64_t mask_seed, int mask_target_level, uint64_t* share_dev, int64_t* req_id) {
  if (!S || !keys || !X || !Y || !req_id || L < 1 || L > S->c->n / 2) return BLB_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto wit = S->weights.find(weight_id);
  if (wit == S->weights.end()) return BLB_EINVAL;
  if ((int)S->queue.size() >= S->cfg.max_queue) return BLB_EBUSY;
  const Weights& w = wit->second;
  const int Lp = 1 << ceil_log2i(L);
  const int cc = (S->c->n / 2) / Lp;
  const int blocks = (w.d_out + cc - 1) / cc;
  if (n_in != (w.d_in + cc - 1) / cc || n_out != (w.cplx ? (blocks + 1) / 2 : blocks)) return BLB_EINVAL;
  for (int a = 0; a < n_in; ++a)
    if (!X[a].data || X[a].level != w.level || X[a].degree != 1) return BLB_ELEVEL;
  for (int b = 0; b < n_out; ++b)
    if (!Y[b].data) return BLB_EINVAL;
  // mask-to-share runs on the outputs (level w.level - 1): its target must exist and the share
  // buffer must be given
  if (mask_target_level >= 0 && (mask_target_level > w.level - 1 || !share_dev)) return mask_target_level > w.level - 1 ? BLB_ELEVEL : BLB_EINVAL;
  // a request whose keys lack a rotation is refused here rather than failing a whole batch
  if (cp_check_keys(S->c, keys, L, w.d_in, w.d_out) != BLB_OK) return BLB_ENOKEY;
  Request* r = new (std::nothrow) Request();
  if (!r) return BLB_ENOMEM;
  r->id = S->next_id++;
  r->keys = keys;
  r->weight_id = weight_id;
  r->L = L;
  r->Lp = Lp;
  r->level = w.level;
  r->X.assign(X, X + n_in);
  r->Y = Y;
  r->n_out = n_out;
  r->mask_seed = mask_seed;
  r->share = mask_target_level >= 0 ? share_dev : nullptr;
  r->target_level = mask_target_level;
  r->t_submit = now_s();
  S->queue.push_back(r);
  S->all[r->id] = r;
  *req_id = r->id;
  S->cv.notify_all();
  return BLB_OK;
}

int blb_server_poll(blb_server* S, int64_t req_id, int* state, double* latency_ms) {
  if (!S) return BLB_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->all.find(req_id);
  if (it == S->all.end()) return BLB_EINVAL;
  if (state) *state = it->second->state;
  if (latency_ms) *latency_ms = it->second->state == 2 ? (it->second->t_done - it->second->t_submit) * 1e3 : -1.0;
  return BLB_OK;
}

int blb_server_drain(blb_server* S, double timeout_s) {
  if (!S) return BLB_EINVAL;
  const double t_end = now_s() + timeout_s;
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool busy = !S->queue.empty();
    for (auto& kv : S->all) busy |= kv.second->state == 0 || kv.second->state == 1;
    if (!busy) return BLB_OK;
    if (now_s() > t_end) return BLB_EBUSY;
    S->cv.wait_for(lk, std::chrono::milliseconds(1));
  }
}

int blb_server_stats(blb_server* S, double* out, int cap) {
  if (!S || !out || cap < 10) return BLB_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  out[0] = (double)S->completed;
  out[1] = (double)S->rejected;
  out[2] = percentile(S->latencies, 0.5) * 1e3;
  out[3] = percentile(S->latencies, 0.99) * 1e3;
  double m = 0;
  for (double v : S->latencies) m += v;
  out[4] = S->latencies.empty() ? 0 : m / S->latencies.size() * 1e3;
  out[5] = (double)S->hits.load();
  out[6] = (double)S->misses.load();
  out[7] = (double)S->batches.load();
  out[8] = (double)S->gen_ns.load() * 1e-9;
  out[9] = (double)S->plan_bytes.load();
  if (cap > 10) out[10] = (double)S->failed;
  if (cap > 15) {
    out[11] = (double)S->defer_room.load();
    out[12] = (double)S->defer_mem.load();
    out[13] = (double)S->gen_bytes.load();
    out[14] = (double)S->launch_retries.load();
    out[15] = (double)S->stall_ns.load() * 1e-9;
  }
  return BLB_OK;
}

void blb_server_destroy(blb_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (hipStream_t s : S->streams) {
    (void)hipStreamSynchronize(s);
    uploader_forget_stream(S->c, s);
    stack_forget_stream(S->c, s);
    (void)hipStreamDestroy(s);
  }
  (void)hipStreamSynchronize(S->gen_stream);
  uploader_forget_stream(S->c, S->gen_stream);
  stack_forget_stream(S->c, S->gen_stream);
  (void)hipStreamDestroy(S->gen_stream);
  (void)hipHostFree(S->gen_flag);
  for (auto& kv : S->plans)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  for (auto& kv : S->plans) blb_plan_destroy(kv.second.plan);
  for (auto& kv : S->weights) (void)hipFree(kv.second.W_dev);
  if (S->arena.base) {
    (void)hipFree(S->arena.base);
    S->c->dev_bytes -= S->arena.cap;
  }
  for (auto& kv : S->all) delete kv.second;
  delete S;
}

}  // extern "C"
