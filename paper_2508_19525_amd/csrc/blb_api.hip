// Host side of the gfx950 engine: parameters and tables, descriptor uploads, key
// generation, encode/encrypt/decrypt/decode, key switching batches, rescale, matmul_cp and
// mask-and-share, exposed through the C ABI of include/blb.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "blb_internal.h"
#include "blb_kernels.h"

typedef unsigned __int128 u128;

extern "C" void blb_host_enc_tables(int log_n, double* tw, double* twist);
extern "C" void blb_host_cdt(uint64_t out[20]);

namespace {

// ------------------------------------------------------------------------------------------
// host modular helpers (independent of the kernels; used only to build tables)
// ------------------------------------------------------------------------------------------
uint64_t h_mul(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)(((u128)a * b) % m); }
uint64_t h_pow(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = h_mul(r, a, m);
    a = h_mul(a, a, m);
    e >>= 1;
  }
  return r;
}
uint64_t h_inv(uint64_t a, uint64_t p) { return h_pow(a % p, p - 2, p); }

bool h_is_prime(uint64_t n) {
  if (n < 2) return false;
  const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small) {
    if (n % p == 0) return n == p;
  }
  uint64_t d = n - 1;
  int r = 0;
  while (!(d & 1)) { d >>= 1; ++r; }
  for (uint64_t a : small) {
    uint64_t x = h_pow(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool witness = true;
    for (int i = 1; i < r && witness; ++i) {
      x = h_mul(x, x, n);
      if (x == n - 1) witness = false;
    }
    if (witness) return false;
  }
  return true;
}

uint32_t h_brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// a primitive 2N-th root of unity mod q: x^((q-1)/2N) for the first x whose N-th power is -1
uint64_t h_root_2n(uint64_t q, int log_n) {
  const uint64_t two_n = 2ull << log_n;
  for (uint64_t x = 3;; x += 2) {
    const uint64_t r = h_pow(x, (q - 1) / two_n, q);
    if (h_pow(r, two_n / 2, q) == q - 1) return r;
  }
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

#define HIP_OK(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return BLB_EDEVICE; \
  } while (0)

// ------------------------------------------------------------------------------------------
// device memory with budget accounting
// ------------------------------------------------------------------------------------------
int dalloc(blb_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return BLB_OK;
  if (c->budget && c->dev_bytes + bytes > c->budget) return BLB_ENOMEM;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return BLB_ENOMEM;
  }
  c->dev_bytes += bytes;
  return BLB_OK;
}
void dfree(blb_ctx* c, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  c->dev_bytes -= bytes;
}

// ------------------------------------------------------------------------------------------
// temporaries: per-stream stacks (stream-ordered pool for what does not fit)
// ------------------------------------------------------------------------------------------
Workspace* stack_for(blb_ctx* c) {
  for (Workspace* w : c->stacks)
    if (w->stream == c->stream) return w;
  Workspace* w = new (std::nothrow) Workspace();
  if (!w) return nullptr;
  w->stream = c->stream;
  c->stacks.push_back(w);
  return w;
}
void stack_release(blb_ctx* c, Workspace* w) {
  if (w->base) {
    (void)hipFree(w->base);
    c->dev_bytes -= w->cap;
  }
  w->base = nullptr;
  w->cap = 0;
}
// grow an empty stack to the deepest one seen (its earlier bytes may still be read by work
// enqueued on its stream, so that stream drains first)
void stack_fit(blb_ctx* c, Workspace* w) {
  if (w->need <= w->cap || w->frozen) return;
  const size_t quantum = size_t(64) << 20;
  // a quarter of headroom over the deepest need seen (doubling would hold tens of GB idle once
  // batches of large operators have run)
  const size_t cap = (w->need + w->need / 4 + quantum - 1) / quantum * quantum;
  (void)hipStreamSynchronize(w->stream);
  stack_release(c, w);
  bool ok = !c->budget || c->dev_bytes + cap <= c->budget;
  if (ok && hipMalloc((void**)&w->base, cap) != hipSuccess) {
    // memory the stream-ordered pool keeps cached may be what is missing: release it, retry
    (void)hipGetLastError();
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
    ok = hipMalloc((void**)&w->base, cap) == hipSuccess;
  }
  if (!ok) {
    (void)hipGetLastError();
    w->base = nullptr;
    w->frozen = true;  // temporaries that do not fit keep coming from the pool
    return;
  }
  c->dev_bytes += cap;
  w->cap = cap;
}

// Temporaries of one scope.  Eager calls carve them from the current stream's stack (released
// when the scope ends); a graph being recorded carves them from the executor's arena.
struct Tmp {
  blb_ctx* c;
  Workspace* w = nullptr;
  size_t off0 = 0, virt0 = 0;
  std::vector<void*> ptrs;
  bool failed = false;
  explicit Tmp(blb_ctx* cc) : c(cc) {
    if (c->rec) return;
    if (c->fixed) {
      off0 = c->fixed->off;
      return;
    }
    w = stack_for(c);
    if (!w) return;
    if (w->off == 0) stack_fit(c, w);
    off0 = w->off;
    virt0 = w->virt;
  }
  template <class T>
  T* get(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    if (c->rec) {  // recording a graph: carve from the executor's arena, never freed
      ExecRec* r = c->rec;
      const size_t off = align_up(r->arena_off, 256);
      if (off + bytes > r->arena_cap) {
        r->overflow = true;
        failed = true;
        return nullptr;
      }
      r->arena_off = off + bytes;
      return (T*)(r->arena + off);
    }
    if (c->fixed) {  // allocation-free entry point: carve from its fixed region, never allocate
      FixedArena* f = c->fixed;
      const size_t off = align_up(f->off, 256);
      if (off + bytes > f->cap) {
        f->overflow = true;
        failed = true;
        return nullptr;
      }
      f->off = off + bytes;
      return (T*)(f->base + off);
    }
    if (w) {
      w->virt = align_up(w->virt, 256) + bytes;
      w->need = std::max(w->need, w->virt);
      const size_t off = align_up(w->off, 256);
      if (off + bytes <= w->cap) {
        w->off = off + bytes;
        return (T*)(w->base + off);
      }
    }
    if (hipMallocAsync(&p, bytes, c->stream) != hipSuccess) {
      (void)hipGetLastError();
      failed = true;
      return nullptr;
    }
    ptrs.push_back(p);
    return (T*)p;
  }
  ~Tmp() {
    if (w) {
      w->off = off0;
      w->virt = virt0;
    } else if (c->fixed && !c->rec) {
      c->fixed->off = off0;
    }
    for (void* p : ptrs) (void)hipFreeAsync(p, c->stream);
  }
};

// ------------------------------------------------------------------------------------------
// descriptor upload ring
// ------------------------------------------------------------------------------------------
const size_t kUploadCap = 64u << 20;

void ring_free(Uploader* u) {
  for (auto& e : u->inflight) (void)hipEventDestroy(e.copied);
  for (auto e : u->free_events) (void)hipEventDestroy(e);
  if (u->host) (void)hipHostFree(u->host);
  if (u->dev) (void)hipFree(u->dev);
  delete u;
}
// the ring of the context's current stream, created on first use
Uploader* ring_for(blb_ctx* c) {
  for (Uploader* u : c->ups)
    if (u->stream == c->stream) return u;
  Uploader* u = new (std::nothrow) Uploader();
  if (!u) return nullptr;
  u->stream = c->stream;
  u->cap = kUploadCap;
  if (hipHostMalloc((void**)&u->host, u->cap, hipHostMallocDefault) != hipSuccess || hipMalloc((void**)&u->dev, u->cap) != hipSuccess) {
    (void)hipGetLastError();
    ring_free(u);
    return nullptr;
  }
  c->ups.push_back(u);
  return u;
}
int uploader_init(blb_ctx* c) { return ring_for(c) ? BLB_OK : BLB_ENOMEM; }
void uploader_free(blb_ctx* c) {
  for (Uploader* u : c->ups) ring_free(u);
  c->ups.clear();
}
// Copies `bytes` from host memory to a device region that stays valid for all work enqueued
// on the stream before the ring wraps back onto it.
void* upload(blb_ctx* c, const void* data, size_t bytes) {
  if (c->rec) {  // recording: the table lives in the executor's blob, copied once after capture
    ExecRec* r = c->rec;
    const size_t off = align_up(r->blob_host.size(), 256);
    if (off + bytes > r->blob_cap) {
      r->overflow = true;
      return nullptr;
    }
    r->blob_host.resize(off + bytes);
    memcpy(r->blob_host.data() + off, data, bytes);
    return r->blob_dev + off;
  }
  Uploader* up = nullptr;
  if (c->fixed) {  // allocation-free entry point: only an existing ring (made with the context)
    for (Uploader* x : c->ups)
      if (x->stream == c->stream) up = x;
  } else {
    up = ring_for(c);
  }
  if (!up) return nullptr;
  Uploader& u = *up;
  bytes = align_up(bytes, 256);
  if (bytes > u.cap) return nullptr;
  size_t lo = u.head;
  if (lo + bytes > u.cap) lo = 0;
  const size_t hi = lo + bytes;
  // staging bytes about to be rewritten may still be read by their earlier copy
  std::deque<UploadRegion> keep;
  for (const UploadRegion& e : u.inflight) {
    if (e.lo < hi && lo < e.hi) {
      (void)hipEventSynchronize(e.copied);
      u.free_events.push_back(e.copied);
    } else {
      keep.push_back(e);
    }
  }
  u.inflight.swap(keep);
  memcpy(u.host + lo, data, bytes);
  if (hipMemcpyAsync(u.dev + lo, u.host + lo, bytes, hipMemcpyHostToDevice, c->stream) != hipSuccess) return nullptr;
  hipEvent_t ev;
  if (!u.free_events.empty()) {
    ev = u.free_events.back();
    u.free_events.pop_back();
  } else if (c->fixed || hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamSynchronize(c->stream);
    u.head = hi;
    return u.dev + lo;
  }
  (void)hipEventRecord(ev, c->stream);
  u.inflight.push_back(UploadRegion{lo, hi, ev});
  u.head = hi;
  return u.dev + lo;
}

template <class T>
const T* upload_vec(blb_ctx* c, const std::vector<T>& v) {
  return (const T*)upload(c, v.data(), v.size() * sizeof(T));
}

// ------------------------------------------------------------------------------------------
// kernel timing spans
// ------------------------------------------------------------------------------------------
hipEvent_t pool_event(blb_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}
struct Span {
  blb_ctx* c;
  int kind;
  double units;
  hipEvent_t a = nullptr;
  Span(blb_ctx* cc, int k, double u) : c(cc), kind(k), units(u) {
    if (c->timing && !c->rec && !c->fixed) {
      a = pool_event(c);
      (void)hipEventRecord(a, c->stream);
    }
  }
  ~Span() {
    if (c->timing && a) {
      hipEvent_t b = pool_event(c);
      (void)hipEventRecord(b, c->stream);
      c->spans.push_back(TimedSpan{kind, a, b, units});
    }
  }
};

// descriptor batches can exceed the ring: split into chunks
void ntt_descs(blb_ctx* c, const std::vector<PolyDesc>& d, int kind) {
  const size_t chunk = 16384;
  for (size_t off = 0; off < d.size(); off += chunk) {
    const size_t cnt = std::min(chunk, d.size() - off);
    const PolyDesc* dd = (const PolyDesc*)upload(c, d.data() + off, cnt * sizeof(PolyDesc));
    if (!dd) return;
    Span sp(c, BLB_T_NTT, (double)cnt);
    c->counters[1] += (int64_t)cnt;
    switch (kind) {
      case 0: launch_ntt(c, dd, (int)cnt, true); break;
      case 1: launch_ntt(c, dd, (int)cnt, false); break;
      case 2: launch_ntt_rescale(c, dd, (int)cnt); break;
      case 3: launch_ntt_moddown(c, dd, (int)cnt); break;
      case 4: launch_ntt_addto(c, dd, (int)cnt); break;
    }
  }
}
enum { NTT_FWD = 0, NTT_INV = 1, NTT_RESCALE = 2, NTT_MODDOWN = 3, NTT_ADDTO = 4 };

// in-place transform of count limb-polys stored back to back ([item][nl][N]); no table upload
void ntt_regular(blb_ctx* c, uint64_t* base, size_t count, int nl, bool fwd) {
  const size_t chunk = ((size_t)1 << 20) / nl * nl;  // a multiple of nl: every chunk starts at limb 0
  for (size_t off = 0; off < count; off += chunk) {
    const int cnt = (int)std::min(chunk, count - off);
    Span sp(c, BLB_T_NTT, (double)cnt);
    c->counters[1] += cnt;
    launch_ntt_regular(c, base + off * c->n, cnt, nl, fwd);
  }
}

PolyDesc pd(const uint64_t* src, uint64_t* dst, int mod, int log_n) {
  PolyDesc d;
  memset(&d, 0, sizeof(d));
  d.src = src;
  d.dst = dst;
  d.mod = mod;
  d.log_n = log_n;
  return d;
}

ModMap map_identity(int n) {
  ModMap m;
  m.len = n;
  for (int i = 0; i < BLB_MAXM; ++i) m.idx[i] = i < n ? i : 0;
  return m;
}

// ------------------------------------------------------------------------------------------
// key-switching level constants
// ------------------------------------------------------------------------------------------
void build_ks_level(blb_ctx* c, int level, KsLevelConst* k) {
  memset(k, 0, sizeof(*k));
  const int nl = level + 1;
  k->nl = nl;
  k->n_ext = nl + c->n_sp;
  k->n_digits = (nl + c->alpha - 1) / c->alpha;
  k->n_key_mod = c->n_q + c->n_sp;
  uint64_t ext[BLB_MAXM];
  for (int e = 0; e < nl; ++e) ext[e] = c->mod[e];
  for (int t = 0; t < c->n_sp; ++t) ext[nl + t] = c->mod[c->n_q + t];
  for (int e = 0; e < k->n_ext; ++e) {
    const int m = e < nl ? e : c->n_q + (e - nl);
    k->ext[e] = c->mt.m[m];
  }
  for (int j = 0; j < k->n_digits; ++j) {
    const int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, nl);
    k->dlo[j] = lo;
    k->dhi[j] = hi;
    for (int i = lo; i < hi; ++i) {
      uint64_t prod = 1;
      for (int i2 = lo; i2 < hi; ++i2)
        if (i2 != i) prod = h_mul(prod, ext[i2] % ext[i], ext[i]);
      k->qhat_inv[j][i - lo] = (double)h_inv(prod, ext[i]);
      for (int e = 0; e < k->n_ext; ++e) {
        uint64_t pm = 1;
        for (int i2 = lo; i2 < hi; ++i2)
          if (i2 != i) pm = h_mul(pm, ext[i2] % ext[e], ext[e]);
        k->qhat_mod[j][i - lo][e] = (double)pm;
      }
    }
  }
  for (int t = 0; t < c->n_sp; ++t) {
    const uint64_t p = ext[nl + t];
    uint64_t prod = 1;
    for (int t2 = 0; t2 < c->n_sp; ++t2)
      if (t2 != t) prod = h_mul(prod, ext[nl + t2] % p, p);
    k->phat_inv[t] = (double)h_inv(prod, p);
    for (int i = 0; i < nl; ++i) {
      uint64_t pm = 1;
      for (int t2 = 0; t2 < c->n_sp; ++t2)
        if (t2 != t) pm = h_mul(pm, ext[nl + t2] % ext[i], ext[i]);
      k->phat_mod[t][i] = (double)pm;
    }
  }
  for (int i = 0; i < nl; ++i) {
    uint64_t P = 1;
    for (int t = 0; t < c->n_sp; ++t) P = h_mul(P, ext[nl + t] % ext[i], ext[i]);
    k->p_inv[i] = (double)h_inv(P, ext[i]);
  }
}

const SwKey* find_key(const blb_keys* k, uint64_t id) {
  for (const SwKey& s : k->keys)
    if (s.id == id) return &s;
  return nullptr;
}

uint32_t galois_left(const blb_ctx* c, int64_t steps) {
  const int64_t s = c->n / 2;
  const int64_t t = ((steps % s) + s) % s;
  return (uint32_t)h_pow(5, (uint64_t)t, 2ull * c->n);
}

size_t ct_words(const blb_ctx* c, int level, int degree) { return (size_t)(degree + 1) * (level + 1) * c->n; }

// ------------------------------------------------------------------------------------------
// batched key switching
// ------------------------------------------------------------------------------------------
struct KsReq {
  int src;                 // index into the source list
  const SwKey* key;
  uint32_t gal;            // automorphism applied after ModUp (0 = none)
  uint64_t* dst;           // [2][nl][N] output
  const uint64_t* add0;    // added to output poly 0 (permuted by add0_gal), may be null
  uint32_t add0_gal;
  const uint64_t* add1;    // added to output poly 1, may be null
};

// All sources are evaluation-form polys [nl][N] at `level`.  Each request writes
//   dst = (add0' + KS_0, add1 + KS_1), KS = ModDown(sum_j sigma(ModUp_j(src)) * key_j).
// ModUp of every source (hoisted part of the key switch): X[s][j][e] in evaluation form for
// the moduli outside digit j (the digit's own limbs are the source's limbs themselves).
int ks_modup(blb_ctx* c, int level, const std::vector<const uint64_t*>& srcs, uint64_t* X) {
  const KsLevelConst& kc = c->h_kc[level];
  const int nl = kc.nl, n_ext = kc.n_ext, nd = kc.n_digits, n = c->n;
  const int S = (int)srcs.size();
  Tmp tmp(c);
  uint64_t* dcoef = tmp.get<uint64_t>((size_t)S * nl * n);
  if (tmp.failed) return BLB_ENOMEM;
  std::vector<PolyDesc> d;
  d.reserve((size_t)S * nl);
  for (int s = 0; s < S; ++s)
    for (int i = 0; i < nl; ++i) d.push_back(pd(srcs[s] + (size_t)i * n, dcoef + ((size_t)s * nl + i) * n, i, c->log_n));
  ntt_descs(c, d, NTT_INV);
  c->counters[6] += S;
  {
    Span sp(c, BLB_T_MODUP, (double)S * nd * n);
    launch_modup(c, dcoef, X, c->d_kc[level], S, nl, n_ext, nd);
  }
  d.clear();
  for (int s = 0; s < S; ++s)
    for (int j = 0; j < nd; ++j)
      for (int e = 0; e < n_ext; ++e) {
        if (e >= kc.dlo[j] && e < kc.dhi[j]) continue;
        uint64_t* p = X + (((size_t)s * nd + j) * n_ext + e) * n;
        d.push_back(pd(p, p, e < nl ? e : c->n_q + (e - nl), c->log_n));
      }
  ntt_descs(c, d, NTT_FWD);
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}
size_t ks_modup_words(const blb_ctx* c, int level, int n_src) {
  const KsLevelConst& kc = c->h_kc[level];
  return (size_t)n_src * kc.n_digits * kc.n_ext * c->n;
}

// Inner product with the keys (automorphism applied to the hoisted digits), ModDown, and the
// final additions, for each request.
int ks_apply(blb_ctx* c, int level, const std::vector<const uint64_t*>& srcs, const uint64_t* X, const std::vector<KsReq>& reqs) {
  if (reqs.empty()) return BLB_OK;
  const KsLevelConst& kc = c->h_kc[level];
  const int nl = kc.nl, n_ext = kc.n_ext, nd = kc.n_digits, n = c->n;
  const int O = (int)reqs.size();
  Tmp tmp(c);
  uint64_t* U = tmp.get<uint64_t>((size_t)O * 2 * n_ext * n);
  uint64_t* corr = tmp.get<uint64_t>((size_t)O * 2 * nl * n);
  if (tmp.failed) return BLB_ENOMEM;
  std::vector<KsOut> ko(O);
  for (int o = 0; o < O; ++o) {
    ko[o].c1 = srcs[reqs[o].src];
    ko[o].key = reqs[o].key->data;
    ko[o].gal = reqs[o].gal;
    ko[o].src = reqs[o].src;
  }
  const KsOut* ko_dev = upload_vec(c, ko);
  if (!ko_dev) return BLB_EDEVICE;
  c->counters[0] += O;
  // group size: large enough to reuse the key words, small enough to keep about 8192 workgroups
  // in the launch (a small batch keeps one output per thread)
  const int64_t blocks = (int64_t)O * n_ext * ((n / 2 + 255) / 256);
  const int cap = c->ks_variant == 2 ? kKsGroupMax : (int)std::min<int64_t>(kKsGroupMax, std::max<int64_t>(1, blocks / 8192));
  if (c->ks_variant >= 1 && nd <= kKsMaxDigits && cap > 1) {
    // outputs grouped by (key, Galois element), stable, in runs of at most `cap`
    std::vector<int> ord(O);
    for (int o = 0; o < O; ++o) ord[o] = o;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
      if (ko[a].key != ko[b].key) return ko[a].key < ko[b].key;
      return ko[a].gal < ko[b].gal;
    });
    std::vector<KsGroup> groups;
    for (int i = 0; i < O;) {
      int j = i + 1;
      while (j < O && j - i < cap && ko[ord[j]].key == ko[ord[i]].key && ko[ord[j]].gal == ko[ord[i]].gal) ++j;
      groups.push_back(KsGroup{i, j - i});
      i = j;
    }
    const int* ord_dev = upload_vec(c, ord);
    const KsGroup* g_dev = upload_vec(c, groups);
    if (!ord_dev || !g_dev) return BLB_EDEVICE;
    Span sp(c, BLB_T_KS_INNER, (double)O * n_ext * n);
    launch_ks_inner_grouped(c, ko_dev, ord_dev, g_dev, (int)groups.size(), X, c->d_kc[level], U, nl, n_ext, nd);
  } else {
    Span sp(c, BLB_T_KS_INNER, (double)O * n_ext * n);
    launch_ks_inner(c, ko_dev, O, X, c->d_kc[level], U, nl, n_ext, nd);
  }
  std::vector<PolyDesc> d;
  for (int o = 0; o < O; ++o)
    for (int p = 0; p < 2; ++p)
      for (int t = 0; t < c->n_sp; ++t) {
        uint64_t* ptr = U + (((size_t)o * 2 + p) * n_ext + nl + t) * n;
        d.push_back(pd(ptr, ptr, c->n_q + t, c->log_n));
      }
  ntt_descs(c, d, NTT_INV);
  {
    Span sp(c, BLB_T_MODDOWN, (double)O * 2 * n);
    launch_moddown_conv(c, U, corr, c->d_kc[level], O, nl, n_ext);
  }
  d.clear();
  for (int o = 0; o < O; ++o)
    for (int p = 0; p < 2; ++p)
      for (int i = 0; i < nl; ++i) {
        PolyDesc x = pd(corr + (((size_t)o * 2 + p) * nl + i) * n, reqs[o].dst + ((size_t)p * nl + i) * n, i, c->log_n);
        x.src2 = U + (((size_t)o * 2 + p) * n_ext + i) * n;
        x.aux2 = kc.p_inv[i];
        const uint64_t* add = p == 0 ? reqs[o].add0 : reqs[o].add1;
        x.src3 = add ? add + (size_t)i * n : nullptr;
        x.gal = p == 0 ? reqs[o].add0_gal : 0;
        d.push_back(x);
      }
  ntt_descs(c, d, NTT_MODDOWN);
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

// All sources are evaluation-form polys [nl][N] at `level`.  Each request writes
//   dst = (add0' + KS_0, add1 + KS_1), KS = ModDown(sum_j sigma(ModUp_j(src)) * key_j).
int ks_batch(blb_ctx* c, int level, const std::vector<const uint64_t*>& srcs, const std::vector<KsReq>& reqs) {
  if (srcs.empty() || reqs.empty()) return BLB_OK;
  Tmp tmp(c);
  uint64_t* X = tmp.get<uint64_t>(ks_modup_words(c, level, (int)srcs.size()));
  if (tmp.failed) return BLB_ENOMEM;
  int rc = ks_modup(c, level, srcs, X);
  if (rc) return rc;
  return ks_apply(c, level, srcs, X, reqs);
}

// batched rescale: in[t] at `level` (degree+1 polys) -> out[t] at level-1 (compact)
int rescale_batch(blb_ctx* c, int level, int n_poly, const std::vector<const uint64_t*>& in, const std::vector<uint64_t*>& out) {
  const int n = c->n, nl = level + 1;
  const int T = (int)in.size();
  c->counters[5] += T;
  Tmp tmp(c);
  uint64_t* last = tmp.get<uint64_t>((size_t)T * n_poly * n);
  if (tmp.failed) return BLB_ENOMEM;
  std::vector<PolyDesc> d;
  for (int t = 0; t < T; ++t)
    for (int p = 0; p < n_poly; ++p)
      d.push_back(pd(in[t] + ((size_t)p * nl + level) * n, last + ((size_t)t * n_poly + p) * n, level, c->log_n));
  ntt_descs(c, d, NTT_INV);
  d.clear();
  const uint64_t ql = c->mod[level];
  for (int t = 0; t < T; ++t)
    for (int p = 0; p < n_poly; ++p)
      for (int i = 0; i < level; ++i) {
        PolyDesc x = pd(last + ((size_t)t * n_poly + p) * n, out[t] + ((size_t)p * level + i) * n, i, c->log_n);
        x.aux = (double)ql;
        x.src2 = in[t] + ((size_t)p * nl + i) * n;
        x.aux2 = (double)h_inv(ql % c->mod[i], c->mod[i]);
        d.push_back(x);
      }
  ntt_descs(c, d, NTT_RESCALE);
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

int check_ct(const blb_ctx* c, const blb_ct* ct) {
  if (!ct || !ct->data || ct->level < 0 || ct->level >= c->n_q || ct->degree < 1 || ct->degree > 2) return BLB_EINVAL;
  return BLB_OK;
}

// encode `count` dense slot vectors (device, [count][n_vals]) into coefficient residues
int encode_dense_dev(blb_ctx* c, const double* d_vals, int n_vals, int count, double scale, int level, uint64_t* out) {
  const int M = c->n / 2;
  Tmp tmp(c);
  double* a = tmp.get<double>((size_t)count * M * 4);
  double* b = tmp.get<double>((size_t)count * M * 4);
  if (tmp.failed) return BLB_ENOMEM;
  (void)hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream);
  run_encode_dense(c, d_vals, n_vals, count, a, b, scale, level + 1, out, c->d_flag);
  int flag = 0;
  (void)hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return BLB_EDEVICE;
  return flag ? BLB_EINVAL : BLB_OK;
}

}  // namespace

// a stream is about to be destroyed after a synchronisation: drop its stack of temporaries
void stack_forget_stream(blb_ctx* c, hipStream_t s) {
  for (size_t i = 0; i < c->stacks.size(); ++i)
    if (c->stacks[i]->stream == s) {
      stack_release(c, c->stacks[i]);
      delete c->stacks[i];
      c->stacks.erase(c->stacks.begin() + i);
      return;
    }
}

// a stream is about to be destroyed after a synchronisation: drop its upload ring
void uploader_forget_stream(blb_ctx* c, hipStream_t s) {
  for (size_t i = 0; i < c->ups.size(); ++i)
    if (c->ups[i]->stream == s) {
      ring_free(c->ups[i]);
      c->ups.erase(c->ups.begin() + i);
      return;
    }
}

// ------------------------------------------------------------------------------------------
// scratch of the allocation-free entry points: one fixed array per device, held until the
// process ends
// ------------------------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)8 << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) uint64_t scratch[kScratchBytes / 8];
std::mutex g_scratch_mu;
char* g_scratch_dev[kScratchDevices] = {};

// Looks up the device address of this device's copy of `scratch` once per device, with that
// device current (in host code the array's name is a host-side stand-in, never a device
// address: kernels and copies get the looked-up pointer only).
int scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices) return BLB_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return BLB_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return BLB_EDEVICE;
  }
  g_scratch_dev[device] = (char*)p;
  return BLB_OK;
}
char* scratch_of(int device) {
  if (device < 0 || device >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_dev[device];
}

// ==========================================================================================
// C ABI
// ==========================================================================================
extern "C" {

const char* blb_status_str(int code) {
  switch (code) {
    case BLB_OK: return "ok";
    case BLB_EINVAL: return "invalid argument";
    case BLB_ELEVEL: return "level mismatch or not enough limbs";
    case BLB_ESCALE: return "scale mismatch";
    case BLB_ENOKEY: return "missing Galois or relinearisation key";
    case BLB_ENOMEM: return "out of device memory or over the HBM budget";
    case BLB_EDEVICE: return "HIP runtime error";
    case BLB_EBUSY: return "queue full";
    case BLB_ETOOBIG: return "operand needs more than the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

int blb_ctx_create(const blb_params* prm, blb_ctx** out) {
  if (!prm || !out) return BLB_EINVAL;
  *out = nullptr;
  if (prm->log_n < 12 || prm->log_n > 14 || prm->n_q < 1 || prm->n_q > BLB_MAXQ || prm->n_special < 1 ||
      prm->n_special > BLB_MAXSP || prm->dnum < 1 || prm->dnum > prm->n_q)
    return BLB_EINVAL;
  const int alpha = (prm->n_q + prm->dnum - 1) / prm->dnum;
  if (alpha > BLB_MAXALPHA) return BLB_EINVAL;
  if (hipSetDevice(prm->device) != hipSuccess) return BLB_EDEVICE;
  {
    const int src = scratch_init(prm->device);
    if (src) return src;
  }
  blb_ctx* c = new (std::nothrow) blb_ctx();
  if (!c) return BLB_ENOMEM;
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, prm->device) == hipSuccess && prop.multiProcessorCount > 0) c->n_cu = prop.multiProcessorCount;
  }
  c->log_n = prm->log_n;
  c->n = 1 << prm->log_n;
  c->n_q = prm->n_q;
  c->n_sp = prm->n_special;
  c->dnum = prm->dnum;
  c->alpha = alpha;
  c->device = prm->device;
  c->stream = (hipStream_t)prm->stream;
  c->budget = prm->hbm_budget_bytes;
  const int n = c->n, nm = c->n_q + c->n_sp;
  // primes: the largest q = k 2N + 1 below 2^50, in decreasing order
  {
    const uint64_t two_n = 2ull * n;
    int found = 0;
    for (uint64_t k = ((1ull << 50) - 2) / two_n; k > 0 && found < nm; --k) {
      const uint64_t q = k * two_n + 1;
      if (h_is_prime(q)) c->mod[found++] = q;
    }
  }
  std::vector<double> tw_f((size_t)nm * n), tw_i((size_t)nm * n);
  for (int m = 0; m < nm; ++m) {
    const uint64_t q = c->mod[m];
    c->mt.m[m].q = (double)q;
    c->mt.m[m].qinv = 1.0 / (double)q;
    c->mt.m[m].ninv = (double)h_inv((uint64_t)n, q);
    const uint64_t psi = h_root_2n(q, c->log_n), ipsi = h_inv(psi, q);
    for (int k = 0; k < n; ++k) {
      const uint32_t e = h_brv((uint32_t)k, c->log_n);
      tw_f[(size_t)m * n + k] = (double)h_pow(psi, e, q);
      tw_i[(size_t)m * n + k] = (double)h_pow(ipsi, e, q);
    }
  }
  int rc = BLB_OK;
  auto fail = [&](int code) {
    blb_ctx_destroy(c);
    return code;
  };
  if ((rc = dalloc(c, (void**)&c->d_tw_fwd, sizeof(double) * nm * n))) return fail(rc);
  if ((rc = dalloc(c, (void**)&c->d_tw_inv, sizeof(double) * nm * n))) return fail(rc);
  if ((rc = dalloc(c, (void**)&c->d_mods, sizeof(uint64_t) * BLB_MAXM))) return fail(rc);
  if (hipMemcpy(c->d_tw_fwd, tw_f.data(), sizeof(double) * nm * n, hipMemcpyHostToDevice) != hipSuccess) return fail(BLB_EDEVICE);
  if (hipMemcpy(c->d_tw_inv, tw_i.data(), sizeof(double) * nm * n, hipMemcpyHostToDevice) != hipSuccess) return fail(BLB_EDEVICE);
  if (hipMemcpy(c->d_mods, c->mod, sizeof(uint64_t) * BLB_MAXM, hipMemcpyHostToDevice) != hipSuccess) return fail(BLB_EDEVICE);
  // encoder tables (double-double from quad precision)
  {
    const int M = n / 2;
    std::vector<double> tw((size_t)(M / 2) * 4), twist((size_t)M * 4);
    blb_host_enc_tables(c->log_n, tw.data(), twist.data());
    std::vector<int32_t> su(M);  // position (5^j mod 2N - 1) / 4 -> slot j
    uint64_t e = 1;
    for (int j = 0; j < M; ++j) {
      su[(e - 1) / 4] = j;
      e = e * 5 % (2ull * n);
    }
    if ((rc = dalloc(c, (void**)&c->d_enc_tw, tw.size() * sizeof(double)))) return fail(rc);
    if ((rc = dalloc(c, (void**)&c->d_enc_twist, twist.size() * sizeof(double)))) return fail(rc);
    if ((rc = dalloc(c, (void**)&c->d_slot_inv, su.size() * sizeof(int32_t)))) return fail(rc);
    if ((rc = dalloc(c, (void**)&c->d_flag, 256))) return fail(rc);
    if (hipMemcpy(c->d_enc_tw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(BLB_EDEVICE);
    if (hipMemcpy(c->d_enc_twist, twist.data(), twist.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(BLB_EDEVICE);
    if (hipMemcpy(c->d_slot_inv, su.data(), su.size() * 4, hipMemcpyHostToDevice) != hipSuccess) return fail(BLB_EDEVICE);
  }
  for (int l = 0; l < c->n_q; ++l) {
    build_ks_level(c, l, &c->h_kc[l]);
    if ((rc = dalloc(c, (void**)&c->d_kc[l], sizeof(KsLevelConst)))) return fail(rc);
    if (hipMemcpy(c->d_kc[l], &c->h_kc[l], sizeof(KsLevelConst), hipMemcpyHostToDevice) != hipSuccess) return fail(BLB_EDEVICE);
  }
  uint64_t cdt[20];
  blb_host_cdt(cdt);
  upload_cdt(cdt);
  if ((rc = uploader_init(c))) return fail(rc);
  {
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
  }
  if (hipDeviceSynchronize() != hipSuccess) return fail(BLB_EDEVICE);
  *out = c;
  return BLB_OK;
}

void blb_ctx_destroy(blb_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (Workspace* w : c->stacks) {
    (void)hipStreamSynchronize(w->stream);
    stack_release(c, w);
    delete w;
  }
  c->stacks.clear();
  {
    // the context made the device's stream-ordered pool keep what it frees; hand that back
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
  }
  for (TimedSpan& t : c->spans) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  uploader_free(c);
  const int nm = c->n_q + c->n_sp;
  dfree(c, c->d_tw_fwd, sizeof(double) * nm * c->n);
  dfree(c, c->d_tw_inv, sizeof(double) * nm * c->n);
  dfree(c, c->d_mods, sizeof(uint64_t) * BLB_MAXM);
  dfree(c, c->d_enc_tw, sizeof(double) * (c->n / 4) * 4);
  dfree(c, c->d_enc_twist, sizeof(double) * (c->n / 2) * 4);
  dfree(c, c->d_slot_inv, sizeof(int32_t) * (c->n / 2));
  dfree(c, c->d_flag, 256);
  for (int l = 0; l < BLB_MAXQ; ++l) dfree(c, c->d_kc[l], sizeof(KsLevelConst));
  delete c;
}

int blb_ctx_moduli(const blb_ctx* c, uint64_t* out) {
  if (!c || !out) return BLB_EINVAL;
  memcpy(out, c->mod, sizeof(uint64_t) * (c->n_q + c->n_sp));
  return BLB_OK;
}
uint64_t blb_ctx_device_bytes(const blb_ctx* c) { return c ? c->dev_bytes : 0; }

int blb_ctx_trim(blb_ctx* c) {
  if (!c) return BLB_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return BLB_EDEVICE;
  for (Workspace* w : c->stacks)
    if (w->off == 0 && hipStreamSynchronize(w->stream) == hipSuccess) {  // idle: give the bytes back
      stack_release(c, w);
      w->need = 0;
      w->frozen = false;  // it may grow again once memory is free
    }
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
  return BLB_OK;
}

int blb_ctx_set_knob(blb_ctx* c, int knob, int value) {
  if (!c) return BLB_EINVAL;
  switch (knob) {
    case BLB_KNOB_MAC_VARIANT:
      if (value < 0 || value >= BLB_MAC_VARIANTS) return BLB_EINVAL;
      c->mac_variant = value;
      return BLB_OK;
    case BLB_KNOB_BATCH_VARIANT:
      if (value < 0 || value >= BLB_BATCH_VARIANTS) return BLB_EINVAL;
      c->batch_variant = value;
      return BLB_OK;
    case BLB_KNOB_BATCH_GRID:
      if (value < 1 || value > (1 << 20)) return BLB_EINVAL;
      c->batch_grid = value;
      return BLB_OK;
    case BLB_KNOB_NTT_VARIANT:
      if (value < 0 || value > 1) return BLB_EINVAL;
      c->ntt_variant = value;
      return BLB_OK;
    case BLB_KNOB_KS_VARIANT:
      if (value < 0 || value > 2) return BLB_EINVAL;
      c->ks_variant = value;
      return BLB_OK;
    case BLB_KNOB_NTT_RADIX:
      if (value != 16 && value != 32) return BLB_EINVAL;
      c->ntt_radix = value;
      return BLB_OK;
    case BLB_KNOB_BATCH_LIMBS:
      if (value < 0 || value > BLB_MAXQ) return BLB_EINVAL;
      c->batch_limbs = value;
      return BLB_OK;
    case BLB_KNOB_PLAN_FORMAT:
      if (value < 0 || value > 1) return BLB_EINVAL;
      c->plan_p50 = value;
      return BLB_OK;
    default: return BLB_EINVAL;
  }
}
int blb_ctx_get_knob(const blb_ctx* c, int knob) {
  if (!c) return BLB_EINVAL;
  switch (knob) {
    case BLB_KNOB_MAC_VARIANT: return c->mac_variant;
    case BLB_KNOB_BATCH_VARIANT: return c->batch_variant;
    case BLB_KNOB_BATCH_GRID: return c->batch_grid;
    case BLB_KNOB_NTT_VARIANT: return c->ntt_variant;
    case BLB_KNOB_KS_VARIANT: return c->ks_variant;
    case BLB_KNOB_NTT_RADIX: return c->ntt_radix;
    case BLB_KNOB_BATCH_LIMBS: return c->batch_limbs;
    case BLB_KNOB_PLAN_FORMAT: return c->plan_p50;
    default: return BLB_EINVAL;
  }
}

int blb_ctx_counters(blb_ctx* c, int64_t* out, int reset) {
  if (!c || !out) return BLB_EINVAL;
  for (int i = 0; i < 8; ++i) out[i] = c->counters[i];
  if (reset)
    for (int i = 0; i < 8; ++i) c->counters[i] = 0;
  return BLB_OK;
}

int blb_ctx_set_timing(blb_ctx* c, int enable) {
  if (!c) return BLB_EINVAL;
  c->timing = enable != 0;
  return BLB_OK;
}
int blb_ctx_reset_timing(blb_ctx* c) {
  if (!c) return BLB_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return BLB_EDEVICE;
  for (TimedSpan& t : c->spans) {
    c->ev_pool.push_back(t.a);
    c->ev_pool.push_back(t.b);
  }
  c->spans.clear();
  return BLB_OK;
}
int blb_ctx_read_timing(blb_ctx* c, int kind, double* total_ms, int64_t* launches, double* units) {
  if (!c || kind < 0 || kind >= BLB_T_KINDS) return BLB_EINVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return BLB_EDEVICE;
  double ms = 0, u = 0;
  int64_t cnt = 0;
  for (const TimedSpan& t : c->spans) {
    if (t.kind != kind) continue;
    float e = 0;
    if (hipEventElapsedTime(&e, t.a, t.b) != hipSuccess) return BLB_EDEVICE;
    ms += e;
    u += t.units;
    ++cnt;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = cnt;
  if (units) *units = u;
  return BLB_OK;
}
uint64_t blb_galois_elt(const blb_ctx* c, int32_t steps) { return c ? galois_left(c, steps) : 0; }

// ------------------------------------------------------------------------------------------
// keys
// ------------------------------------------------------------------------------------------
static int make_swk(blb_ctx* c, blb_keys* K, const uint64_t* sp_ntt, uint64_t id, SwKey* out) {
  const int n = c->n, nm = c->n_q + c->n_sp;
  const size_t words = (size_t)c->dnum * 2 * nm * n;
  int rc = dalloc(c, (void**)&out->data, words * 8);
  if (rc) return rc;
  out->id = id;
  K->bytes += words * 8;
  Tmp tmp(c);
  uint64_t* e = tmp.get<uint64_t>((size_t)nm * n);
  if (tmp.failed) return BLB_ENOMEM;
  const ModMap all = map_identity(nm);
  uint64_t P_mod[BLB_MAXM];
  for (int m = 0; m < nm; ++m) {
    uint64_t P = 1;
    for (int t = 0; t < c->n_sp; ++t) P = h_mul(P, c->mod[c->n_q + t] % c->mod[m], c->mod[m]);
    P_mod[m] = P;
  }
  for (int j = 0; j < c->dnum; ++j) {
    const uint32_t obj = (uint32_t)(id * 64 + (uint64_t)j);
    uint64_t* b = out->data + (size_t)(j * 2 + 0) * nm * n;
    uint64_t* a = out->data + (size_t)(j * 2 + 1) * nm * n;
    launch_sample_uniform(c, a, nm, all, K->seed, obj, 4 /* key-a */);
    launch_sample_int(c, e, nm, all, K->seed, obj, 5 /* key-e */, true);
    std::vector<PolyDesc> d;
    for (int m = 0; m < nm; ++m) {
      d.push_back(pd(a + (size_t)m * n, a + (size_t)m * n, m, c->log_n));
      d.push_back(pd(e + (size_t)m * n, e + (size_t)m * n, m, c->log_n));
    }
    ntt_descs(c, d, NTT_FWD);
    LimbVals lv;
    lv.use = 1;
    for (int m = 0; m < BLB_MAXM; ++m) lv.v[m] = 0.0;
    const int lo = j * c->alpha, hi = std::min((j + 1) * c->alpha, c->n_q);
    for (int m = lo; m < hi; ++m) lv.v[m] = (double)P_mod[m];
    launch_rlwe_combine(c, b, a, K->s_ntt, e, sp_ntt, lv, nm, all);
  }
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

int blb_keygen(blb_ctx* c, uint64_t seed, const int32_t* rot_steps, int n_rot, blb_keys** out) {
  if (!c || !out || n_rot < 0 || (n_rot > 0 && !rot_steps)) return BLB_EINVAL;
  *out = nullptr;
  const int n = c->n, nm = c->n_q + c->n_sp;
  blb_keys* K = new (std::nothrow) blb_keys();
  if (!K) return BLB_ENOMEM;
  K->ctx = c;
  K->seed = seed;
  K->bytes = 0;
  int rc = dalloc(c, (void**)&K->s_ntt, (size_t)nm * n * 8);
  if (rc) {
    delete K;
    return rc;
  }
  K->bytes += (size_t)nm * n * 8;
  const ModMap all = map_identity(nm);
  launch_sample_int(c, K->s_ntt, nm, all, seed, 0, 1 /* sk */, false);
  std::vector<PolyDesc> d;
  for (int m = 0; m < nm; ++m) d.push_back(pd(K->s_ntt + (size_t)m * n, K->s_ntt + (size_t)m * n, m, c->log_n));
  ntt_descs(c, d, NTT_FWD);
  Tmp tmp(c);
  uint64_t* sp = tmp.get<uint64_t>((size_t)nm * n);
  if (tmp.failed) {
    blb_keys_destroy(K);
    return BLB_ENOMEM;
  }
  // public key over the ciphertext primes: p1 = a (uniform, tag pk-a), p0 = -a s + e (tag pk-e)
  {
    const size_t pkw = (size_t)2 * c->n_q * n;
    if ((rc = dalloc(c, (void**)&K->pk, pkw * 8))) {
      blb_keys_destroy(K);
      return rc;
    }
    K->bytes += pkw * 8;
    const ModMap qs = map_identity(c->n_q);
    uint64_t* p1 = K->pk + (size_t)c->n_q * n;
    launch_sample_uniform(c, p1, c->n_q, qs, seed, 0, 7 /* pk-a */);
    launch_sample_int(c, sp, c->n_q, qs, seed, 0, 8 /* pk-e */, true);
    d.clear();
    for (int m = 0; m < c->n_q; ++m) {
      d.push_back(pd(p1 + (size_t)m * n, p1 + (size_t)m * n, m, c->log_n));
      d.push_back(pd(sp + (size_t)m * n, sp + (size_t)m * n, m, c->log_n));
    }
    ntt_descs(c, d, NTT_FWD);
    LimbVals none;
    none.use = 0;
    launch_rlwe_combine(c, K->pk, p1, K->s_ntt, sp, nullptr, none, c->n_q, qs);
  }
  // relinearisation key: s' = s^2
  launch_ew(c, EW_MUL, sp, K->s_ntt, K->s_ntt, nullptr, nm, all);
  K->keys.push_back(SwKey{0, nullptr});
  if ((rc = make_swk(c, K, sp, 0, &K->keys.back()))) {
    blb_keys_destroy(K);
    return rc;
  }
  for (int r = 0; r < n_rot; ++r) {
    const uint32_t g = galois_left(c, rot_steps[r]);
    if (g == 1 || find_key(K, g)) continue;
    launch_automorph(c, sp, K->s_ntt, nm, g);
    K->keys.push_back(SwKey{g, nullptr});
    if ((rc = make_swk(c, K, sp, g, &K->keys.back()))) {
      blb_keys_destroy(K);
      return rc;
    }
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    blb_keys_destroy(K);
    return BLB_EDEVICE;
  }
  *out = K;
  return BLB_OK;
}

void blb_keys_destroy(blb_keys* K) {
  if (!K) return;
  blb_ctx* c = K->ctx;
  (void)hipStreamSynchronize(c->stream);
  const size_t kw = (size_t)c->dnum * 2 * (c->n_q + c->n_sp) * c->n * 8;
  for (SwKey& s : K->keys) dfree(c, s.data, kw);
  dfree(c, K->s_ntt, (size_t)(c->n_q + c->n_sp) * c->n * 8);
  dfree(c, K->pk, (size_t)2 * c->n_q * c->n * 8);
  delete K;
}

// ------------------------------------------------------------------------------------------
// encode / encrypt / decrypt / decode / export / import
// ------------------------------------------------------------------------------------------
int blb_encode(blb_ctx* c, const double* v, int64_t n_vals, double scale, int level, uint64_t* pt_dev) {
  if (!c || !pt_dev || n_vals < 0 || n_vals > c->n / 2 || (n_vals > 0 && !v) || level < 0 || level >= c->n_q || !(scale > 0))
    return BLB_EINVAL;
  Tmp tmp(c);
  double* dv = tmp.get<double>((size_t)std::max<int64_t>(n_vals, 1));
  if (tmp.failed) return BLB_ENOMEM;
  if (n_vals > 0 && hipMemcpyAsync(dv, v, n_vals * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess) return BLB_EDEVICE;
  return encode_dense_dev(c, dv, (int)n_vals, 1, scale, level, pt_dev);
}

int blb_encrypt(blb_ctx* c, const blb_keys* K, const uint64_t* pt_dev, int level, double scale, uint64_t seed, uint32_t ct_id,
                blb_ct* out) {
  if (!c || !K || !pt_dev || !out || !out->data || level < 0 || level >= c->n_q) return BLB_EINVAL;
  const int n = c->n, nl = level + 1;
  Tmp tmp(c);
  uint64_t* e = tmp.get<uint64_t>((size_t)nl * n);
  uint64_t* pt = tmp.get<uint64_t>((size_t)nl * n);
  if (tmp.failed) return BLB_ENOMEM;
  uint64_t* c0 = out->data;
  uint64_t* c1 = out->data + (size_t)nl * n;
  const ModMap lim = map_identity(nl);
  launch_sample_uniform(c, c1, nl, lim, seed, ct_id, 2 /* enc-a */);
  launch_sample_int(c, e, nl, lim, seed, ct_id, 3 /* enc-e */, true);
  std::vector<PolyDesc> d;
  for (int i = 0; i < nl; ++i) {
    d.push_back(pd(c1 + (size_t)i * n, c1 + (size_t)i * n, i, c->log_n));
    d.push_back(pd(e + (size_t)i * n, e + (size_t)i * n, i, c->log_n));
    d.push_back(pd(pt_dev + (size_t)i * n, pt + (size_t)i * n, i, c->log_n));
  }
  ntt_descs(c, d, NTT_FWD);
  LimbVals none;
  none.use = 0;
  launch_rlwe_combine(c, c0, c1, K->s_ntt, e, pt, none, nl, lim);
  out->level = level;
  out->degree = 1;
  out->scale = scale;
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

int blb_decrypt(blb_ctx* c, const blb_keys* K, const blb_ct* ct, uint64_t* pt_dev) {
  if (!c || !K || !pt_dev || check_ct(c, ct)) return BLB_EINVAL;
  const int n = c->n, nl = ct->level + 1;
  const ModMap lim = map_identity(nl);
  Tmp tmp(c);
  uint64_t* acc = tmp.get<uint64_t>((size_t)nl * n);
  uint64_t* s2 = tmp.get<uint64_t>((size_t)nl * n);
  if (tmp.failed) return BLB_ENOMEM;
  launch_ew(c, EW_MULADD, acc, ct->data + (size_t)nl * n, K->s_ntt, ct->data, nl, lim);
  if (ct->degree == 2) {
    launch_ew(c, EW_MUL, s2, K->s_ntt, K->s_ntt, nullptr, nl, lim);
    launch_ew(c, EW_MULADD, acc, ct->data + (size_t)2 * nl * n, s2, acc, nl, lim);
  }
  std::vector<PolyDesc> d;
  for (int i = 0; i < nl; ++i) d.push_back(pd(acc + (size_t)i * n, pt_dev + (size_t)i * n, i, c->log_n));
  ntt_descs(c, d, NTT_INV);
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

}  // extern "C"

// slot values of a coefficient-form plaintext: real parts into v, imaginary parts into v_im (when
// given)
static int decode_host(blb_ctx* c, const uint64_t* pt_dev, int level, double scale, double* v, double* v_im, int64_t n_vals) {
  if (!c || !pt_dev || !v || level < 0 || level >= c->n_q || n_vals < 0 || n_vals > c->n / 2 || !(scale > 0)) return BLB_EINVAL;
  const int n = c->n, nl = level + 1;
  std::vector<uint64_t> h((size_t)nl * n);
  if (hipMemcpyAsync(h.data(), pt_dev, h.size() * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess) return BLB_EDEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return BLB_EDEVICE;
  // centred CRT lift (mixed radix, long double), then the slot evaluation
  // m_j = Delta^-1 sum_k p_k zeta^(e_j k): real part sum_k p_k cos(pi e_j k / N), imaginary
  // part sum_k p_k sin(pi e_j k / N)
  std::vector<long double> lift(n);
  std::vector<uint64_t> invs((size_t)nl * nl);
  for (int i = 0; i < nl; ++i)
    for (int j = 0; j < i; ++j) invs[(size_t)i * nl + j] = h_inv(c->mod[j] % c->mod[i], c->mod[i]);
  for (int k = 0; k < n; ++k) {
    uint64_t dig[BLB_MAXQ], ndig[BLB_MAXQ];
    for (int i = 0; i < nl; ++i) {
      const uint64_t q = c->mod[i];
      uint64_t x = h[(size_t)i * n + k] % q, y = (q - x) % q;
      for (int j = 0; j < i; ++j) {
        x = h_mul((x + q - dig[j] % q) % q, invs[(size_t)i * nl + j], q);
        y = h_mul((y + q - ndig[j] % q) % q, invs[(size_t)i * nl + j], q);
      }
      dig[i] = x;
      ndig[i] = y;
    }
    long double a = 0, b = 0;
    for (int i = nl - 1; i >= 0; --i) {
      a = a * (long double)c->mod[i] + (long double)dig[i];
      b = b * (long double)c->mod[i] + (long double)ndig[i];
    }
    lift[k] = a <= b ? a : -b;
  }
  std::vector<long double> cosv(2 * n), sinv(v_im ? 2 * n : 0);
  for (int t = 0; t < 2 * n; ++t) cosv[t] = cosl(3.14159265358979323846264338327950288L * (long double)t / (long double)n);
  if (v_im)
    for (int t = 0; t < 2 * n; ++t) sinv[t] = sinl(3.14159265358979323846264338327950288L * (long double)t / (long double)n);
  uint64_t e = 1;
  for (int64_t j = 0; j < n_vals; ++j) {
    long double acc = 0, acc_im = 0;
    uint64_t idx = 0;
    for (int k = 0; k < n; ++k) {
      acc += lift[k] * cosv[idx];
      if (v_im) acc_im += lift[k] * sinv[idx];
      idx += e;
      if (idx >= 2ull * n) idx -= 2ull * n;
    }
    v[j] = (double)(acc / (long double)scale);
    if (v_im) v_im[j] = (double)(acc_im / (long double)scale);
    e = e * 5 % (2ull * n);
  }
  return BLB_OK;
}

extern "C" {

int blb_decode(blb_ctx* c, const uint64_t* pt_dev, int level, double scale, double* v, int64_t n_vals) {
  return decode_host(c, pt_dev, level, scale, v, nullptr, n_vals);
}

int blb_decode_cplx(blb_ctx* c, const uint64_t* pt_dev, int level, double scale, double* v_re, double* v_im, int64_t n_vals) {
  if (!v_im) return BLB_EINVAL;
  return decode_host(c, pt_dev, level, scale, v_re, v_im, n_vals);
}

int blb_export(blb_ctx* c, const blb_ct* ct, uint64_t* host_words) {
  if (!c || !host_words || check_ct(c, ct)) return BLB_EINVAL;
  const int n = c->n, nl = ct->level + 1, np = ct->degree + 1;
  Tmp tmp(c);
  uint64_t* w = tmp.get<uint64_t>((size_t)np * nl * n);
  if (tmp.failed) return BLB_ENOMEM;
  std::vector<PolyDesc> d;
  for (int p = 0; p < np; ++p)
    for (int i = 0; i < nl; ++i)
      d.push_back(pd(ct->data + ((size_t)p * nl + i) * n, w + ((size_t)p * nl + i) * n, i, c->log_n));
  ntt_descs(c, d, NTT_INV);
  if (hipMemcpyAsync(host_words, w, (size_t)np * nl * n * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess) return BLB_EDEVICE;
  return hipStreamSynchronize(c->stream) == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

int blb_import(blb_ctx* c, const uint64_t* host_words, blb_ct* ct) {
  if (!c || !host_words || check_ct(c, ct)) return BLB_EINVAL;
  const int n = c->n, nl = ct->level + 1, np = ct->degree + 1;
  for (int p = 0; p < np; ++p)
    for (int i = 0; i < nl; ++i)
      for (int k = 0; k < n; ++k)
        if (host_words[((size_t)p * nl + i) * n + k] >= c->mod[i]) return BLB_EINVAL;
  if (hipMemcpyAsync(ct->data, host_words, (size_t)np * nl * n * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess) return BLB_EDEVICE;
  std::vector<PolyDesc> d;
  for (int p = 0; p < np; ++p)
    for (int i = 0; i < nl; ++i) {
      uint64_t* x = ct->data + ((size_t)p * nl + i) * n;
      d.push_back(pd(x, x, i, c->log_n));
    }
  ntt_descs(c, d, NTT_FWD);
  return hipStreamSynchronize(c->stream) == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

// ------------------------------------------------------------------------------------------
// rotate / rescale
// ------------------------------------------------------------------------------------------
int blb_rotate(blb_ctx* c, const blb_keys* K, const blb_ct* in, int32_t steps, blb_ct* out) {
  if (!c || !K || !out || !out->data || check_ct(c, in) || in->degree != 1 || in->data == out->data) return BLB_EINVAL;
  const int n = c->n, nl = in->level + 1;
  const uint32_t g = galois_left(c, steps);
  if (g == 1) {
    if (hipMemcpyAsync(out->data, in->data, (size_t)2 * nl * n * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) return BLB_EDEVICE;
  } else {
    const SwKey* key = find_key(K, g);
    if (!key) return BLB_ENOKEY;
    std::vector<const uint64_t*> srcs{in->data + (size_t)nl * n};
    std::vector<KsReq> reqs{KsReq{0, key, g, out->data, in->data, g, nullptr}};
    const int rc = ks_batch(c, in->level, srcs, reqs);
    if (rc) return rc;
  }
  out->level = in->level;
  out->degree = 1;
  out->scale = in->scale;
  return BLB_OK;
}

// blb_rotate with every temporary in the device's fixed scratch array: the key switch's
// ModUp digits, inner products and ModDown corrections (all written before they are read, so
// nothing needs clearing).  No allocation of any kind.
int blb_rotate_noalloc(blb_ctx* c, const blb_keys* K, const blb_ct* in, int32_t steps, blb_ct* out) {
  if (!c || !K || !out || !out->data || check_ct(c, in) || in->degree != 1 || in->data == out->data) return BLB_EINVAL;
  if (c->rec) return BLB_EINVAL;
  char* base = scratch_of(c->device);
  if (!base) return BLB_EDEVICE;
  const KsLevelConst& kc = c->h_kc[in->level];
  const size_t n = (size_t)c->n;
  const size_t need = 8 * n * ((size_t)kc.nl + (size_t)kc.n_digits * kc.n_ext + 2 * (size_t)kc.n_ext + 2 * (size_t)kc.nl) + 4 * 256;
  if (need > kScratchBytes) return BLB_ETOOBIG;
  FixedArena fa{base, kScratchBytes, 0, false};
  c->fixed = &fa;
  int rc = blb_rotate(c, K, in, steps, out);
  c->fixed = nullptr;
  if (fa.overflow) rc = BLB_ETOOBIG;
  return rc;
}

int blb_rescale(blb_ctx* c, const blb_ct* in, blb_ct* out) {
  if (!c || !out || !out->data || check_ct(c, in) || in->data == out->data) return BLB_EINVAL;
  if (in->level < 1) return BLB_ELEVEL;
  const int rc = rescale_batch(c, in->level, in->degree + 1, {in->data}, {out->data});
  if (rc) return rc;
  out->level = in->level - 1;
  out->degree = in->degree;
  out->scale = in->scale / (double)c->mod[in->level];
  return BLB_OK;
}

// Batched negacyclic transform of caller-owned limb-polys [n_polys][n_limbs][N], in place;
// limb i is taken modulo prime i of the chain (ciphertext primes, then special primes).
int blb_ntt(blb_ctx* c, uint64_t* data, int64_t n_polys, int32_t n_limbs, int32_t inverse) {
  if (!c || n_polys < 0 || n_limbs < 1 || n_limbs > c->n_q + c->n_sp || (inverse != 0 && inverse != 1)) return BLB_EINVAL;
  if (n_polys == 0) return BLB_OK;
  if (!data) return BLB_EINVAL;
  ntt_regular(c, data, (size_t)n_polys * n_limbs, n_limbs, inverse == 0);
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

// ------------------------------------------------------------------------------------------
// matmul_cp
// ------------------------------------------------------------------------------------------
static int ceil_log2(int64_t v) {
  int r = 0;
  while ((1ll << r) < v) ++r;
  return r;
}

static CpGeom cp_geometry(const blb_ctx* c, int L, int d_in, int d_out) {
  CpGeom g;
  const int s = c->n / 2;
  g.d_in = d_in;
  g.d_out = d_out;
  g.L = L;
  g.Lp = 1 << ceil_log2(L);
  g.c = s / g.Lp;
  const int din_p = 1 << ceil_log2(d_in), dout_p = 1 << ceil_log2(d_out);
  g.c_eff = std::min(g.c, din_p);
  g.c_out = std::min(g.c, dout_p);
  g.n_in = (d_in + g.c - 1) / g.c;
  g.n_out = (d_out + g.c - 1) / g.c;
  g.B = 1 << ((ceil_log2(g.c_eff) + 1) / 2);
  g.G = g.c_eff / g.B;
  g.cplx = 0;
  return g;
}

}  // extern "C"

// head groups of matmul_cc: powers of two, largest first (12 = 8 + 4)
static void cc_group_sizes(int heads, std::vector<int>& out) {  // powers of two, largest first
  int h = heads;
  while (h > 0) {
    int g = 1;
    while (g * 2 <= h) g *= 2;
    out.push_back(g);
    h -= g;
  }
}

// BLB_OK when K holds every Galois key matmul_cp needs at this geometry (baby and giant steps)
int cp_check_keys(const blb_ctx* c, const blb_keys* K, int L, int d_in, int d_out) {
  const CpGeom g = cp_geometry(c, L, d_in, d_out);
  for (int i = 1; i < g.B; ++i)
    if (!find_key(K, galois_left(c, (int64_t)i * g.Lp))) return BLB_ENOKEY;
  for (int j = 1; j < g.G; ++j)
    if (!find_key(K, galois_left(c, (int64_t)j * g.B * g.Lp))) return BLB_ENOKEY;
  return BLB_OK;
}

size_t cp_plan_bytes(const blb_ctx* c, int L, int d_in, int d_out, int level, int cplx, int p50) {
  const CpGeom g = cp_geometry(c, L, d_in, d_out);
  const int n_out = cplx ? (g.n_out + 1) / 2 : g.n_out;
  return (size_t)n_out * g.G * g.n_in * g.B * (level + 1) * pt_poly_bytes(c->n, p50);
}

// matmul_cp plan; the plaintexts go to `mem` (cp_plan_bytes bytes, caller-owned) when given,
// else to library memory.  With flag_host (pinned) the call returns once the work is enqueued:
// the encoder's overflow flag lands in *flag_host when the stream reaches it (non-zero: the
// plan is unusable), and W must stay valid until then.
int cp_plan_create(blb_ctx* c, const double* W, int d_in, int d_out, int L, int level, uint64_t* mem, blb_plan** out, int* flag_host,
                   const double* W_dev, int diag_heads, int diag_dv, int cplx, int p50) {
  if (!c || (!W && !W_dev) || !out || d_in < 1 || d_out < 1 || L < 1 || L > c->n / 2 || level < 1 || level >= c->n_q) return BLB_EINVAL;
  *out = nullptr;
  if (p50 < 0) p50 = c->plan_p50;
  // diagonal-packed input: one table entry per input ciphertext (head groups in the order
  // matmul_cc forms them); the geometry is that of a spatial-first input of n_heads d_v' columns
  std::vector<CpDiagIn> dtab;
  CpDiag dg{nullptr, 0, 0, 0};
  int d_geom = d_in;
  if (diag_heads > 0) {
    if (diag_dv < 1 || (int64_t)diag_heads * diag_dv != d_in) return BLB_EINVAL;
    const int S = c->n / 2, lp = 1 << ceil_log2(L), dvp = 1 << ceil_log2(diag_dv);
    if (dvp > lp) return BLB_EINVAL;
    std::vector<int> gs;
    cc_group_sizes(diag_heads, gs);
    int h0 = 0;
    for (int H : gs) {
      if (S % (lp * H)) return BLB_EINVAL;
      const int cg = S / (lp * H);
      if (cg > dvp) return BLB_EINVAL;
      for (int o = 0; o < dvp / cg; ++o) dtab.push_back(CpDiagIn{h0, ceil_log2(H), cg, o});
      h0 += H;
    }
    d_geom = diag_heads * dvp;
    dg = CpDiag{nullptr, diag_dv, dvp, L};
  }
  CpGeom g = cp_geometry(c, L, d_geom, d_out);
  if (diag_heads > 0 && ((int)dtab.size() != g.n_in || g.c_eff != g.c)) return BLB_EINVAL;
  if (cplx) {
    g.cplx = 1;
    g.n_out = (g.n_out + 1) / 2;
  }
  const int n = c->n, nl = level + 1;
  const int n_bj = g.n_out * g.G, n_ai = g.n_in * g.B;
  const size_t n_pt = (size_t)n_bj * n_ai;
  blb_plan* P = new (std::nothrow) blb_plan();
  if (!P) return BLB_ENOMEM;
  P->ctx = c;
  P->kind = 1;
  P->level = level;
  P->g = g;
  P->p50 = p50 ? 1 : 0;
  P->bytes = n_pt * nl * pt_poly_bytes(n, P->p50);
  int rc = BLB_OK;
  if (mem) {
    P->pt = mem;
    P->owns_pt = false;
  } else if ((rc = dalloc(c, (void**)&P->pt, P->bytes))) {
    delete P;
    return rc;
  }
  const int M = n / 2;
  const int chunk = 512;
  {
    Tmp tmp(c);
    const double* dW = W_dev;
    double* a = tmp.get<double>((size_t)chunk * M * 4);
    double* b = tmp.get<double>((size_t)chunk * M * 4);
    // 50-bit format: a chunk of plaintexts is encoded here, then transformed and packed into the plan
    uint64_t* raw = P->p50 ? tmp.get<uint64_t>((size_t)chunk * nl * n) : nullptr;
    if (!dW) {
      double* w = tmp.get<double>((size_t)d_in * d_out);
      if (w && hipMemcpyAsync(w, W, (size_t)d_in * d_out * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
        blb_plan_destroy(P);
        return BLB_EDEVICE;
      }
      dW = w;
    }
    if (!dtab.empty()) {
      CpDiagIn* t = tmp.get<CpDiagIn>(dtab.size());
      if (t && hipMemcpyAsync(t, dtab.data(), dtab.size() * sizeof(CpDiagIn), hipMemcpyHostToDevice, c->stream) != hipSuccess) {
        blb_plan_destroy(P);
        return BLB_EDEVICE;
      }
      dg.tab = t;
    }
    if (tmp.failed) {
      blb_plan_destroy(P);
      return BLB_ENOMEM;
    }
    (void)hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream);
    const double scale = (double)c->mod[level] / BLB_NOISE_BOOST;
    for (size_t p0 = 0; p0 < n_pt; p0 += chunk) {
      const int cnt = (int)std::min<size_t>(chunk, n_pt - p0);
      uint64_t* dst = P->p50 ? raw : P->pt + p0 * nl * n;
      run_encode_cp(c, dW, g, (int)p0, cnt, a, b, scale, nl, dst, c->d_flag, dg);
      if (P->p50) {
        Span sp(c, BLB_T_NTT, (double)cnt * nl);
        c->counters[1] += (int64_t)cnt * nl;
        launch_ntt_pack50(c, raw, (uint8_t*)P->pt + p0 * nl * pt50_bytes(n), cnt * nl, nl);
      } else {
        ntt_regular(c, dst, (size_t)cnt * nl, nl, true);
      }
    }
    if (flag_host) {
      if (hipMemcpyAsync(flag_host, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess) {
        (void)hipStreamSynchronize(c->stream);
        blb_plan_destroy(P);
        return BLB_EDEVICE;
      }
    } else {
      int flag = 0;
      (void)hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
      if (hipStreamSynchronize(c->stream) != hipSuccess || flag) {
        blb_plan_destroy(P);
        return flag ? BLB_EINVAL : BLB_EDEVICE;
      }
    }
  }
  *out = P;
  return BLB_OK;
}

extern "C" {

int blb_plan_matmul_cp(blb_ctx* c, const double* W, int d_in, int d_out, int L, int level, blb_plan** out) {
  return cp_plan_create(c, W, d_in, d_out, L, level, nullptr, out, nullptr, nullptr);
}

int blb_plan_matmul_cp_mhp(blb_ctx* c, const double* W, int d_in, int n_heads, int d_head, int L, int level, blb_plan** out) {
  if (!c || !W || !out || d_in < 1 || n_heads < 1 || d_head < 1 || L < 1 || L > c->n / 2) return BLB_EINVAL;
  *out = nullptr;
  // output ciphertext b of the plan is operand ciphertext b of the ct-ct product: block u holds
  // column a c_g + u / H of head h0 + (u mod H) for the group (H heads from h0) that b belongs to
  const int S = c->n / 2, lp = 1 << ceil_log2(L), cc = S / lp;
  std::vector<int> gs;
  cc_group_sizes(n_heads, gs);
  std::vector<int> src;  // W column for each reordered column, -1 for a zero column
  int h0 = 0;
  for (int H : gs) {
    if (S % (lp * H) || S / (lp * H) > lp) return BLB_EINVAL;
    const int cg = S / (lp * H), nct = (d_head + cg - 1) / cg;
    for (int a = 0; a < nct; ++a)
      for (int u = 0; u < cc; ++u) {
        const int col = a * cg + u / H;
        src.push_back(col < d_head ? (h0 + u % H) * d_head + col : -1);
      }
    h0 += H;
  }
  const int n_cols = (int)src.size(), w_cols = n_heads * d_head;
  std::vector<double> Wp((size_t)d_in * n_cols);
  for (int r = 0; r < d_in; ++r)
    for (int j = 0; j < n_cols; ++j) Wp[(size_t)r * n_cols + j] = src[j] < 0 ? 0.0 : W[(size_t)r * w_cols + src[j]];
  return cp_plan_create(c, Wp.data(), d_in, n_cols, L, level, nullptr, out, nullptr, nullptr);
}

int blb_plan_matmul_cp_diag(blb_ctx* c, const double* W, int n_heads, int d_v, int d_out, int L, int level, blb_plan** out) {
  if (n_heads < 1 || d_v < 1) return BLB_EINVAL;
  return cp_plan_create(c, W, n_heads * d_v, d_out, L, level, nullptr, out, nullptr, nullptr, n_heads, d_v);
}

int blb_plan_matmul_cp_cplx(blb_ctx* c, const double* W, int d_in, int d_out, int L, int level, blb_plan** out) {
  return cp_plan_create(c, W, d_in, d_out, L, level, nullptr, out, nullptr, nullptr, 0, 0, 1);
}

int blb_plan_matmul_cp_diag_cplx(blb_ctx* c, const double* W, int n_heads, int d_v, int d_out, int L, int level, blb_plan** out) {
  if (n_heads < 1 || d_v < 1) return BLB_EINVAL;
  return cp_plan_create(c, W, n_heads * d_v, d_out, L, level, nullptr, out, nullptr, nullptr, n_heads, d_v, 1);
}

void blb_plan_destroy(blb_plan* P) {
  if (!P) return;
  (void)hipStreamSynchronize(P->ctx->stream);
  if (P->owns_pt) dfree(P->ctx, P->pt, P->bytes);
  for (size_t i = 0; i < P->extra.size(); ++i) dfree(P->ctx, P->extra[i], P->extra_bytes[i]);
  delete P;
}

int blb_plan_info(const blb_plan* P, int32_t* info) {
  if (!P || !info) return BLB_EINVAL;
  const CpGeom& g = P->g;
  const int32_t v[8] = {g.Lp, g.c, g.c_eff, g.c_out, g.n_in, g.n_out, g.B, g.G};
  memcpy(info, v, sizeof(v));
  return BLB_OK;
}

int blb_matmul_cp(blb_ctx* c, const blb_keys* K, const blb_plan* P, const blb_ct* X, int n_in, blb_ct* Y, int n_out) {
  if (!c || !K || !P || !X || !Y || P->kind != 1) return BLB_EINVAL;
  const CpGeom& g = P->g;
  if (n_in != g.n_in || n_out != g.n_out) return BLB_EINVAL;
  const int level = P->level, nl = level + 1, n = c->n;
  for (int a = 0; a < n_in; ++a) {
    if (check_ct(c, &X[a]) || X[a].degree != 1) return BLB_EINVAL;
    if (X[a].level != level) return BLB_ELEVEL;
    if (fabs(X[a].scale / X[0].scale - 1.0) > 1e-9) return BLB_ESCALE;
  }
  for (int b = 0; b < n_out; ++b)
    if (!Y[b].data) return BLB_EINVAL;
  std::vector<const SwKey*> kb(g.B, nullptr), kg(g.G, nullptr);
  for (int i = 1; i < g.B; ++i)
    if (!(kb[i] = find_key(K, galois_left(c, (int64_t)i * g.Lp)))) return BLB_ENOKEY;
  for (int j = 1; j < g.G; ++j)
    if (!(kg[j] = find_key(K, galois_left(c, (int64_t)j * g.B * g.Lp)))) return BLB_ENOKEY;
  const size_t ctw = (size_t)2 * nl * n;
  const int n_ai = g.n_in * g.B, n_bj = g.n_out * g.G;
  Tmp tmp(c);
  uint64_t* RX = tmp.get<uint64_t>((size_t)std::max(1, g.n_in * (g.B - 1)) * ctw);
  uint64_t* inner = tmp.get<uint64_t>((size_t)n_bj * ctw);
  uint64_t* rot = tmp.get<uint64_t>((size_t)std::max(1, g.n_out * (g.G - 1)) * ctw);
  uint64_t* acc = tmp.get<uint64_t>((size_t)g.n_out * ctw);
  if (tmp.failed) return BLB_ENOMEM;
  // noise boost: Xs_a = 2^10 X_a (the diagonals are encoded at q_level / 2^10)
  uint64_t* Xs = tmp.get<uint64_t>((size_t)n_in * ctw);
  if (!Xs) return BLB_ENOMEM;
  {
    std::vector<const uint64_t*> xin;
    for (int a = 0; a < n_in; ++a) xin.push_back(X[a].data);
    const uint64_t* const* xin_dev = upload_vec(c, xin);
    if (!xin_dev) return BLB_EDEVICE;
    launch_scale_cts(c, xin_dev, Xs, n_in, nl, BLB_NOISE_BOOST);
  }
  // baby steps, hoisted per input: RX[a][i-1] = Rot_l^{i L'}(Xs_a), i >= 1
  std::vector<const uint64_t*> srcs;
  std::vector<KsReq> reqs;
  std::vector<const uint64_t*> rx_tab(n_ai);
  for (int a = 0; a < n_in; ++a) {
    const uint64_t* xa = Xs + (size_t)a * ctw;
    srcs.push_back(xa + (size_t)nl * n);
    rx_tab[(size_t)a * g.B] = xa;
    for (int i = 1; i < g.B; ++i) {
      const uint32_t gal = galois_left(c, (int64_t)i * g.Lp);
      uint64_t* dst = RX + (size_t)(a * (g.B - 1) + i - 1) * ctw;
      rx_tab[(size_t)a * g.B + i] = dst;
      reqs.push_back(KsReq{a, kb[i], gal, dst, xa, gal, nullptr});
    }
  }
  int rc = ks_batch(c, level, srcs, reqs);
  if (rc) return rc;
  // plaintext MACs
  {
    const uint64_t* const* rx_dev = upload_vec(c, rx_tab);
    if (!rx_dev) return BLB_EDEVICE;
    Span sp(c, BLB_T_CP_MAC, (double)n_bj * nl * n);
    c->counters[2] += (int64_t)n_ai * n_bj;
    c->counters[7] += (int64_t)n_ai * n_bj * nl * (int64_t)pt_poly_bytes(n, P->p50);
    launch_cp_mac(c, P->pt, rx_dev, inner, nl, n_ai, n_bj, c->mac_variant, P->p50);
  }
  // giant steps
  if (g.G > 1) {
    srcs.clear();
    reqs.clear();
    for (int b = 0; b < g.n_out; ++b)
      for (int j = 1; j < g.G; ++j) {
        const uint64_t* src = inner + (size_t)(b * g.G + j) * ctw;
        const uint32_t gal = galois_left(c, (int64_t)j * g.B * g.Lp);
        srcs.push_back(src + (size_t)nl * n);
        reqs.push_back(KsReq{(int)srcs.size() - 1, kg[j], gal, rot + (size_t)(b * (g.G - 1) + j - 1) * ctw, src, gal, nullptr});
      }
    if ((rc = ks_batch(c, level, srcs, reqs))) return rc;
  }
  {
    std::vector<const uint64_t*> terms;
    std::vector<uint64_t*> outs;
    for (int b = 0; b < g.n_out; ++b) {
      terms.push_back(inner + (size_t)(b * g.G) * ctw);
      for (int j = 1; j < g.G; ++j) terms.push_back(rot + (size_t)(b * (g.G - 1) + j - 1) * ctw);
      outs.push_back(acc + (size_t)b * ctw);
    }
    const uint64_t* const* t_dev = upload_vec(c, terms);
    uint64_t* const* o_dev = (uint64_t* const*)upload(c, outs.data(), outs.size() * sizeof(uint64_t*));
    if (!t_dev || !o_dev) return BLB_EDEVICE;
    Span sp(c, BLB_T_EW, (double)g.n_out * ctw);
    launch_sum_cts(c, t_dev, o_dev, g.n_out, g.G, nl);
  }
  std::vector<const uint64_t*> rin;
  std::vector<uint64_t*> rout;
  for (int b = 0; b < g.n_out; ++b) {
    rin.push_back(acc + (size_t)b * ctw);
    rout.push_back(Y[b].data);
  }
  if ((rc = rescale_batch(c, level, 2, rin, rout))) return rc;
  for (int b = 0; b < g.n_out; ++b) {
    Y[b].level = level - 1;
    Y[b].degree = 1;
    Y[b].scale = X[0].scale;  // plaintexts are encoded at q_level, which the rescale removes
  }
  return BLB_OK;
}

// ------------------------------------------------------------------------------------------
// mask-and-share
// ------------------------------------------------------------------------------------------
int blb_rerandomize(blb_ctx* c, const blb_keys* K, blb_ct* cts, int n_ct, uint64_t seed, int flood_bits) {
  if (!c || !K || !cts || n_ct < 1 || flood_bits < 32 || flood_bits > 48) return BLB_EINVAL;
  int max_nl = 0;
  for (int t = 0; t < n_ct; ++t) {
    if (check_ct(c, &cts[t]) || cts[t].degree != 1) return BLB_EINVAL;
    max_nl = std::max(max_nl, cts[t].level + 1);
  }
  if (!K->pk) return BLB_ENOKEY;
  const int n = c->n;
  Tmp tmp(c);
  uint64_t* V = tmp.get<uint64_t>((size_t)4 * max_nl * n);
  if (tmp.failed) return BLB_ENOMEM;
  for (int t = 0; t < n_ct; ++t) {
    const int nl = cts[t].level + 1;
    uint64_t *E0 = V + (size_t)nl * n, *E1 = V + (size_t)2 * nl * n, *T = V + (size_t)3 * nl * n;
    const ModMap lim = map_identity(nl);
    launch_sample_int(c, V, nl, lim, seed, (uint32_t)t, 9 /* rr-v */, false);
    launch_sample_flood(c, E0, nl, lim, seed, (uint32_t)t, 10 /* rr-e0 */, flood_bits);
    launch_sample_int(c, E1, nl, lim, seed, (uint32_t)t, 11 /* rr-e1 */, true);
    std::vector<PolyDesc> d;
    for (int p = 0; p < 3; ++p)
      for (int i = 0; i < nl; ++i) {
        uint64_t* x = V + ((size_t)p * nl + i) * n;
        d.push_back(pd(x, x, i, c->log_n));
      }
    ntt_descs(c, d, NTT_FWD);
    uint64_t* c0 = cts[t].data;
    uint64_t* c1 = cts[t].data + (size_t)nl * n;
    launch_ew(c, EW_MULADD, T, V, K->pk, E0, nl, lim);
    launch_ew(c, EW_ADD, c0, c0, T, nullptr, nl, lim);
    launch_ew(c, EW_MULADD, T, V, K->pk + (size_t)c->n_q * n, E1, nl, lim);
    launch_ew(c, EW_ADD, c1, c1, T, nullptr, nl, lim);
  }
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

int blb_mask_to_share(blb_ctx* c, blb_ct* cts, int n_ct, uint64_t seed, int target_level, uint64_t* share_dev) {
  if (!c || !cts || n_ct < 1 || !share_dev) return BLB_EINVAL;
  for (int t = 0; t < n_ct; ++t) {
    if (check_ct(c, &cts[t]) || cts[t].degree != 1) return BLB_EINVAL;
    if (target_level < 0 || target_level > cts[t].level) return BLB_ELEVEL;
  }
  const int n = c->n, tl = target_level + 1;
  Tmp tmp(c);
  uint64_t* r = tmp.get<uint64_t>((size_t)n_ct * tl * n);
  if (tmp.failed) return BLB_ENOMEM;
  // level drop: move c1's first tl limbs next to c0's first tl limbs
  for (int t = 0; t < n_ct; ++t) {
    const int nl = cts[t].level + 1;
    if (nl != tl) {
      uint64_t* c1tmp = tmp.get<uint64_t>((size_t)tl * n);
      if (!c1tmp) return BLB_ENOMEM;
      if (hipMemcpyAsync(c1tmp, cts[t].data + (size_t)nl * n, (size_t)tl * n * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return BLB_EDEVICE;
      if (hipMemcpyAsync(cts[t].data + (size_t)tl * n, c1tmp, (size_t)tl * n * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
        return BLB_EDEVICE;
    }
  }
  {
    Span sp(c, BLB_T_MASK, (double)n_ct * tl * n);
    launch_mask_sample(c, r, share_dev, n_ct, tl, seed, c->rec ? c->rec->param : nullptr, 6 /* mask */);
  }
  std::vector<PolyDesc> d;
  for (int t = 0; t < n_ct; ++t)
    for (int i = 0; i < tl; ++i) {
      PolyDesc x = pd(r + ((size_t)t * tl + i) * n, cts[t].data + (size_t)i * n, i, c->log_n);
      x.src2 = cts[t].data + (size_t)i * n;
      d.push_back(x);
    }
  ntt_descs(c, d, NTT_ADDTO);
  for (int t = 0; t < n_ct; ++t) cts[t].level = target_level;
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

// c0 += NTT(share) for every ciphertext: the server's step of the MPC-to-CKKS conversion
int blb_add_share(blb_ctx* c, blb_ct* cts, int n_ct, const uint64_t* share_dev) {
  if (!c || !cts || n_ct < 1 || !share_dev) return BLB_EINVAL;
  for (int t = 0; t < n_ct; ++t) {
    if (check_ct(c, &cts[t]) || cts[t].degree != 1) return BLB_EINVAL;
    if (cts[t].level != cts[0].level) return BLB_ELEVEL;
  }
  const int n = c->n, nl = cts[0].level + 1;
  std::vector<PolyDesc> d;
  for (int t = 0; t < n_ct; ++t)
    for (int i = 0; i < nl; ++i) {
      PolyDesc x = pd(share_dev + ((size_t)t * nl + i) * n, cts[t].data + (size_t)i * n, i, c->log_n);
      x.src2 = cts[t].data + (size_t)i * n;
      d.push_back(x);
    }
  {
    Span sp(c, BLB_T_MASK, (double)n_ct * nl * n);
    ntt_descs(c, d, NTT_ADDTO);
  }
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

}  // extern "C"

// ==========================================================================================
// matmul_cc (Section "Efficient Protocol for Fused MatMuls": building blocks, multi-head
// packing), diagonal-packed output
// ==========================================================================================
namespace {

// encode `count` host slot vectors (S values each) at `scale` into evaluation-form
// plaintexts out[count][level+1][N]
int encode_vectors_ntt(blb_ctx* c, const std::vector<double>& vecs, int count, double scale, int level, uint64_t* out) {
  const int S = c->n / 2, nl = level + 1, n = c->n;
  const int chunk = 256;
  Tmp tmp(c);
  double* dv = tmp.get<double>((size_t)chunk * S);
  if (tmp.failed) return BLB_ENOMEM;
  for (int p0 = 0; p0 < count; p0 += chunk) {
    const int cnt = std::min(chunk, count - p0);
    if (hipMemcpyAsync(dv, vecs.data() + (size_t)p0 * S, (size_t)cnt * S * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess)
      return BLB_EDEVICE;
    uint64_t* dst = out + (size_t)p0 * nl * n;
    int rc = encode_dense_dev(c, dv, S, cnt, scale, level, dst);
    if (rc) return rc;
    std::vector<PolyDesc> d;
    for (int p = 0; p < cnt; ++p)
      for (int i = 0; i < nl; ++i) {
        uint64_t* x = dst + ((size_t)p * nl + i) * n;
        d.push_back(pd(x, x, i, c->log_n));
      }
    ntt_descs(c, d, NTT_FWD);
  }
  return hipStreamSynchronize(c->stream) == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

}  // namespace

extern "C" {

int blb_cc_rotations_sched(const blb_ctx* c, int n_heads, int L, int32_t b_prerotated, int32_t schedule, int32_t* steps, int cap) {
  if (!c || n_heads < 1 || L < 1 || L > c->n / 2 || (schedule != 0 && schedule != 1)) return BLB_EINVAL;
  const int S = c->n / 2, lp = 1 << ceil_log2(L);
  const int Bs = 1 << ((ceil_log2(lp) + 1) / 2), G = lp / Bs;
  std::vector<int> gs;
  cc_group_sizes(n_heads, gs);
  std::vector<int32_t> v;
  if (schedule == 0) {
    for (int t = 1; t < lp; ++t) {
      v.push_back(t);
      v.push_back(-(lp - t));
    }
  } else {
    for (int i = 1; i < Bs; ++i) {  // baby inner rotations of B'
      v.push_back(i);
      v.push_back(-(lp - i));
    }
    for (int j = 1; j < G; ++j) {  // giant inner rotations of A and the postponed giant rotations
      v.push_back(lp - j * Bs);
      v.push_back(-(j * Bs));
      v.push_back(j * Bs);
      v.push_back(-(lp - j * Bs));
    }
  }
  for (int H : gs) {
    if (S % (lp * H)) return BLB_EINVAL;
    const int cc = S / (lp * H);
    for (int tau = 1; tau < cc; ++tau) v.push_back(-(tau * H * lp));
    if (schedule == 1 && !b_prerotated) {  // step 1: baby left i, giant left j b1, right L' - j b1
      const int b1 = 1 << ((ceil_log2(cc) + 1) / 2), g1 = cc / b1;
      for (int i = 1; i < b1; ++i) v.push_back(i);
      for (int j = 1; j < g1; ++j) v.push_back(j * b1);
      for (int j = 0; j < g1; ++j) v.push_back(-(lp - j * b1));
    }
  }
  std::vector<int32_t> u;
  for (int32_t x : v) {
    bool dup = false;
    for (int32_t y : u) dup |= galois_left(c, x) == galois_left(c, y);
    if (!dup) u.push_back(x);
  }
  if (steps) {
    if ((int)u.size() > cap) return BLB_EINVAL;
    memcpy(steps, u.data(), u.size() * sizeof(int32_t));
  }
  return (int)u.size();
}

int blb_cc_rotations(const blb_ctx* c, int n_heads, int L, int32_t* steps, int cap) {
  return blb_cc_rotations_sched(c, n_heads, L, 1, 0, steps, cap);
}

}  // extern "C"

// matmul_cc plan; fold_dv > 0 (Softmax x V_h): V_h has fold_dv columns, zero-padded to L', and the
// L'/c diagonal ciphertexts of each group are accumulated mod d_v'/c into d_v'/c dense outputs
static int cc_plan_create(blb_ctx* c, int n_heads, int L, int d_head, int level, int32_t b_prerotated, int fold_dv, int sched,
                          blb_plan** out) {
  if (!c || !out || n_heads < 1 || L < 1 || d_head < 1 || fold_dv < 0 || (b_prerotated != 0 && b_prerotated != 1)) return BLB_EINVAL;
  if (sched != 0 && sched != 1) return BLB_EINVAL;
  if (level < (b_prerotated ? 3 : 4) || level >= c->n_q) return BLB_EINVAL;
  *out = nullptr;
  const int S = c->n / 2, n = c->n, lp = 1 << ceil_log2(L);
  if (lp > S) return BLB_EINVAL;
  const int dvp = fold_dv > 0 ? 1 << ceil_log2(fold_dv) : lp;
  if (dvp > lp) return BLB_EINVAL;
  std::vector<int> gs;
  cc_group_sizes(n_heads, gs);
  blb_plan* P = new (std::nothrow) blb_plan();
  if (!P) return BLB_ENOMEM;
  P->ctx = c;
  P->kind = 2;
  P->level = level;
  P->hom1 = b_prerotated ? 0 : 1;
  P->heads = n_heads;
  P->L = L;
  P->d = d_head;
  P->Lp = lp;
  P->pt = nullptr;
  P->bytes = 0;
  P->sched = sched;
  {
    const int lb = ceil_log2(lp);
    P->bs_B = 1 << ((lb + 1) / 2);
    P->bs_G = lp / P->bs_B;
  }
  int ct0 = 0, out0 = 0;
  for (int H : gs) {
    if (S % (lp * H)) {
      delete P;
      return BLB_EINVAL;
    }
    CcGroup g;
    g.H = H;
    g.c = S / (lp * H);
    if (g.c > lp || g.c < 1) {
      delete P;
      return BLB_EINVAL;
    }
    g.n_ct = (d_head + g.c - 1) / g.c;
    g.n_diag = lp / g.c;
    if (g.c > dvp) {
      delete P;
      return BLB_EINVAL;
    }
    g.n_out = dvp / g.c;
    g.ct0 = ct0;
    g.out0 = out0;
    g.m_ge = g.m_lt = g.m_s1 = g.m_bs = nullptr;
    {
      const int lc = ceil_log2(g.c);
      g.b1 = 1 << ((lc + 1) / 2);
      g.g1 = g.c / g.b1;
    }
    ct0 += g.n_ct;
    out0 += g.n_out;
    P->groups.push_back(g);
  }
  P->n_ct = ct0;
  P->n_out = out0;
  int rc = BLB_OK;
  // step 1 on the server: masks at the input level, scale q_level / 2^10
  if (P->hom1) {
    for (CcGroup& g : P->groups) {
      const size_t b = (size_t)2 * g.c * (level + 1) * n * 8;
      if ((rc = dalloc(c, (void**)&g.m_s1, b))) {
        blb_plan_destroy(P);
        return rc;
      }
      P->extra.push_back(g.m_s1);
      P->extra_bytes.push_back(b);
      std::vector<double> v((size_t)2 * g.c * S, 0.0);
      for (int j = 0; j < S; ++j) {
        const int i = j % lp, cls = (j / lp) / g.H;
        if (cls == 0) v[j] = 1.0;
        else if (i < lp - cls) v[(size_t)cls * S + j] = 1.0;
        else v[(size_t)(g.c + cls) * S + j] = 1.0;
      }
      if (sched == 1) {
        // BSGS: mask kappa = j b1 + i of family 0 pre-rotated right by j b1 (slot k takes slot
        // k - j b1), of family 1 left by L' - j b1, stored at [family][j][i]
        std::vector<double> u((size_t)2 * g.c * S, 0.0);
        for (int fam = 0; fam < 2; ++fam)
          for (int jj = 0; jj < g.g1; ++jj)
            for (int ii = 0; ii < g.b1; ++ii) {
              const int kap = jj * g.b1 + ii;
              const double* src = v.data() + (size_t)(fam * g.c + kap) * S;
              double* dst = u.data() + (size_t)((fam * g.g1 + jj) * g.b1 + ii) * S;
              if (fam == 1 && kap == 0) continue;  // M^2_0 = 0
              const int64_t r = fam == 0 ? -(int64_t)jj * g.b1 : (int64_t)(lp - jj * g.b1);
              const int64_t rr = ((r % S) + S) % S;
              for (int k = 0; k < S; ++k) dst[k] = src[(k + rr) % S];
            }
        v.swap(u);
      }
      if ((rc = encode_vectors_ntt(c, v, 2 * g.c, (double)c->mod[level] / BLB_NOISE_BOOST, level, g.m_s1))) {
        blb_plan_destroy(P);
        return rc;
      }
    }
    level -= 1;  // steps 2-3 start one level down
  }
  const int nl = level + 1, nl3 = level - 1;
  // step-2 masks at `level`, scale q_level * 2^10: M^lo_t (slot mod L' < L'-t), M^hi_t, for every
  // t < L' (plain schedule) or the baby steps t < B (BSGS)
  const int n_t2 = sched ? P->bs_B : lp;
  P->bytes = (size_t)2 * n_t2 * nl * n * 8;
  rc = dalloc(c, (void**)&P->pt, P->bytes);
  if (rc) {
    delete P;
    return rc;
  }
  {
    std::vector<double> vecs((size_t)2 * n_t2 * S);
    for (int t = 0; t < n_t2; ++t)
      for (int j = 0; j < S; ++j) {
        vecs[(size_t)t * S + j] = (j % lp) < lp - t ? 1.0 : 0.0;
        vecs[(size_t)(n_t2 + t) * S + j] = (j % lp) >= lp - t ? 1.0 : 0.0;
      }
    if ((rc = encode_vectors_ntt(c, vecs, 2 * n_t2, (double)c->mod[level] * 1024.0, level, P->pt))) {
      blb_plan_destroy(P);
      return rc;
    }
  }
  // BSGS: masks of the giant inner rotations of A by t = L' - jB at `level`, scale q_level / 2^10
  if (sched) {
    const int G = P->bs_G, Bs = P->bs_B;
    const size_t b = (size_t)2 * G * nl * n * 8;
    if ((rc = dalloc(c, (void**)&P->pt_a, b))) {
      blb_plan_destroy(P);
      return rc;
    }
    P->extra.push_back(P->pt_a);
    P->extra_bytes.push_back(b);
    std::vector<double> vecs((size_t)2 * G * S, 0.0);
    for (int j = 1; j < G; ++j) {
      const int t = lp - j * Bs;
      for (int k = 0; k < S; ++k) {
        vecs[(size_t)j * S + k] = (k % lp) < lp - t ? 1.0 : 0.0;
        vecs[(size_t)(G + j) * S + k] = (k % lp) >= lp - t ? 1.0 : 0.0;
      }
    }
    if ((rc = encode_vectors_ntt(c, vecs, 2 * G, (double)c->mod[level] / BLB_NOISE_BOOST, level, P->pt_a))) {
      blb_plan_destroy(P);
      return rc;
    }
  }
  // step-3 masks per group at level-2, scale q_{level-2}: M^{>=tau}, M^{<tau} over blocks of L' H
  for (CcGroup& g : P->groups) {
    const size_t b = (size_t)g.c * nl3 * n * 8;
    if ((rc = dalloc(c, (void**)&g.m_ge, b)) || (P->extra.push_back(g.m_ge), P->extra_bytes.push_back(b), 0) ||
        (rc = dalloc(c, (void**)&g.m_lt, b)) || (P->extra.push_back(g.m_lt), P->extra_bytes.push_back(b), 0)) {
      blb_plan_destroy(P);
      return rc ? rc : BLB_ENOMEM;
    }
    const int blk = lp * g.H;
    std::vector<double> ge((size_t)g.c * S), lt((size_t)g.c * S);
    for (int tau = 0; tau < g.c; ++tau)
      for (int j = 0; j < S; ++j) {
        ge[(size_t)tau * S + j] = (j / blk) >= tau ? 1.0 : 0.0;
        lt[(size_t)tau * S + j] = (j / blk) < tau ? 1.0 : 0.0;
      }
    const double sc = (double)c->mod[level - 2] / BLB_NOISE_BOOST;
    if ((rc = encode_vectors_ntt(c, ge, g.c, sc, level - 2, g.m_ge)) || (rc = encode_vectors_ntt(c, lt, g.c, sc, level - 2, g.m_lt))) {
      blb_plan_destroy(P);
      return rc;
    }
    if (sched && P->bs_G > 1) {
      // BSGS step 3: product masks [j - 1][side * 2 + half][tau]: side 0 M^{>=tau}, 1 M^{<tau};
      // half 0 H_j (in-block position >= jB), 1 Lo_j (position < jB)
      const int G = P->bs_G, Bs = P->bs_B;
      const size_t cnt = (size_t)(G - 1) * 4 * g.c;
      const size_t bb = cnt * nl3 * n * 8;
      if ((rc = dalloc(c, (void**)&g.m_bs, bb))) {
        blb_plan_destroy(P);
        return rc;
      }
      P->extra.push_back(g.m_bs);
      P->extra_bytes.push_back(bb);
      std::vector<double> mv(cnt * S);
      for (int j = 1; j < G; ++j)
        for (int q4 = 0; q4 < 4; ++q4)
          for (int tau = 0; tau < g.c; ++tau) {
            double* dst = mv.data() + ((size_t)((j - 1) * 4 + q4) * g.c + tau) * S;
            const double* side = (q4 >> 1) == 0 ? ge.data() + (size_t)tau * S : lt.data() + (size_t)tau * S;
            for (int k = 0; k < S; ++k) {
              const bool hi = (k % lp) >= j * Bs;
              dst[k] = side[k] * (((q4 & 1) == 0) == hi ? 1.0 : 0.0);
            }
          }
      if ((rc = encode_vectors_ntt(c, mv, (int)cnt, sc, level - 2, g.m_bs))) {
        blb_plan_destroy(P);
        return rc;
      }
    }
  }
  *out = P;
  return BLB_OK;
}

extern "C" {

int blb_plan_matmul_cc(blb_ctx* c, int n_heads, int L, int d_head, int level, int32_t b_prerotated, blb_plan** out) {
  return cc_plan_create(c, n_heads, L, d_head, level, b_prerotated, 0, 0, out);
}

int blb_plan_matmul_cc_sv(blb_ctx* c, int n_heads, int L, int d_v, int level, int32_t b_prerotated, blb_plan** out) {
  if (d_v < 1) return BLB_EINVAL;
  return cc_plan_create(c, n_heads, L, L, level, b_prerotated, d_v, 0, out);
}

int blb_plan_matmul_cc_sched(blb_ctx* c, int n_heads, int L, int d_head, int level, int32_t b_prerotated, int32_t schedule,
                             blb_plan** out) {
  return cc_plan_create(c, n_heads, L, d_head, level, b_prerotated, 0, schedule, out);
}

int blb_plan_matmul_cc_sv_sched(blb_ctx* c, int n_heads, int L, int d_v, int level, int32_t b_prerotated, int32_t schedule,
                                blb_plan** out) {
  if (d_v < 1) return BLB_EINVAL;
  return cc_plan_create(c, n_heads, L, L, level, b_prerotated, d_v, schedule, out);
}

int blb_plan_cc_info(const blb_plan* P, int32_t* info, int cap) {
  if (!P || P->kind != 2) return BLB_EINVAL;
  const int ng = (int)P->groups.size();
  if (info) {
    if (cap < 3 + 5 * ng) return BLB_EINVAL;
    info[0] = P->Lp;
    info[1] = P->n_ct;
    info[2] = P->n_out;
    for (int i = 0; i < ng; ++i) {
      const CcGroup& g = P->groups[i];
      info[3 + 5 * i + 0] = g.H;
      info[3 + 5 * i + 1] = g.c;
      info[3 + 5 * i + 2] = g.n_ct;
      info[3 + 5 * i + 3] = g.n_out;
      info[3 + 5 * i + 4] = g.ct0;
    }
  }
  return ng;
}

}  // extern "C"

namespace {

const SwKey* key_for(blb_ctx* c, const blb_keys* K, int64_t steps) { return find_key(K, galois_left(c, steps)); }

// Rotation request of source `src` (a whole ciphertext at `ct`, its c1 being the source poly):
// dst = (sigma(c0) + KS_0, KS_1)
KsReq rot_req(blb_ctx* c, const blb_keys* K, int src, int64_t steps, const uint64_t* ct, uint64_t* dst) {
  const uint32_t gal = galois_left(c, steps);
  return KsReq{src, key_for(c, K, steps), gal, dst, ct, gal, nullptr};
}

// Step 1 with BSGS for one head group (m = g.n_ct ciphertexts B_a at level_in, [2][level_in+1][N]):
// with kappa = j b1 + i and B''_a = 2^10 B_a,
//   B'_a = Rescale( sum_j Rot_l^{j b1}( sum_i Rot_l^i(B'') (.) Rot_r^{j b1}(M^1_kappa) )
//                 + sum_j Rot_r^{L' - j b1}( sum_i Rot_l^i(B'') (.) Rot_l^{L' - j b1}(M^2_kappa) ) ),
// the baby rotations Rot_l^i(B'') hoisted and shared by both families; Bq gets [m][2][level_in][N].
int cc_step1_bsgs_dev(blb_ctx* c, const blb_keys* K, const blb_plan* P, const CcGroup& g, const blb_ct* Bin, int level_in,
                      uint64_t* Bq) {
  const int m = g.n_ct, n = c->n, lp = P->Lp, b1 = g.b1, g1 = g.g1;
  const int nl0 = level_in + 1;
  const size_t w0 = (size_t)2 * nl0 * n;
  Tmp tmp(c);
  uint64_t* B0 = tmp.get<uint64_t>((size_t)m * w0);
  uint64_t* X0 = tmp.get<uint64_t>(ks_modup_words(c, level_in, m));
  uint64_t* XB = tmp.get<uint64_t>((size_t)(b1 - 1) * m * w0 + 1);
  uint64_t* Pp = tmp.get<uint64_t>((size_t)m * g1 * 2 * w0);
  uint64_t* PR = tmp.get<uint64_t>((size_t)m * g1 * 2 * w0);
  uint64_t* S0 = tmp.get<uint64_t>((size_t)m * w0);
  if (tmp.failed) return BLB_ENOMEM;
  std::vector<const uint64_t*> bin;
  for (int a = 0; a < m; ++a) bin.push_back(Bin[g.ct0 + a].data);
  const uint64_t* const* bin_dev = upload_vec(c, bin);
  if (!bin_dev) return BLB_EDEVICE;
  launch_scale_cts(c, bin_dev, B0, m, nl0, BLB_NOISE_BOOST);
  int rc;
  std::vector<const uint64_t*> srcs0;
  for (int a = 0; a < m; ++a) srcs0.push_back(B0 + (size_t)a * w0 + (size_t)nl0 * n);
  std::vector<KsReq> baby;
  for (int i = 1; i < b1; ++i)
    for (int a = 0; a < m; ++a) baby.push_back(rot_req(c, K, a, i, B0 + (size_t)a * w0, XB + ((size_t)(i - 1) * m + a) * w0));
  if (!baby.empty()) {
    if ((rc = ks_modup(c, level_in, srcs0, X0))) return rc;
    if ((rc = ks_apply(c, level_in, srcs0, X0, baby))) return rc;
  }
  // partial sums [a][j][family]
  std::vector<CcTerm> terms;
  std::vector<int> off{0};
  std::vector<uint64_t*> outs;
  std::vector<int> has((size_t)m * g1 * 2, 0);
  for (int a = 0; a < m; ++a)
    for (int j = 0; j < g1; ++j)
      for (int fam = 0; fam < 2; ++fam) {
        const size_t before = terms.size();
        for (int i = 0; i < b1; ++i) {
          if (fam == 1 && j == 0 && i == 0) continue;  // M^2_0 = 0
          const uint64_t* x = i == 0 ? B0 + (size_t)a * w0 : XB + ((size_t)(i - 1) * m + a) * w0;
          terms.push_back(CcTerm{x, g.m_s1 + (size_t)((fam * g1 + j) * b1 + i) * nl0 * n});
        }
        if (terms.size() == before) continue;
        has[((size_t)a * g1 + j) * 2 + fam] = 1;
        off.push_back((int)terms.size());
        outs.push_back(Pp + (((size_t)a * g1 + j) * 2 + fam) * w0);
      }
  {
    const CcTerm* terms_dev = upload_vec(c, terms);
    const int* off_dev = upload_vec(c, off);
    uint64_t* const* outs_dev = (uint64_t* const*)upload(c, outs.data(), outs.size() * sizeof(uint64_t*));
    if (!terms_dev || !off_dev || !outs_dev) return BLB_EDEVICE;
    Span sp(c, BLB_T_EW, (double)outs.size() * w0);
    c->counters[2] += (int64_t)terms.size();
    launch_masked_acc(c, terms_dev, off_dev, outs_dev, (int)outs.size(), nl0, false);
  }
  // giant rotations of the partial sums (each its own source), then B' = Rescale(sum)
  std::vector<const uint64_t*> gsrc;
  std::vector<KsReq> greq;
  std::vector<const uint64_t*> sum_src;
  std::vector<int> sum_off{0};
  std::vector<uint64_t*> sum_dst;
  for (int a = 0; a < m; ++a) {
    for (int j = 0; j < g1; ++j)
      for (int fam = 0; fam < 2; ++fam) {
        const size_t k = ((size_t)a * g1 + j) * 2 + fam;
        if (!has[k]) continue;
        uint64_t* part = Pp + k * w0;
        if (fam == 0 && j == 0) {
          sum_src.push_back(part);
          continue;
        }
        const int64_t steps = fam == 0 ? (int64_t)j * b1 : -(int64_t)(lp - j * b1);
        gsrc.push_back(part + (size_t)nl0 * n);
        greq.push_back(rot_req(c, K, (int)gsrc.size() - 1, steps, part, PR + k * w0));
        sum_src.push_back(PR + k * w0);
      }
    sum_off.push_back((int)sum_src.size());
    sum_dst.push_back(S0 + (size_t)a * w0);
  }
  if ((rc = ks_batch(c, level_in, gsrc, greq))) return rc;
  {
    const uint64_t* const* s_dev = upload_vec(c, sum_src);
    const int* o_dev = upload_vec(c, sum_off);
    uint64_t* const* d_dev = (uint64_t* const*)upload(c, sum_dst.data(), sum_dst.size() * sizeof(uint64_t*));
    if (!s_dev || !o_dev || !d_dev) return BLB_EDEVICE;
    Span sp(c, BLB_T_EW, (double)m * w0);
    launch_sum_var(c, s_dev, o_dev, d_dev, m, nl0);
  }
  std::vector<const uint64_t*> rin;
  std::vector<uint64_t*> rout;
  for (int a = 0; a < m; ++a) {
    rin.push_back(S0 + (size_t)a * w0);
    rout.push_back(Bq + (size_t)a * 2 * level_in * n);
  }
  return rescale_batch(c, level_in, 2, rin, rout);
}

// Steps 2-3 with BSGS for one head group: A_a (a_nl limbs per poly, used through its first
// level + 1) and B'_a (compact, level + 1 limbs) at `level`; with t = j B + i,
//   Y_{a,i}  = Rescale(InnerRot_i(2^10 B'_a))          (baby steps; masks q_level 2^10)
//   A'_{a,j} = Rescale(InnerRot_{L'-jB}(2^10 A_a))      (giant steps, j >= 1; masks q_level / 2^10), Drop(A_a) for j = 0
//   U_t = Rescale(Relin(sum_a A'_{a,j} (x) Y_{a,i})),  V_t = Rot_r^{tau H L'}(U_t)
// step 3: j = 0 terms go to O_g / O_{g+1} with M^{>=tau} / M^{<tau}; j >= 1 terms go to the
// accumulators (g, j, half) with the product masks, which are rotated by the postponed giant step
// (half H_j left by jB, half Lo_j right by L' - jB) and added to O_g; outputs = Rescale(O_g).
int cc_steps23_bsgs_dev(blb_ctx* c, const blb_keys* K, const blb_plan* P, const CcGroup& g, const std::vector<const uint64_t*>& asrc,
                        int a_nl, const std::vector<const uint64_t*>& bsrc, int level, const blb_ct* Cd) {
  const int m = g.n_ct, n = c->n, lp = P->Lp, Bb = P->bs_B, G = P->bs_G;
  const int nl = level + 1, nl2 = level, nl3 = level - 1;
  const size_t w1 = (size_t)2 * nl * n, w2 = (size_t)2 * nl2 * n, w3 = (size_t)2 * nl3 * n;
  const int TC = std::min(lp, 128);
  Tmp tmp(c);
  uint64_t* Bs = tmp.get<uint64_t>((size_t)m * w1);
  uint64_t* As = tmp.get<uint64_t>((size_t)m * w1);
  uint64_t* X = tmp.get<uint64_t>(ks_modup_words(c, level, 2 * m));
  uint64_t* RL = tmp.get<uint64_t>((size_t)(Bb - 1) * m * w1 + 1);
  uint64_t* RR = tmp.get<uint64_t>((size_t)(Bb - 1) * m * w1 + 1);
  uint64_t* GL = tmp.get<uint64_t>((size_t)(G - 1) * m * w1 + 1);
  uint64_t* GR = tmp.get<uint64_t>((size_t)(G - 1) * m * w1 + 1);
  uint64_t* Pre = tmp.get<uint64_t>((size_t)(Bb + G - 1) * m * w1);
  uint64_t* Y = tmp.get<uint64_t>((size_t)Bb * m * w2);
  uint64_t* Ap = tmp.get<uint64_t>((size_t)G * m * w2);
  uint64_t* Oacc = tmp.get<uint64_t>((size_t)g.n_out * w3);
  uint64_t* Acc = tmp.get<uint64_t>((size_t)g.n_out * (G - 1) * 2 * w3 + 1);
  uint64_t* F = tmp.get<uint64_t>((size_t)g.n_out * (G - 1) * 2 * w3 + 1);
  uint64_t* T3 = tmp.get<uint64_t>((size_t)TC * 3 * nl2 * n);
  uint64_t* Trl = tmp.get<uint64_t>((size_t)TC * w2);
  uint64_t* T = tmp.get<uint64_t>((size_t)TC * w3);
  uint64_t* V = tmp.get<uint64_t>((size_t)TC * w3);
  if (tmp.failed) return BLB_ENOMEM;
  int rc;
  {
    const uint64_t* const* b_dev = upload_vec(c, bsrc);
    const uint64_t* const* a_dev = upload_vec(c, asrc);
    if (!b_dev || !a_dev) return BLB_EDEVICE;
    launch_scale_cts(c, b_dev, Bs, m, nl, BLB_NOISE_BOOST);
    launch_scale_cts(c, a_dev, As, m, nl, BLB_NOISE_BOOST, a_nl);
    launch_scale_cts(c, a_dev, Ap, m, nl2, 1.0, a_nl);  // A'_{a,0} = Drop(A_a)
  }
  launch_zero(c, Oacc, (size_t)g.n_out * w3);
  if (G > 1) launch_zero(c, Acc, (size_t)g.n_out * (G - 1) * 2 * w3);
  // hoisted baby rotations of B' and giant rotations of A, one ModUp for both
  std::vector<const uint64_t*> srcs;
  for (int a = 0; a < m; ++a) srcs.push_back(Bs + (size_t)a * w1 + (size_t)nl * n);
  for (int a = 0; a < m; ++a) srcs.push_back(As + (size_t)a * w1 + (size_t)nl * n);
  std::vector<KsReq> reqs;
  for (int i = 1; i < Bb; ++i)
    for (int a = 0; a < m; ++a) {
      const size_t k = (size_t)(i - 1) * m + a;
      reqs.push_back(rot_req(c, K, a, i, Bs + (size_t)a * w1, RL + k * w1));
      reqs.push_back(rot_req(c, K, a, -(int64_t)(lp - i), Bs + (size_t)a * w1, RR + k * w1));
    }
  for (int j = 1; j < G; ++j)
    for (int a = 0; a < m; ++a) {
      const size_t k = (size_t)(j - 1) * m + a;
      reqs.push_back(rot_req(c, K, m + a, lp - j * Bb, As + (size_t)a * w1, GL + k * w1));
      reqs.push_back(rot_req(c, K, m + a, -(int64_t)(j * Bb), As + (size_t)a * w1, GR + k * w1));
    }
  if (!reqs.empty()) {
    if ((rc = ks_modup(c, level, srcs, X))) return rc;
    if ((rc = ks_apply(c, level, srcs, X, reqs))) return rc;
  }
  // masks, then one rescale batch: Y [i][a] and A' [j][a] (j >= 1)
  std::vector<CcPair> pairs;
  std::vector<const uint64_t*> rin;
  std::vector<uint64_t*> rout;
  for (int i = 0; i < Bb; ++i)
    for (int a = 0; a < m; ++a) {
      const size_t k = (size_t)i * m + a;
      CcPair pr;
      pr.mx = P->pt + (size_t)i * nl * n;
      pr.my = P->pt + (size_t)(Bb + i) * nl * n;
      pr.out = Pre + k * w1;
      if (i == 0) {
        pr.x = Bs + (size_t)a * w1;
        pr.y = nullptr;
      } else {
        pr.x = RL + ((size_t)(i - 1) * m + a) * w1;
        pr.y = RR + ((size_t)(i - 1) * m + a) * w1;
      }
      pairs.push_back(pr);
      rin.push_back(Pre + k * w1);
      rout.push_back(Y + k * w2);
    }
  for (int j = 1; j < G; ++j)
    for (int a = 0; a < m; ++a) {
      const size_t k = (size_t)(Bb + j - 1) * m + a, kg = (size_t)(j - 1) * m + a;
      CcPair pr;
      pr.mx = P->pt_a + (size_t)j * nl * n;
      pr.my = P->pt_a + (size_t)(G + j) * nl * n;
      pr.x = GL + kg * w1;
      pr.y = GR + kg * w1;
      pr.out = Pre + k * w1;
      pairs.push_back(pr);
      rin.push_back(Pre + k * w1);
      rout.push_back(Ap + ((size_t)j * m + a) * w2);
    }
  {
    const CcPair* pairs_dev = upload_vec(c, pairs);
    if (!pairs_dev) return BLB_EDEVICE;
    Span sp(c, BLB_T_EW, (double)pairs.size() * w1);
    for (const CcPair& pr : pairs) c->counters[2] += pr.y ? 2 : 1;
    launch_mask_pair(c, pairs_dev, (int)pairs.size(), nl);
  }
  if ((rc = rescale_batch(c, level, 2, rin, rout))) return rc;
  // accumulator index of (output o, giant step j >= 1, half)
  auto acc_idx = [&](int o, int j, int half) { return ((size_t)o * (G - 1) + (j - 1)) * 2 + half; };
  std::vector<char> used((size_t)g.n_out * (G > 1 ? G - 1 : 0) * 2, 0);
  for (int t0 = 0; t0 < lp; t0 += TC) {
    const int nt = std::min(TC, lp - t0);
    std::vector<const uint64_t*> a_tab, r_tab;
    for (int tt = 0; tt < nt; ++tt) {
      const int t = t0 + tt, j = t / Bb, i = t % Bb;
      for (int a = 0; a < m; ++a) {
        a_tab.push_back(Ap + ((size_t)j * m + a) * w2);
        r_tab.push_back(Y + ((size_t)i * m + a) * w2);
      }
    }
    {
      const uint64_t* const* a_dev = upload_vec(c, a_tab);
      const uint64_t* const* r_dev = upload_vec(c, r_tab);
      if (!a_dev || !r_dev) return BLB_EDEVICE;
      Span sp(c, BLB_T_CC_TENSOR, (double)nt * nl2 * n);
      c->counters[3] += (int64_t)nt * m;
      c->counters[4] += nt;
      launch_tensor_sum(c, a_dev, r_dev, T3, nt, m, nl2, nl2, true);
    }
    std::vector<const uint64_t*> rs;
    std::vector<KsReq> rr;
    const SwKey* relin = find_key(K, 0);
    for (int tt = 0; tt < nt; ++tt) {
      const uint64_t* t3 = T3 + (size_t)tt * 3 * nl2 * n;
      rs.push_back(t3 + (size_t)2 * nl2 * n);
      rr.push_back(KsReq{tt, relin, 0, Trl + (size_t)tt * w2, t3, 0, t3 + (size_t)nl2 * n});
    }
    if ((rc = ks_batch(c, level - 1, rs, rr))) return rc;
    rin.clear();
    rout.clear();
    for (int tt = 0; tt < nt; ++tt) {
      rin.push_back(Trl + (size_t)tt * w2);
      rout.push_back(T + (size_t)tt * w3);
    }
    if ((rc = rescale_batch(c, level - 1, 2, rin, rout))) return rc;
    std::vector<const uint64_t*> vs;
    std::vector<KsReq> vr;
    std::vector<const uint64_t*> vsrc(nt);
    for (int tt = 0; tt < nt; ++tt) {
      const int t = t0 + tt, tau = t % g.c;
      const uint64_t* tp = T + (size_t)tt * w3;
      if (tau == 0) {
        vsrc[tt] = tp;
        continue;
      }
      vs.push_back(tp + (size_t)nl3 * n);
      vr.push_back(rot_req(c, K, (int)vs.size() - 1, -(int64_t)tau * g.H * lp, tp, V + (size_t)tt * w3));
      vsrc[tt] = V + (size_t)tt * w3;
    }
    if ((rc = ks_batch(c, level - 2, vs, vr))) return rc;
    // step 3 masks into O_g (j = 0) or the giant-step accumulators (j >= 1)
    const size_t n_acc = (size_t)g.n_out * (1 + (G > 1 ? (G - 1) * 2 : 0));
    std::vector<std::vector<CcTerm>> per(n_acc);
    auto slot_of = [&](int o, int j, int half) -> size_t { return j == 0 ? (size_t)o : g.n_out + acc_idx(o, j, half); };
    for (int tt = 0; tt < nt; ++tt) {
      const int t = t0 + tt, gi = t / g.c, tau = t % g.c, j = t / Bb;
      const int o_ge = gi % g.n_out, o_lt = ((gi + 1) % g.n_diag) % g.n_out;
      if (j == 0) {
        per[o_ge].push_back(CcTerm{vsrc[tt], g.m_ge + (size_t)tau * nl3 * n});
        if (tau > 0) per[o_lt].push_back(CcTerm{vsrc[tt], g.m_lt + (size_t)tau * nl3 * n});
        continue;
      }
      for (int half = 0; half < 2; ++half) {
        per[slot_of(o_ge, j, half)].push_back(CcTerm{vsrc[tt], g.m_bs + ((size_t)((j - 1) * 4 + half) * g.c + tau) * nl3 * n});
        used[acc_idx(o_ge, j, half)] = 1;
        if (tau > 0) {
          per[slot_of(o_lt, j, half)].push_back(CcTerm{vsrc[tt], g.m_bs + ((size_t)((j - 1) * 4 + 2 + half) * g.c + tau) * nl3 * n});
          used[acc_idx(o_lt, j, half)] = 1;
        }
      }
    }
    std::vector<CcTerm> terms;
    std::vector<int> off{0};
    std::vector<uint64_t*> outs;
    for (size_t k = 0; k < n_acc; ++k) {
      if (per[k].empty()) continue;
      terms.insert(terms.end(), per[k].begin(), per[k].end());
      off.push_back((int)terms.size());
      outs.push_back(k < (size_t)g.n_out ? Oacc + k * w3 : Acc + (k - g.n_out) * w3);
    }
    const CcTerm* terms_dev = upload_vec(c, terms);
    const int* off_dev = upload_vec(c, off);
    uint64_t* const* outs_dev = (uint64_t* const*)upload(c, outs.data(), outs.size() * sizeof(uint64_t*));
    if (!terms_dev || !off_dev || !outs_dev) return BLB_EDEVICE;
    Span sp(c, BLB_T_EW, (double)outs.size() * w3);
    c->counters[2] += (int64_t)terms.size();
    launch_masked_acc(c, terms_dev, off_dev, outs_dev, (int)outs.size(), nl3, true);
  }
  // the postponed giant rotations, then O_g += their sum and the final rescale
  std::vector<const uint64_t*> fsrc;
  std::vector<KsReq> freq;
  std::vector<std::vector<const uint64_t*>> add(g.n_out);
  for (int o = 0; o < g.n_out; ++o) {
    add[o].push_back(Oacc + (size_t)o * w3);
    for (int j = 1; j < G; ++j)
      for (int half = 0; half < 2; ++half) {
        const size_t k = acc_idx(o, j, half);
        if (!used[k]) continue;
        const uint64_t* accp = Acc + k * w3;
        const int64_t steps = half == 0 ? (int64_t)j * Bb : -(int64_t)(lp - j * Bb);
        fsrc.push_back(accp + (size_t)nl3 * n);
        freq.push_back(rot_req(c, K, (int)fsrc.size() - 1, steps, accp, F + k * w3));
        add[o].push_back(F + k * w3);
      }
  }
  if ((rc = ks_batch(c, level - 2, fsrc, freq))) return rc;
  if (!fsrc.empty()) {
    std::vector<const uint64_t*> ssrc;
    std::vector<int> soff{0};
    std::vector<uint64_t*> sdst;
    for (int o = 0; o < g.n_out; ++o) {
      ssrc.insert(ssrc.end(), add[o].begin(), add[o].end());
      soff.push_back((int)ssrc.size());
      sdst.push_back(Oacc + (size_t)o * w3);
    }
    const uint64_t* const* s_dev = upload_vec(c, ssrc);
    const int* o_dev = upload_vec(c, soff);
    uint64_t* const* d_dev = (uint64_t* const*)upload(c, sdst.data(), sdst.size() * sizeof(uint64_t*));
    if (!s_dev || !o_dev || !d_dev) return BLB_EDEVICE;
    Span sp(c, BLB_T_EW, (double)g.n_out * w3);
    launch_sum_var(c, s_dev, o_dev, d_dev, g.n_out, nl3);
  }
  std::vector<const uint64_t*> oin;
  std::vector<uint64_t*> oout;
  for (int o = 0; o < g.n_out; ++o) {
    oin.push_back(Oacc + (size_t)o * w3);
    oout.push_back(Cd[g.out0 + o].data);
  }
  return rescale_batch(c, level - 2, 2, oin, oout);
}

}  // namespace

extern "C" {

int blb_matmul_cc(blb_ctx* c, const blb_keys* K, const blb_plan* P, const blb_ct* A, const blb_ct* Bp, int n_ct, blb_ct* Cd, int n_out) {
  if (!c || !K || !P || !A || !Bp || !Cd || P->kind != 2) return BLB_EINVAL;
  if (n_ct != P->n_ct || n_out != P->n_out) return BLB_EINVAL;
  const int level_in = P->level, level = P->level - P->hom1, n = c->n, lp = P->Lp;
  for (int a = 0; a < n_ct; ++a) {
    if (check_ct(c, &A[a]) || check_ct(c, &Bp[a]) || A[a].degree != 1 || Bp[a].degree != 1) return BLB_EINVAL;
    if (A[a].level != level_in || Bp[a].level != level_in) return BLB_ELEVEL;
    if (fabs(A[a].scale / A[0].scale - 1.0) > 1e-9 || fabs(Bp[a].scale / Bp[0].scale - 1.0) > 1e-9) return BLB_ESCALE;
  }
  for (int o = 0; o < n_out; ++o)
    if (!Cd[o].data) return BLB_EINVAL;
  const SwKey* relin = find_key(K, 0);
  if (!relin) return BLB_ENOKEY;
  std::vector<const SwKey*> kl(lp, nullptr), kr(lp, nullptr);
  {
    const int nk = blb_cc_rotations_sched(c, P->heads, P->L, P->hom1 ? 0 : 1, P->sched, nullptr, 0);
    if (nk < 0) return BLB_EINVAL;
    std::vector<int32_t> st(nk);
    if (blb_cc_rotations_sched(c, P->heads, P->L, P->hom1 ? 0 : 1, P->sched, st.data(), nk) < 0) return BLB_EINVAL;
    for (int32_t x : st)
      if (!find_key(K, galois_left(c, x))) return BLB_ENOKEY;
  }
  if (P->sched == 0)
    for (int t = 1; t < lp; ++t) {
      kl[t] = find_key(K, galois_left(c, t));
      kr[t] = find_key(K, galois_left(c, -(lp - t)));
    }
  const int nl = level + 1, nl2 = level, nl3 = level - 1, nlA = level_in + 1;
  const size_t w1 = (size_t)2 * nl * n, w2 = (size_t)2 * nl2 * n, w3 = (size_t)2 * nl3 * n;
  // t values per chunk: large chunks give every stage launch hundreds of limb-polys (the
  // relinearisation and step-3 stages only have one ciphertext per t); about 40 MB per t
  const int TC = std::min(lp, 128);
  int rc = BLB_OK;
  double b_scale = Bp[0].scale;
  for (const CcGroup& g : P->groups) {
    const int m = g.n_ct;
    if (P->sched == 1) {
      Tmp tmp(c);
      std::vector<const uint64_t*> asrc, bsrc;
      for (int a = 0; a < m; ++a) {
        asrc.push_back(A[g.ct0 + a].data);
        bsrc.push_back(Bp[g.ct0 + a].data);
      }
      if (P->hom1) {
        uint64_t* Bq = tmp.get<uint64_t>((size_t)m * w1);
        if (tmp.failed) return BLB_ENOMEM;
        if ((rc = cc_step1_bsgs_dev(c, K, P, g, Bp, level_in, Bq))) return rc;
        for (int a = 0; a < m; ++a) bsrc[a] = Bq + (size_t)a * w1;
      }
      if ((rc = cc_steps23_bsgs_dev(c, K, P, g, asrc, nlA, bsrc, level, Cd))) return rc;
      continue;
    }
    Tmp tmp(c);
    // step 1 on the server: B'_a = Rescale(sum of the masked rotations of 2^10 B_a)
    std::vector<const uint64_t*> bsrc;
    for (int a = 0; a < m; ++a) bsrc.push_back(Bp[g.ct0 + a].data);
    if (P->hom1) {
      const int nl0 = level_in + 1;
      const size_t w0 = (size_t)2 * nl0 * n;
      uint64_t* B0 = tmp.get<uint64_t>((size_t)m * w0);
      uint64_t* X0 = tmp.get<uint64_t>(ks_modup_words(c, level_in, m));
      uint64_t* R0 = tmp.get<uint64_t>((size_t)2 * (g.c - 1) * m * w0 + 1);
      uint64_t* S0 = tmp.get<uint64_t>((size_t)m * w0);
      uint64_t* Bq = tmp.get<uint64_t>((size_t)m * w1);
      if (tmp.failed) return BLB_ENOMEM;
      {
        const uint64_t* const* bin_dev = upload_vec(c, bsrc);
        if (!bin_dev) return BLB_EDEVICE;
        launch_scale_cts(c, bin_dev, B0, m, nl0, BLB_NOISE_BOOST);
      }
      std::vector<const uint64_t*> srcs0;
      for (int a = 0; a < m; ++a) srcs0.push_back(B0 + (size_t)a * w0 + (size_t)nl0 * n);
      if ((rc = ks_modup(c, level_in, srcs0, X0))) return rc;
      std::vector<KsReq> reqs0;
      std::vector<CcTerm> terms0;
      std::vector<int> off0{0};
      std::vector<uint64_t*> outs0;
      for (int a = 0; a < m; ++a) {
        const uint64_t* b = B0 + (size_t)a * w0;
        terms0.push_back(CcTerm{b, g.m_s1});
        for (int kap = 1; kap < g.c; ++kap) {
          uint64_t* rl = R0 + ((size_t)(2 * (kap - 1)) * m + a) * w0;
          uint64_t* rr = R0 + ((size_t)(2 * (kap - 1) + 1) * m + a) * w0;
          const uint32_t gl = galois_left(c, kap), gr = galois_left(c, -(int64_t)(lp - kap));
          reqs0.push_back(KsReq{a, kl[kap], gl, rl, b, gl, nullptr});
          reqs0.push_back(KsReq{a, kr[kap], gr, rr, b, gr, nullptr});
          terms0.push_back(CcTerm{rl, g.m_s1 + (size_t)kap * nl0 * n});
          terms0.push_back(CcTerm{rr, g.m_s1 + (size_t)(g.c + kap) * nl0 * n});
        }
        off0.push_back((int)terms0.size());
        outs0.push_back(S0 + (size_t)a * w0);
      }
      if (!reqs0.empty() && (rc = ks_apply(c, level_in, srcs0, X0, reqs0))) return rc;
      const CcTerm* terms_dev = upload_vec(c, terms0);
      const int* off_dev = upload_vec(c, off0);
      uint64_t* const* outs_dev = (uint64_t* const*)upload(c, outs0.data(), outs0.size() * sizeof(uint64_t*));
      if (!terms_dev || !off_dev || !outs_dev) return BLB_EDEVICE;
      {
        Span sp(c, BLB_T_EW, (double)m * w0);
        c->counters[2] += (int64_t)terms0.size();
        launch_masked_acc(c, terms_dev, off_dev, outs_dev, m, nl0, false);
      }
      std::vector<const uint64_t*> rin;
      std::vector<uint64_t*> rout;
      for (int a = 0; a < m; ++a) {
        rin.push_back(S0 + (size_t)a * w0);
        rout.push_back(Bq + (size_t)a * w1);
        bsrc[a] = Bq + (size_t)a * w1;
      }
      if ((rc = rescale_batch(c, level_in, 2, rin, rout))) return rc;
    }
    // noise boost: Bs_a = 2^10 B'_a before the inner rotations (step-3 masks are at q/2^10)
    uint64_t* Bs = tmp.get<uint64_t>((size_t)m * w1);
    if (!Bs) return BLB_ENOMEM;
    {
      std::vector<const uint64_t*> bin = bsrc;
      const uint64_t* const* bin_dev = upload_vec(c, bin);
      if (!bin_dev) return BLB_EDEVICE;
      launch_scale_cts(c, bin_dev, Bs, m, nl, BLB_NOISE_BOOST);
    }
    std::vector<const uint64_t*> srcs;
    for (int a = 0; a < m; ++a) srcs.push_back(Bs + (size_t)a * w1 + (size_t)nl * n);
    uint64_t* X = tmp.get<uint64_t>(ks_modup_words(c, level, m));
    uint64_t* Oacc = tmp.get<uint64_t>((size_t)g.n_out * w3);
    uint64_t* RL = tmp.get<uint64_t>((size_t)TC * m * w1);
    uint64_t* RR = tmp.get<uint64_t>((size_t)TC * m * w1);
    uint64_t* Rpre = tmp.get<uint64_t>((size_t)TC * m * w1);
    uint64_t* R = tmp.get<uint64_t>((size_t)TC * m * w2);
    uint64_t* T3 = tmp.get<uint64_t>((size_t)TC * 3 * nl2 * n);
    uint64_t* Trl = tmp.get<uint64_t>((size_t)TC * w2);
    uint64_t* T = tmp.get<uint64_t>((size_t)TC * w3);
    uint64_t* V = tmp.get<uint64_t>((size_t)TC * w3);
    if (tmp.failed) return BLB_ENOMEM;
    launch_zero(c, Oacc, (size_t)g.n_out * w3);
    if ((rc = ks_modup(c, level, srcs, X))) return rc;
    std::vector<const uint64_t*> a_tab;
    for (int a = 0; a < m; ++a) a_tab.push_back(A[g.ct0 + a].data);
    const uint64_t* const* a_dev = upload_vec(c, a_tab);
    if (!a_dev) return BLB_EDEVICE;
    for (int t0 = 0; t0 < lp; t0 += TC) {
      const int nt = std::min(TC, lp - t0);
      // step 2: inner rotations of every B'_a by t (two hoisted rotations, then masks)
      std::vector<KsReq> reqs;
      std::vector<CcPair> pairs;
      for (int tt = 0; tt < nt; ++tt) {
        const int t = t0 + tt;
        for (int a = 0; a < m; ++a) {
          const size_t slot = (size_t)tt * m + a;
          const uint64_t* b = Bs + (size_t)a * w1;
          CcPair pr;
          pr.mx = P->pt + (size_t)t * nl * n;
          pr.my = P->pt + (size_t)(lp + t) * nl * n;
          pr.out = Rpre + slot * w1;
          if (t == 0) {
            pr.x = b;
            pr.y = nullptr;
          } else {
            const uint32_t gl = galois_left(c, t), gr = galois_left(c, -(lp - t));
            reqs.push_back(KsReq{a, kl[t], gl, RL + slot * w1, b, gl, nullptr});
            reqs.push_back(KsReq{a, kr[t], gr, RR + slot * w1, b, gr, nullptr});
            pr.x = RL + slot * w1;
            pr.y = RR + slot * w1;
          }
          pairs.push_back(pr);
        }
      }
      if ((rc = ks_apply(c, level, srcs, X, reqs))) return rc;
      const CcPair* pairs_dev = upload_vec(c, pairs);
      if (!pairs_dev) return BLB_EDEVICE;
      {
        Span sp(c, BLB_T_EW, (double)pairs.size() * w1);
        for (const CcPair& pr : pairs) c->counters[2] += pr.y ? 2 : 1;
        launch_mask_pair(c, pairs_dev, (int)pairs.size(), nl);
      }
      std::vector<const uint64_t*> rin;
      std::vector<uint64_t*> rout;
      std::vector<const uint64_t*> r_tab;
      for (int i = 0; i < nt * m; ++i) {
        rin.push_back(Rpre + (size_t)i * w1);
        rout.push_back(R + (size_t)i * w2);
        r_tab.push_back(R + (size_t)i * w2);
      }
      if ((rc = rescale_batch(c, level, 2, rin, rout))) return rc;
      // tensor with A (dropped one level) summed over a, one relinearisation per t
      const uint64_t* const* r_dev = upload_vec(c, r_tab);
      if (!r_dev) return BLB_EDEVICE;
      {
        Span sp(c, BLB_T_CC_TENSOR, (double)nt * nl2 * n);
        c->counters[3] += (int64_t)nt * m;
        c->counters[4] += nt;
        launch_tensor_sum(c, a_dev, r_dev, T3, nt, m, nlA, nl2);
      }
      std::vector<const uint64_t*> rs;
      std::vector<KsReq> rr;
      for (int tt = 0; tt < nt; ++tt) {
        const uint64_t* t3 = T3 + (size_t)tt * 3 * nl2 * n;
        rs.push_back(t3 + (size_t)2 * nl2 * n);
        rr.push_back(KsReq{tt, relin, 0, Trl + (size_t)tt * w2, t3, 0, t3 + (size_t)nl2 * n});
      }
      if ((rc = ks_batch(c, level - 1, rs, rr))) return rc;
      rin.clear();
      rout.clear();
      for (int tt = 0; tt < nt; ++tt) {
        rin.push_back(Trl + (size_t)tt * w2);
        rout.push_back(T + (size_t)tt * w3);
      }
      if ((rc = rescale_batch(c, level - 1, 2, rin, rout))) return rc;
      // step 3: rotate T_t right by tau blocks (t = g c + tau), split masks into O_g, O_{g+1}
      std::vector<const uint64_t*> vs;
      std::vector<KsReq> vr;
      std::vector<const uint64_t*> vsrc(nt);
      for (int tt = 0; tt < nt; ++tt) {
        const int t = t0 + tt, tau = t % g.c;
        const uint64_t* tp = T + (size_t)tt * w3;
        if (tau == 0) {
          vsrc[tt] = tp;
          continue;
        }
        const uint32_t gal = galois_left(c, -(int64_t)tau * g.H * lp);
        vs.push_back(tp + (size_t)nl3 * n);
        vr.push_back(KsReq{(int)vs.size() - 1, find_key(K, gal), gal, V + (size_t)tt * w3, tp, gal, nullptr});
        vsrc[tt] = V + (size_t)tt * w3;
      }
      if ((rc = ks_batch(c, level - 2, vs, vr))) return rc;
      std::vector<std::vector<CcTerm>> per_out(g.n_out);
      for (int tt = 0; tt < nt; ++tt) {
        const int t = t0 + tt, gi = t / g.c, tau = t % g.c;
        per_out[gi % g.n_out].push_back(CcTerm{vsrc[tt], g.m_ge + (size_t)tau * nl3 * n});
        if (tau > 0) per_out[((gi + 1) % g.n_diag) % g.n_out].push_back(CcTerm{vsrc[tt], g.m_lt + (size_t)tau * nl3 * n});
      }
      std::vector<CcTerm> terms;
      std::vector<int> off{0};
      std::vector<uint64_t*> outs;
      for (int o = 0; o < g.n_out; ++o) {
        if (per_out[o].empty()) continue;
        terms.insert(terms.end(), per_out[o].begin(), per_out[o].end());
        off.push_back((int)terms.size());
        outs.push_back(Oacc + (size_t)o * w3);
      }
      const CcTerm* terms_dev = upload_vec(c, terms);
      const int* off_dev = upload_vec(c, off);
      uint64_t* const* outs_dev = (uint64_t* const*)upload(c, outs.data(), outs.size() * sizeof(uint64_t*));
      if (!terms_dev || !off_dev || !outs_dev) return BLB_EDEVICE;
      {
        Span sp(c, BLB_T_EW, (double)outs.size() * w3);
        c->counters[2] += (int64_t)terms.size();
        launch_masked_acc(c, terms_dev, off_dev, outs_dev, (int)outs.size(), nl3, true);
      }
    }
    std::vector<const uint64_t*> oin;
    std::vector<uint64_t*> oout;
    for (int o = 0; o < g.n_out; ++o) {
      oin.push_back(Oacc + (size_t)o * w3);
      oout.push_back(Cd[g.out0 + o].data);
    }
    if ((rc = rescale_batch(c, level - 2, 2, oin, oout))) return rc;
  }
  if (P->hom1) b_scale = b_scale * BLB_NOISE_BOOST * ((double)c->mod[level_in] / BLB_NOISE_BOOST) / (double)c->mod[level_in];
  const double out_scale = A[0].scale * b_scale * 1024.0 / (double)c->mod[level - 1];
  for (int o = 0; o < n_out; ++o) {
    Cd[o].level = level - 3;
    Cd[o].degree = 1;
    Cd[o].scale = out_scale;
  }
  return BLB_OK;
}

}  // extern "C"

// ==========================================================================================
// Graph executors: one fused operator invocation recorded into a HIP graph with
// executor-owned scratch and descriptor memory, replayed with one launch.
// ==========================================================================================
struct blb_exec {
  blb_ctx* c = nullptr;
  ExecRec rec;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  size_t arena_bytes = 0, blob_bytes = 0;
  int has_mask = 0;
};

namespace {

void exec_release(blb_exec* E) {
  if (!E) return;
  blb_ctx* c = E->c;
  if (E->exec) (void)hipGraphExecDestroy(E->exec);
  if (E->graph) (void)hipGraphDestroy(E->graph);
  if (E->cap_stream) (void)hipStreamDestroy(E->cap_stream);
  dfree(c, E->rec.arena, E->arena_bytes);
  dfree(c, E->rec.blob_dev, E->blob_bytes);
  dfree(c, E->rec.param, 256);
  E->exec = nullptr;
  E->graph = nullptr;
  E->cap_stream = nullptr;
  E->rec = ExecRec();
}

// Records body() into E's graph.  Retries with a larger arena when the first guess is short.
template <class F>
int exec_record(blb_ctx* c, blb_exec* E, size_t arena_guess, F body) {
  size_t arena = arena_guess;
  for (int attempt = 0; attempt < 5; ++attempt, arena *= 2) {
    exec_release(E);
    E->c = c;
    E->arena_bytes = arena;
    E->blob_bytes = 64u << 20;
    int rc;
    if ((rc = dalloc(c, (void**)&E->rec.arena, E->arena_bytes))) return rc;
    E->rec.arena_cap = E->arena_bytes;
    if ((rc = dalloc(c, (void**)&E->rec.blob_dev, E->blob_bytes))) return rc;
    E->rec.blob_cap = E->blob_bytes;
    if ((rc = dalloc(c, (void**)&E->rec.param, 256))) return rc;
    if (hipStreamCreateWithFlags(&E->cap_stream, hipStreamNonBlocking) != hipSuccess) return BLB_EDEVICE;
    hipStream_t saved = c->stream;
    if (hipStreamSynchronize(saved) != hipSuccess) return BLB_EDEVICE;
    c->stream = E->cap_stream;
    c->rec = &E->rec;
    if (hipStreamBeginCapture(E->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      c->rec = nullptr;
      c->stream = saved;
      return BLB_EDEVICE;
    }
    rc = body();
    const hipError_t ec = hipStreamEndCapture(E->cap_stream, &E->graph);
    c->rec = nullptr;
    c->stream = saved;
    if (E->rec.overflow) continue;  // arena or blob too small: retry bigger
    if (rc) return rc;
    if (ec != hipSuccess || !E->graph) return BLB_EDEVICE;
    if (hipGraphInstantiate(&E->exec, E->graph, nullptr, nullptr, 0) != hipSuccess) return BLB_EDEVICE;
    if (!E->rec.blob_host.empty() &&
        hipMemcpy(E->rec.blob_dev, E->rec.blob_host.data(), E->rec.blob_host.size(), hipMemcpyHostToDevice) != hipSuccess)
      return BLB_EDEVICE;
    return BLB_OK;
  }
  return BLB_ENOMEM;
}

}  // namespace

extern "C" {

int blb_exec_create_cp(blb_ctx* c, const blb_keys* K, const blb_plan* P, const blb_ct* X, int n_in, blb_ct* Y, int n_out,
                       int mask_target_level, uint64_t* share_dev, blb_exec** out) {
  if (!c || !K || !P || !X || !Y || !out || P->kind != 1) return BLB_EINVAL;
  if (mask_target_level >= 0 && !share_dev) return BLB_EINVAL;
  *out = nullptr;
  blb_exec* E = new (std::nothrow) blb_exec();
  if (!E) return BLB_ENOMEM;
  E->has_mask = mask_target_level >= 0;
  const size_t ctw = (size_t)2 * (P->level + 1) * c->n * 8;
  const size_t guess = ctw * (size_t)(P->g.n_in * P->g.B * 6 + P->g.n_out * P->g.G * 6 + 64);
  const int rc = exec_record(c, E, guess, [&]() -> int {
    int r = blb_matmul_cp(c, K, P, X, n_in, Y, n_out);
    if (r) return r;
    if (mask_target_level >= 0) r = blb_mask_to_share(c, Y, n_out, 0, mask_target_level, share_dev);
    return r;
  });
  if (rc) {
    exec_release(E);
    delete E;
    return rc;
  }
  *out = E;
  return BLB_OK;
}

int blb_exec_create_cc(blb_ctx* c, const blb_keys* K, const blb_plan* P, const blb_ct* A, const blb_ct* Bp, int n_ct, blb_ct* Cd, int n_out,
                       int mask_target_level, uint64_t* share_dev, blb_exec** out) {
  if (!c || !K || !P || !A || !Bp || !Cd || !out || P->kind != 2) return BLB_EINVAL;
  if (mask_target_level >= 0 && !share_dev) return BLB_EINVAL;
  *out = nullptr;
  blb_exec* E = new (std::nothrow) blb_exec();
  if (!E) return BLB_ENOMEM;
  E->has_mask = mask_target_level >= 0;
  const size_t ctw = (size_t)2 * (P->level + 1) * c->n * 8;
  int max_m = 1;
  for (const CcGroup& g : P->groups) max_m = std::max(max_m, g.n_ct);
  const size_t tc = (size_t)std::min(P->Lp, 128);  // t values per chunk in blb_matmul_cc
  const size_t guess = ctw * (5 * tc * max_m + 8 * tc + 64 * (size_t)P->n_ct + 256);
  const int rc = exec_record(c, E, guess, [&]() -> int {
    int r = blb_matmul_cc(c, K, P, A, Bp, n_ct, Cd, n_out);
    if (r) return r;
    if (mask_target_level >= 0) r = blb_mask_to_share(c, Cd, n_out, 0, mask_target_level, share_dev);
    return r;
  });
  if (rc) {
    exec_release(E);
    delete E;
    return rc;
  }
  *out = E;
  return BLB_OK;
}

int blb_exec_run(blb_exec* E, uint64_t mask_seed) { return blb_exec_run_stream(E, mask_seed, nullptr); }

int blb_exec_run_stream(blb_exec* E, uint64_t mask_seed, void* stream) {
  if (!E || !E->exec) return BLB_EINVAL;
  blb_ctx* c = E->c;
  const hipStream_t s = stream ? (hipStream_t)stream : c->stream;
  const hipStream_t saved = c->stream;
  c->stream = s;  // the seed write goes on the replay's stream, ahead of it
  if (E->has_mask) launch_set_u64(c, E->rec.param, mask_seed);
  c->stream = saved;
  return hipGraphLaunch(E->exec, s) == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

uint64_t blb_exec_device_bytes(const blb_exec* E) { return E ? E->arena_bytes + E->blob_bytes + 256 : 0; }

void blb_exec_destroy(blb_exec* E) {
  if (!E) return;
  if (E->c) (void)hipStreamSynchronize(E->c->stream);
  exec_release(E);
  delete E;
}

}  // extern "C"

// ==========================================================================================
// Batched matmul_cp over independent instances (own keys, shared or own plans, uneven
// lengths): every stage runs once for the whole batch.
// ==========================================================================================
extern "C" {

int blb_batch_matmul_cp(blb_ctx* c, const blb_cp_instance* inst, int n_inst) {
  if (!c || !inst || n_inst < 1) return BLB_EINVAL;
  const int n = c->n;
  const int level = inst[0].plan ? inst[0].plan->level : -1;
  // validate everything before enqueuing work
  struct Ik {
    std::vector<const SwKey*> kb, kg;
  };
  std::vector<Ik> ik(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const blb_cp_instance& I = inst[i];
    if (!I.keys || !I.plan || !I.X || !I.Y || I.plan->kind != 1) return BLB_EINVAL;
    const CpGeom& g = I.plan->g;
    if (I.plan->level != level) return BLB_ELEVEL;
    if (I.plan->p50 != inst[0].plan->p50) return BLB_EINVAL;  // one plaintext format per call
    if (I.n_in != g.n_in || I.n_out != g.n_out) return BLB_EINVAL;
    for (int a = 0; a < I.n_in; ++a) {
      if (check_ct(c, &I.X[a]) || I.X[a].degree != 1) return BLB_EINVAL;
      if (I.X[a].level != level) return BLB_ELEVEL;
    }
    for (int b = 0; b < I.n_out; ++b)
      if (!I.Y[b].data) return BLB_EINVAL;
    ik[i].kb.assign(g.B, nullptr);
    ik[i].kg.assign(g.G, nullptr);
    for (int b = 1; b < g.B; ++b)
      if (!(ik[i].kb[b] = find_key(I.keys, galois_left(c, (int64_t)b * g.Lp)))) return BLB_ENOKEY;
    for (int j = 1; j < g.G; ++j)
      if (!(ik[i].kg[j] = find_key(I.keys, galois_left(c, (int64_t)j * g.B * g.Lp)))) return BLB_ENOKEY;
  }
  const int nl = level + 1;
  const size_t ctw = (size_t)2 * nl * n;
  Tmp tmp(c);
  std::vector<uint64_t*> RX(n_inst), inner(n_inst), rot(n_inst), acc(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const CpGeom& g = inst[i].plan->g;
    RX[i] = tmp.get<uint64_t>((size_t)std::max(1, g.n_in * (g.B - 1)) * ctw);
    inner[i] = tmp.get<uint64_t>((size_t)g.n_out * g.G * ctw);
    rot[i] = tmp.get<uint64_t>((size_t)std::max(1, g.n_out * (g.G - 1)) * ctw);
    acc[i] = tmp.get<uint64_t>((size_t)g.n_out * ctw);
  }
  if (tmp.failed) return BLB_ENOMEM;
  // noise boost of every input, then the baby steps of every instance in one key-switch batch
  int n_x = 0;
  for (int i = 0; i < n_inst; ++i) n_x += inst[i].n_in;
  uint64_t* Xs = tmp.get<uint64_t>((size_t)n_x * ctw);
  if (!Xs) return BLB_ENOMEM;
  {
    std::vector<const uint64_t*> xin;
    for (int i = 0; i < n_inst; ++i)
      for (int a = 0; a < inst[i].n_in; ++a) xin.push_back(inst[i].X[a].data);
    const uint64_t* const* xin_dev = upload_vec(c, xin);
    if (!xin_dev) return BLB_EDEVICE;
    launch_scale_cts(c, xin_dev, Xs, n_x, nl, BLB_NOISE_BOOST);
  }
  std::vector<const uint64_t*> srcs;
  std::vector<KsReq> reqs;
  std::vector<std::vector<const uint64_t*>> rx_tab(n_inst);
  int xk = 0;
  for (int i = 0; i < n_inst; ++i) {
    const blb_cp_instance& I = inst[i];
    const CpGeom& g = I.plan->g;
    rx_tab[i].assign((size_t)g.n_in * g.B, nullptr);
    for (int a = 0; a < g.n_in; ++a, ++xk) {
      const uint64_t* xa = Xs + (size_t)xk * ctw;
      srcs.push_back(xa + (size_t)nl * n);
      const int s = (int)srcs.size() - 1;
      rx_tab[i][(size_t)a * g.B] = xa;
      for (int b = 1; b < g.B; ++b) {
        const uint32_t gal = galois_left(c, (int64_t)b * g.Lp);
        uint64_t* dst = RX[i] + (size_t)(a * (g.B - 1) + b - 1) * ctw;
        rx_tab[i][(size_t)a * g.B + b] = dst;
        reqs.push_back(KsReq{s, ik[i].kb[b], gal, dst, xa, gal, nullptr});
      }
    }
  }
  int rc = ks_batch(c, level, srcs, reqs);
  if (rc) return rc;
  // MACs: one persistent launch over all plan groups
  {
    std::vector<const blb_plan*> plans;
    std::vector<std::vector<int>> members;
    for (int i = 0; i < n_inst; ++i) {
      int gi = -1;
      for (size_t k = 0; k < plans.size(); ++k)
        if (plans[k] == inst[i].plan) gi = (int)k;
      if (gi < 0) {
        plans.push_back(inst[i].plan);
        members.emplace_back();
        gi = (int)plans.size() - 1;
      }
      members[gi].push_back(i);
    }
    int tb, ib, cpt;
    batch_mac_shape(c->batch_variant, &tb, &ib, &cpt);
    std::vector<MacGroup> groups;
    std::vector<MacItem> items;
    for (size_t gi = 0; gi < plans.size(); ++gi) {
      const CpGeom& g = plans[gi]->g;
      const int n_ai = g.n_in * g.B, n_bj = g.n_out * g.G;
      std::vector<const uint64_t*> rx;
      std::vector<uint64_t*> outs;
      for (int i : members[gi]) {
        rx.insert(rx.end(), rx_tab[i].begin(), rx_tab[i].end());
        outs.push_back(inner[i]);
      }
      MacGroup mg;
      mg.pt = plans[gi]->pt;
      mg.rx = upload_vec(c, rx);
      mg.inner = (uint64_t* const*)upload(c, outs.data(), outs.size() * sizeof(uint64_t*));
      if (!mg.rx || !mg.inner) return BLB_EDEVICE;
      mg.n_ai = n_ai;
      mg.n_bj = n_bj;
      mg.nl = nl;
      mg.n_inst = (int)members[gi].size();
      groups.push_back(mg);
      c->counters[2] += (int64_t)n_ai * n_bj * mg.n_inst;
      c->counters[7] += (int64_t)n_ai * n_bj * nl * (int64_t)pt_poly_bytes(n, plans[gi]->p50) * ((mg.n_inst + ib - 1) / ib);
      const int n_kb = n / (256 * cpt);
      const int lg = c->batch_limbs > 0 ? std::min(c->batch_limbs, nl) : nl;  // limbs per work item
      for (int i0 = 0; i0 < mg.n_inst; i0 += ib)
        for (int limb = 0; limb < nl; limb += lg)
          for (int kb = 0; kb < n_kb; ++kb)
            for (int t = 0; t * tb < n_bj; ++t) items.push_back(MacItem{(int)gi, i0, t, kb, limb, std::min(lg, nl - limb)});
    }
    const MacGroup* g_dev = upload_vec(c, groups);
    const MacItem* it_dev = upload_vec(c, items);
    if (!g_dev || !it_dev) return BLB_EDEVICE;
    double units = 0;
    for (int i = 0; i < n_inst; ++i) units += (double)inst[i].plan->g.n_out * inst[i].plan->g.G * nl * n;
    Span sp(c, BLB_T_CP_MAC, units);
    launch_cp_mac_batch(c, g_dev, it_dev, (int)items.size(), c->batch_variant, c->batch_grid, inst[0].plan->p50);
  }
  // giant steps of every instance in one key-switch batch
  srcs.clear();
  reqs.clear();
  for (int i = 0; i < n_inst; ++i) {
    const CpGeom& g = inst[i].plan->g;
    for (int b = 0; b < g.n_out; ++b)
      for (int j = 1; j < g.G; ++j) {
        const uint64_t* src = inner[i] + (size_t)(b * g.G + j) * ctw;
        const uint32_t gal = galois_left(c, (int64_t)j * g.B * g.Lp);
        srcs.push_back(src + (size_t)nl * n);
        reqs.push_back(KsReq{(int)srcs.size() - 1, ik[i].kg[j], gal, rot[i] + (size_t)(b * (g.G - 1) + j - 1) * ctw, src, gal, nullptr});
      }
  }
  if ((rc = ks_batch(c, level, srcs, reqs))) return rc;
  {
    std::vector<const uint64_t*> terms;
    std::vector<int> off{0};
    std::vector<uint64_t*> outs;
    for (int i = 0; i < n_inst; ++i) {
      const CpGeom& g = inst[i].plan->g;
      for (int b = 0; b < g.n_out; ++b) {
        terms.push_back(inner[i] + (size_t)(b * g.G) * ctw);
        for (int j = 1; j < g.G; ++j) terms.push_back(rot[i] + (size_t)(b * (g.G - 1) + j - 1) * ctw);
        off.push_back((int)terms.size());
        outs.push_back(acc[i] + (size_t)b * ctw);
      }
    }
    const uint64_t* const* t_dev = upload_vec(c, terms);
    const int* off_dev = upload_vec(c, off);
    uint64_t* const* o_dev = (uint64_t* const*)upload(c, outs.data(), outs.size() * sizeof(uint64_t*));
    if (!t_dev || !off_dev || !o_dev) return BLB_EDEVICE;
    Span sp(c, BLB_T_EW, (double)outs.size() * ctw);
    launch_sum_var(c, t_dev, off_dev, o_dev, (int)outs.size(), nl);
  }
  std::vector<const uint64_t*> rin;
  std::vector<uint64_t*> rout;
  for (int i = 0; i < n_inst; ++i)
    for (int b = 0; b < inst[i].n_out; ++b) {
      rin.push_back(acc[i] + (size_t)b * ctw);
      rout.push_back(inst[i].Y[b].data);
    }
  if ((rc = rescale_batch(c, level, 2, rin, rout))) return rc;
  for (int i = 0; i < n_inst; ++i)
    for (int b = 0; b < inst[i].n_out; ++b) {
      inst[i].Y[b].level = level - 1;
      inst[i].Y[b].degree = 1;
      inst[i].Y[b].scale = inst[i].X[0].scale;
    }
  return BLB_OK;
}

int blb_exec_create_batch_cp(blb_ctx* c, const blb_cp_instance* inst, int n_inst, int mask_target_level, uint64_t* share_dev,
                             blb_exec** out) {
  if (!c || !inst || n_inst < 1 || !out) return BLB_EINVAL;
  if (mask_target_level >= 0 && !share_dev) return BLB_EINVAL;
  *out = nullptr;
  blb_exec* E = new (std::nothrow) blb_exec();
  if (!E) return BLB_ENOMEM;
  E->has_mask = mask_target_level >= 0;
  size_t guess = 64u << 20;
  int n_outs = 0;
  for (int i = 0; i < n_inst; ++i) {
    if (!inst[i].plan) {
      delete E;
      return BLB_EINVAL;
    }
    const CpGeom& g = inst[i].plan->g;
    guess += (size_t)2 * (inst[i].plan->level + 1) * c->n * 8 * (size_t)(g.n_in * g.B * 6 + g.n_out * g.G * 6 + 8);
    n_outs += inst[i].n_out;
  }
  std::vector<blb_ct> all;
  const int rc = exec_record(c, E, guess, [&]() -> int {
    int r = blb_batch_matmul_cp(c, inst, n_inst);
    if (r || mask_target_level < 0) return r;
    all.clear();
    for (int i = 0; i < n_inst; ++i)
      for (int b = 0; b < inst[i].n_out; ++b) all.push_back(inst[i].Y[b]);
    r = blb_mask_to_share(c, all.data(), (int)all.size(), 0, mask_target_level, share_dev);
    int k = 0;
    for (int i = 0; i < n_inst; ++i)
      for (int b = 0; b < inst[i].n_out; ++b) inst[i].Y[b].level = all[k++].level;
    return r;
  });
  (void)n_outs;
  if (rc) {
    exec_release(E);
    delete E;
    return rc;
  }
  *out = E;
  return BLB_OK;
}

}  // extern "C"

// ==========================================================================================
// Rotate-and-sum summation and broadcast (Section "Consistent Packing for Single Operator":
// Expansion and Reduction operators)
// ==========================================================================================
extern "C" {

int blb_rotate_sum(blb_ctx* c, const blb_keys* K, const blb_ct* in, int n_ct, int block, int n_blocks, int direction, int mask,
                   blb_ct* out) {
  if (!c || !K || !in || !out || n_ct < 1 || block < 1 || n_blocks < 1 || (n_blocks & (n_blocks - 1))) return BLB_EINVAL;
  if ((direction != 0 && direction != 1) || (mask != 0 && mask != 1) || (mask && direction != 0)) return BLB_EINVAL;
  const int S = c->n / 2, n = c->n;
  if ((int64_t)block * n_blocks > S) return BLB_EINVAL;
  for (int t = 0; t < n_ct; ++t) {
    if (check_ct(c, &in[t]) || in[t].degree != 1 || !out[t].data || in[t].level != in[0].level) return BLB_EINVAL;
    if (fabs(in[t].scale / in[0].scale - 1.0) > 1e-9) return BLB_ESCALE;
  }
  const int level = in[0].level, nl = level + 1;
  if (mask && level < 1) return BLB_ELEVEL;
  std::vector<const SwKey*> keys;
  std::vector<uint32_t> gals;
  for (int64_t st = block; st < (int64_t)block * n_blocks; st *= 2) {
    const uint32_t g = galois_left(c, direction == 0 ? st : -st);
    const SwKey* k = find_key(K, g);
    if (!k) return BLB_ENOKEY;
    keys.push_back(k);
    gals.push_back(g);
  }
  const size_t ctw = (size_t)2 * nl * n;
  Tmp tmp(c);
  uint64_t* cur = tmp.get<uint64_t>((size_t)n_ct * ctw);
  uint64_t* rot = tmp.get<uint64_t>((size_t)n_ct * ctw);
  uint64_t* mpt = mask ? tmp.get<uint64_t>((size_t)nl * n) : nullptr;
  if (tmp.failed) return BLB_ENOMEM;
  for (int t = 0; t < n_ct; ++t)
    if (hipMemcpyAsync(cur + (size_t)t * ctw, in[t].data, ctw * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) return BLB_EDEVICE;
  int rc = BLB_OK;
  // m^i = m^{i-1} + Rot^{2^{i-1} block}(m^{i-1}): one batch of n_ct key switches, then an add
  for (size_t s = 0; s < keys.size(); ++s) {
    std::vector<const uint64_t*> srcs;
    std::vector<KsReq> reqs;
    for (int t = 0; t < n_ct; ++t) {
      const uint64_t* x = cur + (size_t)t * ctw;
      srcs.push_back(x + (size_t)nl * n);
      reqs.push_back(KsReq{t, keys[s], gals[s], rot + (size_t)t * ctw, x, gals[s], nullptr});
    }
    if ((rc = ks_batch(c, level, srcs, reqs))) return rc;
    std::vector<const uint64_t*> terms;
    std::vector<uint64_t*> dsts;
    for (int t = 0; t < n_ct; ++t) {
      terms.push_back(cur + (size_t)t * ctw);
      terms.push_back(rot + (size_t)t * ctw);
      dsts.push_back(cur + (size_t)t * ctw);
    }
    const uint64_t* const* t_dev = upload_vec(c, terms);
    uint64_t* const* d_dev = (uint64_t* const*)upload(c, dsts.data(), dsts.size() * sizeof(uint64_t*));
    if (!t_dev || !d_dev) return BLB_EDEVICE;
    Span sp(c, BLB_T_EW, (double)n_ct * ctw);
    launch_sum_cts(c, t_dev, d_dev, n_ct, 2, nl);
  }
  std::vector<const uint64_t*> rin;
  std::vector<uint64_t*> rout;
  for (int t = 0; t < n_ct; ++t) {
    rin.push_back(cur + (size_t)t * ctw);
    rout.push_back(out[t].data);
  }
  if (mask) {
    // keep the first block: mask [1 x block, 0, ...] at scale q_level, then rescale
    std::vector<double> v((size_t)S, 0.0);
    for (int j = 0; j < block; ++j) v[j] = 1.0;
    if ((rc = encode_vectors_ntt(c, v, 1, (double)c->mod[level], level, mpt))) return rc;
    std::vector<CcPair> pairs;
    for (int t = 0; t < n_ct; ++t) pairs.push_back(CcPair{cur + (size_t)t * ctw, mpt, nullptr, nullptr, cur + (size_t)t * ctw});
    const CcPair* p_dev = upload_vec(c, pairs);
    if (!p_dev) return BLB_EDEVICE;
    {
      Span sp(c, BLB_T_EW, (double)n_ct * ctw);
      c->counters[2] += n_ct;
      launch_mask_pair(c, p_dev, n_ct, nl);
    }
    if ((rc = rescale_batch(c, level, 2, rin, rout))) return rc;
  } else {
    for (int t = 0; t < n_ct; ++t)
      if (hipMemcpyAsync(rout[t], rin[t], ctw * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) return BLB_EDEVICE;
  }
  const double sc = in[0].scale;
  for (int t = 0; t < n_ct; ++t) {
    out[t].level = mask ? level - 1 : level;
    out[t].degree = 1;
    out[t].scale = sc;
  }
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

// ------------------------------------------------------------------------------------------
// Identity and Expansion operators: element-wise ct-ct / ct-pt addition and multiplication,
// scalar addition and multiplication by broadcast (or straight after a summation)
// ------------------------------------------------------------------------------------------
namespace {
// n_ct pairs at one level; `same_scale` requires equal scales (additions)
int check_pairs(const blb_ctx* c, const blb_ct* a, const blb_ct* b, int n_ct, const blb_ct* out, bool same_scale) {
  if (!c || !a || !out || n_ct < 1) return BLB_EINVAL;
  for (int t = 0; t < n_ct; ++t) {
    if (check_ct(c, &a[t]) || a[t].degree != 1 || !out[t].data) return BLB_EINVAL;
    if (a[t].level != a[0].level) return BLB_ELEVEL;
    if (b) {
      if (check_ct(c, &b[t]) || b[t].degree != 1) return BLB_EINVAL;
      if (b[t].level != a[0].level) return BLB_ELEVEL;
      if (same_scale && fabs(b[t].scale / a[t].scale - 1.0) > 1e-9) return BLB_ESCALE;
    }
  }
  return BLB_OK;
}
void set_out(blb_ct* out, int n_ct, int level, const double* scales) {
  for (int t = 0; t < n_ct; ++t) {
    out[t].level = level;
    out[t].degree = 1;
    out[t].scale = scales[t];
  }
}
}  // namespace

int blb_ew_add(blb_ctx* c, const blb_ct* a, const blb_ct* b, int n_ct, blb_ct* out) {
  if (!b) return BLB_EINVAL;
  int rc = check_pairs(c, a, b, n_ct, out, true);
  if (rc) return rc;
  const int nl = a[0].level + 1;
  std::vector<const uint64_t*> terms;
  std::vector<uint64_t*> dsts;
  std::vector<double> sc;
  for (int t = 0; t < n_ct; ++t) {
    terms.push_back(a[t].data);
    terms.push_back(b[t].data);
    dsts.push_back(out[t].data);
    sc.push_back(a[t].scale);
  }
  const uint64_t* const* t_dev = upload_vec(c, terms);
  uint64_t* const* d_dev = (uint64_t* const*)upload(c, dsts.data(), dsts.size() * sizeof(uint64_t*));
  if (!t_dev || !d_dev) return BLB_EDEVICE;
  {
    Span sp(c, BLB_T_EW, (double)n_ct * 2 * nl * c->n);
    launch_sum_cts(c, t_dev, d_dev, n_ct, 2, nl);
  }
  set_out(out, n_ct, a[0].level, sc.data());
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

int blb_ew_add_plain(blb_ctx* c, const blb_ct* a, int n_ct, const uint64_t* pt_dev, blb_ct* out) {
  if (!pt_dev) return BLB_EINVAL;
  int rc = check_pairs(c, a, nullptr, n_ct, out, false);
  if (rc) return rc;
  const int n = c->n, nl = a[0].level + 1;
  const size_t ctw = (size_t)2 * nl * n;
  std::vector<double> sc;
  for (int t = 0; t < n_ct; ++t) {
    sc.push_back(a[t].scale);
    if (out[t].data != a[t].data &&
        hipMemcpyAsync(out[t].data, a[t].data, ctw * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      return BLB_EDEVICE;
  }
  std::vector<PolyDesc> d;
  for (int t = 0; t < n_ct; ++t)
    for (int i = 0; i < nl; ++i) {
      PolyDesc x = pd(pt_dev + ((size_t)t * nl + i) * n, out[t].data + (size_t)i * n, i, c->log_n);
      x.src2 = out[t].data + (size_t)i * n;
      d.push_back(x);
    }
  {
    Span sp(c, BLB_T_EW, (double)n_ct * nl * n);
    ntt_descs(c, d, NTT_ADDTO);
  }
  set_out(out, n_ct, a[0].level, sc.data());
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

int blb_ew_mul_plain(blb_ctx* c, const blb_ct* a, int n_ct, const uint64_t* pt_dev, double pt_scale, blb_ct* out) {
  if (!pt_dev || !(pt_scale > 0)) return BLB_EINVAL;
  int rc = check_pairs(c, a, nullptr, n_ct, out, false);
  if (rc) return rc;
  const int n = c->n, nl = a[0].level + 1;
  Tmp tmp(c);
  uint64_t* ptn = tmp.get<uint64_t>((size_t)n_ct * nl * n);
  if (tmp.failed) return BLB_ENOMEM;
  std::vector<PolyDesc> d;
  for (int t = 0; t < n_ct; ++t)
    for (int i = 0; i < nl; ++i) d.push_back(pd(pt_dev + ((size_t)t * nl + i) * n, ptn + ((size_t)t * nl + i) * n, i, c->log_n));
  ntt_descs(c, d, NTT_FWD);
  std::vector<CcPair> pairs;
  std::vector<double> sc;
  for (int t = 0; t < n_ct; ++t) {
    pairs.push_back(CcPair{a[t].data, ptn + (size_t)t * nl * n, nullptr, nullptr, out[t].data});
    sc.push_back(a[t].scale * pt_scale);
  }
  const CcPair* p_dev = upload_vec(c, pairs);
  if (!p_dev) return BLB_EDEVICE;
  {
    Span sp(c, BLB_T_EW, (double)n_ct * 2 * nl * n);
    c->counters[2] += n_ct;
    launch_mask_pair(c, p_dev, n_ct, nl);
  }
  set_out(out, n_ct, a[0].level, sc.data());
  return hipGetLastError() == hipSuccess ? BLB_OK : BLB_EDEVICE;
}

int blb_ew_mul_relin(blb_ctx* c, const blb_keys* K, const blb_ct* a, const blb_ct* b, int n_ct, blb_ct* out) {
  if (!K || !b) return BLB_EINVAL;
  int rc = check_pairs(c, a, b, n_ct, out, false);
  if (rc) return rc;
  const SwKey* relin = find_key(K, 0);
  if (!relin) return BLB_ENOKEY;
  const int n = c->n, level = a[0].level, nl = level + 1;
  Tmp tmp(c);
  uint64_t* T3 = tmp.get<uint64_t>((size_t)n_ct * 3 * nl * n);
  if (tmp.failed) return BLB_ENOMEM;
  std::vector<const uint64_t*> at, bt;
  std::vector<double> sc;
  for (int t = 0; t < n_ct; ++t) {
    at.push_back(a[t].data);
    bt.push_back(b[t].data);
    sc.push_back(a[t].scale * b[t].scale);
  }
  const uint64_t* const* a_dev = upload_vec(c, at);
  const uint64_t* const* b_dev = upload_vec(c, bt);
  if (!a_dev || !b_dev) return BLB_EDEVICE;
  {
    Span sp(c, BLB_T_CC_TENSOR, (double)n_ct * nl * n);
    c->counters[3] += n_ct;
    c->counters[4] += n_ct;
    launch_tensor_sum(c, a_dev, b_dev, T3, n_ct, 1, nl, nl, true);
  }
  std::vector<const uint64_t*> srcs;
  std::vector<KsReq> reqs;
  for (int t = 0; t < n_ct; ++t) {
    const uint64_t* t3 = T3 + (size_t)t * 3 * nl * n;
    srcs.push_back(t3 + (size_t)2 * nl * n);
    reqs.push_back(KsReq{t, relin, 0, out[t].data, t3, 0, t3 + (size_t)nl * n});
  }
  if ((rc = ks_batch(c, level, srcs, reqs))) return rc;
  set_out(out, n_ct, level, sc.data());
  return BLB_OK;
}

int blb_scalar_op(blb_ctx* c, const blb_keys* K, const blb_ct* a, const blb_ct* s, int n_ct, int block, int n_blocks, int op,
                  int from_sum, blb_ct* out) {
  if (!c || !K || !s || (op != 0 && op != 1) || (from_sum != 0 && from_sum != 1)) return BLB_EINVAL;
  int rc = check_pairs(c, a, s, n_ct, out, op == 0);
  if (rc) return rc;
  if (from_sum && (int64_t)block * n_blocks != c->n / 2) return BLB_EINVAL;
  const int nl = a[0].level + 1;
  const size_t ctw = (size_t)2 * nl * c->n;
  Tmp tmp(c);
  uint64_t* v = tmp.get<uint64_t>((size_t)n_ct * ctw);
  if (tmp.failed) return BLB_ENOMEM;
  std::vector<blb_ct> vs(n_ct);
  for (int t = 0; t < n_ct; ++t) vs[t] = blb_ct{v + (size_t)t * ctw, a[0].level, 1, 0.0};
  // broadcast of the first block (right rotate-and-sum), or the unmasked summation (left)
  if ((rc = blb_rotate_sum(c, K, s, n_ct, block, n_blocks, from_sum ? 0 : 1, 0, vs.data()))) return rc;
  return op == 0 ? blb_ew_add(c, a, vs.data(), n_ct, out) : blb_ew_mul_relin(c, K, a, vs.data(), n_ct, out);
}

}  // extern "C"
