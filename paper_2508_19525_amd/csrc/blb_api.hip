// Host side of the gfx950 engine: parameters and tables, descriptor uploads, key
// generation, encode/encrypt/decrypt/decode, key switching batches, rescale, matmul_cp and
// mask-and-share, exposed through the C ABI of include/blb.h.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <algorithm>
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

// stream-ordered temporaries (pooled by the HIP runtime)
struct Tmp {
  blb_ctx* c;
  std::vector<void*> ptrs;
  bool failed = false;
  explicit Tmp(blb_ctx* cc) : c(cc) {}
  template <class T>
  T* get(size_t count) {
    void* p = nullptr;
    if (count == 0) count = 1;
    if (hipMallocAsync(&p, count * sizeof(T), c->stream) != hipSuccess) {
      (void)hipGetLastError();
      failed = true;
      return nullptr;
    }
    ptrs.push_back(p);
    return (T*)p;
  }
  ~Tmp() {
    for (void* p : ptrs) (void)hipFreeAsync(p, c->stream);
  }
};

// ------------------------------------------------------------------------------------------
// descriptor upload ring
// ------------------------------------------------------------------------------------------
const size_t kUploadCap = 32u << 20;

int uploader_init(blb_ctx* c) {
  Uploader& u = c->up;
  u.cap = kUploadCap;
  HIP_OK(hipHostMalloc((void**)&u.host, u.cap, hipHostMallocDefault));
  HIP_OK(hipMalloc((void**)&u.dev, u.cap));
  return BLB_OK;
}
void uploader_free(blb_ctx* c) {
  Uploader& u = c->up;
  for (auto& e : u.inflight) (void)hipEventDestroy(e.second);
  for (auto e : u.free_events) (void)hipEventDestroy(e);
  if (u.host) (void)hipHostFree(u.host);
  if (u.dev) (void)hipFree(u.dev);
}
// Copies `bytes` from host memory to a device region that stays valid for all work enqueued
// on the stream before the ring wraps back onto it.
void* upload(blb_ctx* c, const void* data, size_t bytes) {
  Uploader& u = c->up;
  bytes = align_up(bytes, 256);
  if (bytes > u.cap) return nullptr;
  size_t lo = u.head;
  if (lo + bytes > u.cap) lo = 0;
  const size_t hi = lo + bytes;
  // the pinned region may be read by a copy still in flight: wait for those copies
  std::deque<std::pair<size_t, hipEvent_t>> keep;
  size_t prev_end = 0;
  (void)prev_end;
  while (!u.inflight.empty()) {
    auto e = u.inflight.front();
    u.inflight.pop_front();
    const size_t e_end = e.first & 0xFFFFFFFFFFull;
    const size_t e_lo = e.first >> 40;
    if (e_lo < hi && lo < e_end) {
      (void)hipEventSynchronize(e.second);
      u.free_events.push_back(e.second);
    } else if (hipEventQuery(e.second) == hipSuccess) {
      u.free_events.push_back(e.second);
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
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamSynchronize(c->stream);
    u.head = hi;
    return u.dev + lo;
  }
  (void)hipEventRecord(ev, c->stream);
  u.inflight.push_back({(lo << 40) | hi, ev});
  u.head = hi;
  return u.dev + lo;
}

template <class T>
const T* upload_vec(blb_ctx* c, const std::vector<T>& v) {
  return (const T*)upload(c, v.data(), v.size() * sizeof(T));
}

// descriptor batches can exceed the ring: split into chunks
void ntt_descs(blb_ctx* c, const std::vector<PolyDesc>& d, int kind) {
  const size_t chunk = 16384;
  for (size_t off = 0; off < d.size(); off += chunk) {
    const size_t cnt = std::min(chunk, d.size() - off);
    const PolyDesc* dd = (const PolyDesc*)upload(c, d.data() + off, cnt * sizeof(PolyDesc));
    if (!dd) return;
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
int ks_batch(blb_ctx* c, int level, const std::vector<const uint64_t*>& srcs, const std::vector<KsReq>& reqs) {
  if (srcs.empty() || reqs.empty()) return BLB_OK;
  const KsLevelConst& kc = c->h_kc[level];
  const int nl = kc.nl, n_ext = kc.n_ext, nd = kc.n_digits, n = c->n;
  const int S = (int)srcs.size(), O = (int)reqs.size();
  Tmp tmp(c);
  uint64_t* dcoef = tmp.get<uint64_t>((size_t)S * nl * n);
  uint64_t* X = tmp.get<uint64_t>((size_t)S * nd * n_ext * n);
  uint64_t* U = tmp.get<uint64_t>((size_t)O * 2 * n_ext * n);
  uint64_t* corr = tmp.get<uint64_t>((size_t)O * 2 * nl * n);
  if (tmp.failed) return BLB_ENOMEM;
  std::vector<PolyDesc> d;
  d.reserve((size_t)S * nl);
  for (int s = 0; s < S; ++s)
    for (int i = 0; i < nl; ++i) d.push_back(pd(srcs[s] + (size_t)i * n, dcoef + ((size_t)s * nl + i) * n, i, c->log_n));
  ntt_descs(c, d, NTT_INV);
  launch_modup(c, dcoef, X, c->d_kc[level], S, nl, n_ext, nd);
  d.clear();
  for (int s = 0; s < S; ++s)
    for (int j = 0; j < nd; ++j)
      for (int e = 0; e < n_ext; ++e) {
        if (e >= kc.dlo[j] && e < kc.dhi[j]) continue;
        uint64_t* p = X + (((size_t)s * nd + j) * n_ext + e) * n;
        d.push_back(pd(p, p, e < nl ? e : c->n_q + (e - nl), c->log_n));
      }
  ntt_descs(c, d, NTT_FWD);
  std::vector<KsOut> ko(O);
  for (int o = 0; o < O; ++o) {
    ko[o].c1 = srcs[reqs[o].src];
    ko[o].key = reqs[o].key->data;
    ko[o].gal = reqs[o].gal;
    ko[o].src = reqs[o].src;
  }
  const KsOut* ko_dev = upload_vec(c, ko);
  if (!ko_dev) return BLB_EDEVICE;
  launch_ks_inner(c, ko_dev, O, X, c->d_kc[level], U, nl, n_ext, nd);
  d.clear();
  for (int o = 0; o < O; ++o)
    for (int p = 0; p < 2; ++p)
      for (int t = 0; t < c->n_sp; ++t) {
        uint64_t* ptr = U + (((size_t)o * 2 + p) * n_ext + nl + t) * n;
        d.push_back(pd(ptr, ptr, c->n_q + t, c->log_n));
      }
  ntt_descs(c, d, NTT_INV);
  launch_moddown_conv(c, U, corr, c->d_kc[level], O, nl, n_ext);
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

// batched rescale: in[t] at `level` (degree+1 polys) -> out[t] at level-1 (compact)
int rescale_batch(blb_ctx* c, int level, int n_poly, const std::vector<const uint64_t*>& in, const std::vector<uint64_t*>& out) {
  const int n = c->n, nl = level + 1;
  const int T = (int)in.size();
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
  launch_enc_scatter_dense(c, d_vals, n_vals, count, a);
  (void)hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream);
  run_encode_core(c, a, b, count, scale, level + 1, out, c->d_flag);
  int flag = 0;
  (void)hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (hipStreamSynchronize(c->stream) != hipSuccess) return BLB_EDEVICE;
  return flag ? BLB_EINVAL : BLB_OK;
}

}  // namespace

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
  blb_ctx* c = new (std::nothrow) blb_ctx();
  if (!c) return BLB_ENOMEM;
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
    std::vector<int32_t> su(M);
    uint64_t e = 1;
    for (int j = 0; j < M; ++j) {
      su[j] = (int32_t)((e - 1) / 4);
      e = e * 5 % (2ull * n);
    }
    if ((rc = dalloc(c, (void**)&c->d_enc_tw, tw.size() * sizeof(double)))) return fail(rc);
    if ((rc = dalloc(c, (void**)&c->d_enc_twist, twist.size() * sizeof(double)))) return fail(rc);
    if ((rc = dalloc(c, (void**)&c->d_slot_u, su.size() * sizeof(int32_t)))) return fail(rc);
    if ((rc = dalloc(c, (void**)&c->d_flag, 256))) return fail(rc);
    if (hipMemcpy(c->d_enc_tw, tw.data(), tw.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(BLB_EDEVICE);
    if (hipMemcpy(c->d_enc_twist, twist.data(), twist.size() * 8, hipMemcpyHostToDevice) != hipSuccess) return fail(BLB_EDEVICE);
    if (hipMemcpy(c->d_slot_u, su.data(), su.size() * 4, hipMemcpyHostToDevice) != hipSuccess) return fail(BLB_EDEVICE);
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
  uploader_free(c);
  const int nm = c->n_q + c->n_sp;
  dfree(c, c->d_tw_fwd, sizeof(double) * nm * c->n);
  dfree(c, c->d_tw_inv, sizeof(double) * nm * c->n);
  dfree(c, c->d_mods, sizeof(uint64_t) * BLB_MAXM);
  dfree(c, c->d_enc_tw, sizeof(double) * (c->n / 4) * 4);
  dfree(c, c->d_enc_twist, sizeof(double) * (c->n / 2) * 4);
  dfree(c, c->d_slot_u, sizeof(int32_t) * (c->n / 2));
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

int blb_decode(blb_ctx* c, const uint64_t* pt_dev, int level, double scale, double* v, int64_t n_vals) {
  if (!c || !pt_dev || !v || level < 0 || level >= c->n_q || n_vals < 0 || n_vals > c->n / 2 || !(scale > 0)) return BLB_EINVAL;
  const int n = c->n, nl = level + 1;
  std::vector<uint64_t> h((size_t)nl * n);
  if (hipMemcpyAsync(h.data(), pt_dev, h.size() * 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess) return BLB_EDEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return BLB_EDEVICE;
  // centred CRT lift (mixed radix, long double), then the slot evaluation
  // m_j = Delta^-1 sum_k p_k cos(pi e_j k / N)
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
  std::vector<long double> cosv(2 * n);
  for (int t = 0; t < 2 * n; ++t) cosv[t] = cosl(3.14159265358979323846264338327950288L * (long double)t / (long double)n);
  uint64_t e = 1;
  for (int64_t j = 0; j < n_vals; ++j) {
    long double acc = 0;
    uint64_t idx = 0;
    for (int k = 0; k < n; ++k) {
      acc += lift[k] * cosv[idx];
      idx += e;
      if (idx >= 2ull * n) idx -= 2ull * n;
    }
    v[j] = (double)(acc / (long double)scale);
    e = e * 5 % (2ull * n);
  }
  return BLB_OK;
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
  return g;
}

int blb_plan_matmul_cp(blb_ctx* c, const double* W, int d_in, int d_out, int L, int level, blb_plan** out) {
  if (!c || !W || !out || d_in < 1 || d_out < 1 || L < 1 || L > c->n / 2 || level < 1 || level >= c->n_q) return BLB_EINVAL;
  *out = nullptr;
  const CpGeom g = cp_geometry(c, L, d_in, d_out);
  const int n = c->n, nl = level + 1;
  const int n_bj = g.n_out * g.G, n_ai = g.n_in * g.B;
  const size_t n_pt = (size_t)n_bj * n_ai;
  blb_plan* P = new (std::nothrow) blb_plan();
  if (!P) return BLB_ENOMEM;
  P->ctx = c;
  P->kind = 1;
  P->level = level;
  P->g = g;
  P->bytes = n_pt * nl * n * 8;
  int rc = dalloc(c, (void**)&P->pt, P->bytes);
  if (rc) {
    delete P;
    return rc;
  }
  const int M = n / 2;
  const int chunk = 512;
  {
    Tmp tmp(c);
    double* dW = tmp.get<double>((size_t)d_in * d_out);
    double* a = tmp.get<double>((size_t)chunk * M * 4);
    double* b = tmp.get<double>((size_t)chunk * M * 4);
    if (tmp.failed) {
      blb_plan_destroy(P);
      return BLB_ENOMEM;
    }
    if (hipMemcpyAsync(dW, W, (size_t)d_in * d_out * 8, hipMemcpyHostToDevice, c->stream) != hipSuccess) {
      blb_plan_destroy(P);
      return BLB_EDEVICE;
    }
    (void)hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream);
    const double scale = (double)c->mod[level];
    std::vector<PolyDesc> d;
    for (size_t p0 = 0; p0 < n_pt; p0 += chunk) {
      const int cnt = (int)std::min<size_t>(chunk, n_pt - p0);
      launch_enc_scatter_cp(c, dW, g, (int)p0, cnt, a);
      uint64_t* dst = P->pt + p0 * nl * n;
      run_encode_core(c, a, b, cnt, scale, nl, dst, c->d_flag);
      d.clear();
      for (int p = 0; p < cnt; ++p)
        for (int i = 0; i < nl; ++i) {
          uint64_t* x = dst + ((size_t)p * nl + i) * n;
          d.push_back(pd(x, x, i, c->log_n));
        }
      ntt_descs(c, d, NTT_FWD);
    }
    int flag = 0;
    (void)hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (hipStreamSynchronize(c->stream) != hipSuccess || flag) {
      blb_plan_destroy(P);
      return flag ? BLB_EINVAL : BLB_EDEVICE;
    }
  }
  *out = P;
  return BLB_OK;
}

void blb_plan_destroy(blb_plan* P) {
  if (!P) return;
  (void)hipStreamSynchronize(P->ctx->stream);
  dfree(P->ctx, P->pt, P->bytes);
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
  uint64_t* RX = tmp.get<uint64_t>((size_t)n_ai * ctw);
  uint64_t* inner = tmp.get<uint64_t>((size_t)n_bj * ctw);
  uint64_t* rot = tmp.get<uint64_t>((size_t)std::max(1, g.n_out * (g.G - 1)) * ctw);
  uint64_t* acc = tmp.get<uint64_t>((size_t)g.n_out * ctw);
  if (tmp.failed) return BLB_ENOMEM;
  // baby steps, hoisted per input: RX[a][i] = Rot_l^{i L'}(X_a)
  std::vector<const uint64_t*> srcs;
  std::vector<KsReq> reqs;
  for (int a = 0; a < n_in; ++a) {
    if (hipMemcpyAsync(RX + (size_t)(a * g.B) * ctw, X[a].data, ctw * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
      return BLB_EDEVICE;
    srcs.push_back(X[a].data + (size_t)nl * n);
    for (int i = 1; i < g.B; ++i) {
      const uint32_t gal = galois_left(c, (int64_t)i * g.Lp);
      reqs.push_back(KsReq{a, kb[i], gal, RX + (size_t)(a * g.B + i) * ctw, X[a].data, gal, nullptr});
    }
  }
  int rc = ks_batch(c, level, srcs, reqs);
  if (rc) return rc;
  // plaintext MACs
  launch_cp_mac(c, P->pt, RX, inner, nl, n_ai, n_bj);
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
  const ModMap lim = map_identity(nl);
  for (int b = 0; b < g.n_out; ++b) {
    uint64_t* ab = acc + (size_t)b * ctw;
    const uint64_t* first = inner + (size_t)(b * g.G) * ctw;
    if (g.G == 1) {
      if (hipMemcpyAsync(ab, first, ctw * 8, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) return BLB_EDEVICE;
    } else {
      launch_ew(c, EW_ADD, ab, first, rot + (size_t)(b * (g.G - 1)) * ctw, nullptr, 2 * nl, lim);
      for (int j = 2; j < g.G; ++j) launch_ew(c, EW_ADD, ab, ab, rot + (size_t)(b * (g.G - 1) + j - 1) * ctw, nullptr, 2 * nl, lim);
    }
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
  launch_mask_sample(c, r, share_dev, n_ct, tl, seed, 6 /* mask */);
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

}  // extern "C"
