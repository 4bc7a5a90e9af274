// Batched negacyclic NTT / inverse NTT for gfx950 on FP64 lanes.
//
// One workgroup transforms one N-word polynomial (N = 4096 / 8192 / 16384), exchanging
// values through LDS (N doubles + 1/16 padding, 136 KiB at N = 16384 against 160 KiB per
// CU).  Each of the N/PT work-items keeps PT = 16 (or 32) values in registers and runs up to
// four (five) radix-2 stages on them per pass; the first pass reads global memory and the last
// writes it, so a transform costs (passes - 1) LDS round trips.  The forward transform is the
// Cooley-Tukey ordering with twiddles psi^brv(m+i) (natural in, bit-reversed out, value j is
// the evaluation at psi^(2 brv(j) + 1)); the inverse is the Gentleman-Sande ordering with
// psi^-brv(m+i) followed by N^-1.  Polys are addressed through a descriptor table so a
// launch can gather from arbitrary buffers and moduli.
#include "blb_internal.h"
#include "blb_kernels.h"
#include <algorithm>
#include <type_traits>

namespace {

// Values per work-item (the radix of a pass: log2 of it is the number of radix-2 stages a pass
// runs in registers).  16 (passes of 4 stages, N/16 work-items) or 32 (passes of 5 stages, N/32
// work-items, one LDS round trip fewer); chosen per context by the autotuner, never changing a
// result.
constexpr int kPT16 = 16, kPT32 = 32;

// Where a launch finds its polynomials: a descriptor table, or (descs == null) a regular
// batch of `count` limb-polys stored back to back at `base`, transformed in place, poly p
// taken modulo prime p mod nl (the [item][limb][N] layout of ciphertexts and plaintexts).
struct NttSrc {
  const PolyDesc* descs;
  uint64_t* base;
  int nl;
  int log_n;
  __device__ __forceinline__ PolyDesc get(int p) const {
    if (descs) {
      // scalar loads (the table is read-only while the kernel runs): they do not join the
      // in-order vector-memory counter, so fetching a descriptor never waits for the stores
      // of the previous polynomial
      typedef __attribute__((address_space(4))) const uint64_t ku64;
      static_assert(sizeof(PolyDesc) == 64, "descriptor layout");
      const ku64* w = (const ku64*)(descs + p);
      union {
        uint64_t u[8];
        PolyDesc d;
      } r;
#pragma unroll
      for (int i = 0; i < 8; ++i) r.u[i] = w[i];
      return r.d;
    }
    PolyDesc d;
    d.src = base + ((size_t)p << log_n);
    d.dst = base + ((size_t)p << log_n);
    d.src2 = nullptr;
    d.src3 = nullptr;
    d.aux = 0.0;
    d.aux2 = 0.0;
    d.mod = p % nl;
    d.gal = 0;
    d.log_n = log_n;
    d.pad = 0;
    return d;
  }
};

__host__ __device__ constexpr int pad_idx(int j) { return j + (j >> 4); }

// One pass of R_LOG radix-2 stages starting at global stage S0.  Work-item `tid` holds
// PT values in registers: GPT groups of GS = 2^R_LOG values each, group h being the
// butterfly group g = tid + h T (T = N / PT) whose members sit TL = N >> (S0 + R_LOG)
// words apart.
template <int LOGN, int PT, int S0, int R_LOG>
struct Pass {
  static constexpr int N = 1 << LOGN;
  static constexpr int T = N / PT;
  static constexpr int GS = 1 << R_LOG;
  static constexpr int GPT = PT / GS;
  static constexpr int TL = N >> (S0 + R_LOG);
  static_assert(S0 + R_LOG <= LOGN && GS <= PT, "pass shape");
  // twiddles differ across the lanes of a wave (vector loads) unless the pass spans whole
  // columns (TL >= T) or a butterfly tree covers at least 64 work-items (TL >= 64)
  static constexpr bool LANE_TW = !(TL >= T || TL >= 64);

  // coefficient index of register slot i (= h GS + k)
  __host__ __device__ static constexpr int idx(int tid, int i) {
    const int h = i / GS, k = i % GS;
    const int g = tid + h * T;
    return (g / TL) * (TL << R_LOG) + (g % TL) + k * TL;
  }

  // Padded LDS word of slot i relative to slot 0.  In every pass shape used here it does not
  // depend on the work-item (asserted for all work-items at compile time below), so an exchange
  // needs one address per work-item and the slots become immediate offsets.
  static constexpr int lds_off(int i) { return pad_idx(idx(0, i)) - pad_idx(idx(0, 0)); }

  // FWD: Cooley-Tukey stages in increasing order; else Gentleman-Sande in decreasing order.
  template <bool FWD>
  __device__ static __forceinline__ void run(double (&x)[PT], const double* __restrict__ tw, double q, double qi, int tid) {
#pragma unroll
    for (int uu = 0; uu < R_LOG; ++uu) {
      const int u = FWD ? uu : (R_LOG - 1 - uu);
      const int t_loc = GS >> (u + 1);
#pragma unroll
      for (int h = 0; h < GPT; ++h) {
        // group index; compile-time when a pass spans whole columns (first pass), and uniform
        // over the 64-lane wave when TL >= 64, so the twiddles come through scalar loads
        int hi = (tid + h * T) / TL;
        if constexpr (TL >= T) hi = (h * T) / TL;
        else if constexpr (TL >= 64) hi = __builtin_amdgcn_readfirstlane(hi);
#pragma unroll
        for (int k = 0; k < GS; ++k) {
          if (k & t_loc) continue;
          const int widx = (1 << (S0 + u)) + (hi << u) + (k >> (R_LOG - u));
          const double w = tw[widx];
          double& a = x[h * GS + k];
          double& b = x[h * GS + k + t_loc];
          // lazy reduction.  For |b| <= B, mulmod_s returns |v| < q/2 + 1.5 B q 2^-52
          // < q/2 + 0.375 B (the quotient estimate is off by < B 2^-52, the dropped low part
          // of b w is < B q 2^-53), so in the forward (Cooley-Tukey) butterfly the bound grows
          // as B' = 1.375 B + q/2: from |x| <= q at the start of a pass, four stages stay below
          // 7.01 q < 2^53, where every FP64 sum and product step is exact (a fifth would reach
          // 10.1 q > 2^53); values are reduced after the fourth stage and at the end of the
          // pass.  In the inverse (Gentleman-Sande) butterfly a + b can double, so it reduces
          // after every second stage and at the end of the pass.
          const bool red = FWD ? (u == R_LOG - 1 || u == 3) : ((u & 1) || (u == R_LOG - 1));
          if (FWD) {
            const double v = mulmod_s(b, w, q, qi);
            const double sum = a + v, dif = a - v;
            a = red ? reduce_s(sum, q, qi) : sum;
            b = red ? reduce_s(dif, q, qi) : dif;
          } else {
            const double sum = a + b, dif = a - b;
            a = red ? reduce_s(sum, q, qi) : sum;
            b = mulmod_s(dif, w, q, qi);
          }
        }
      }
    }
  }
};

// Workgroup barrier that orders LDS accesses only: global loads in flight (the persistent
// kernel's prefetch of the next polynomial) are not waited for, unlike __syncthreads().
// Global memory is never exchanged between work-items of a workgroup here: each work-item
// consumes its own loads before its first barrier, and stores come after the last one.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Move the register values from the layout of pass PA to the layout of pass PB through LDS.
// The leading barrier keeps the writes behind every read of the previous exchange (also of
// the previous polynomial in the persistent kernel).
template <class PA, class PB, int PT>
__device__ __forceinline__ void relayout(double* lds, double (&x)[PT], int tid) {
  double* la = lds + pad_idx(PA::idx(tid, 0));
  const double* lb = lds + pad_idx(PB::idx(tid, 0));
  lds_barrier();
#pragma unroll
  for (int i = 0; i < PT; ++i) la[PA::lds_off(i)] = x[i];
  lds_barrier();
#pragma unroll
  for (int i = 0; i < PT; ++i) x[i] = lb[PB::lds_off(i)];
}

// lds_off(i) is the same for every work-item of pass P
template <class P>
constexpr bool lds_affine() {
  for (int i = 1; i < P::GS * P::GPT; ++i) {
    const int off = P::lds_off(i);
    for (int tid = 1; tid < P::T; ++tid)
      if (pad_idx(P::idx(tid, i)) - pad_idx(P::idx(tid, 0)) != off) return false;
  }
  return true;
}

// Pass schedule (forward order).  PT = 16: three passes of four stages, then the remaining
// LOGN - 12 stages; PT = 32: two passes of five stages, then the remaining LOGN - 10.  The first
// pass reads its operands straight from global memory and the last pass writes straight to
// global memory, so a transform makes (passes - 1) LDS round trips.
template <int LOGN, int PT>
struct Sched {
  static constexpr int R = PT == 32 ? 5 : 4;
  static constexpr int REM = LOGN - 3 * R;  // stages of a fourth pass (PT = 16 only)
  static_assert(PT == 16 || PT == 32, "values per work-item");
  static_assert(PT == 16 || LOGN - 2 * R >= 1, "third pass");
  using P0 = Pass<LOGN, PT, 0, R>;
  using P1 = Pass<LOGN, PT, R, R>;
  using P2 = Pass<LOGN, PT, 2 * R, (PT == 32 ? LOGN - 2 * R : R)>;
  using P3 = Pass<LOGN, PT, 3 * R, (PT == 16 && REM > 0 ? REM : 1)>;
  static constexpr bool HAS3 = PT == 16 && REM > 0;
  using Tail = std::conditional_t<HAS3, P3, P2>;  // forward-last / inverse-first pass
  static_assert(lds_affine<P0>(), "LDS offsets of the first pass depend on the work-item");
  static_assert(lds_affine<P1>(), "LDS offsets of the second pass depend on the work-item");
  static_assert(lds_affine<P2>(), "LDS offsets of the third pass depend on the work-item");
  static_assert(lds_affine<Tail>(), "LDS offsets of the last pass depend on the work-item");
  static constexpr int NP = HAS3 ? 4 : 3;  // passes
  // passes (in execution order) that run before the persistent kernel's prefetch is issued:
  // the leading run of passes with per-lane twiddles
  template <bool FWD>
  static constexpr int issue_after() {
    const bool lane[4] = {P0::LANE_TW, P1::LANE_TW, P2::LANE_TW, HAS3 ? Tail::LANE_TW : false};
    int k = 0;
    while (k < NP && lane[FWD ? k : NP - 1 - k]) ++k;
    return k;
  }
};
template <int LOGN, int PT, bool FWD>
using FirstPass = std::conditional_t<FWD, typename Sched<LOGN, PT>::P0, typename Sched<LOGN, PT>::Tail>;
template <int LOGN, int PT, bool FWD>
using LastPass = std::conditional_t<FWD, typename Sched<LOGN, PT>::Tail, typename Sched<LOGN, PT>::P0>;

struct NoIssue {
  __device__ void operator()() const {}
};

// x holds the first pass's operands on entry and the last pass's results on exit.  issue()
// enqueues the persistent kernel's prefetch of the next polynomial.  Vector loads complete in
// issue order, so a per-lane twiddle load issued after the prefetch is waited for only once
// the whole prefetch has arrived: issue() runs after the leading passes that load per-lane
// twiddles (before the first pass when it has none).
template <int LOGN, int PT, bool FWD, class Issue = NoIssue>
__device__ __forceinline__ void ntt_core(double* lds, double (&x)[PT], const double* tw, double q, double qi, int tid,
                                         const Issue& issue = Issue()) {
  using S = Sched<LOGN, PT>;
  using P0 = typename S::P0;
  using P1 = typename S::P1;
  using P2 = typename S::P2;
  using P3 = typename S::P3;
  constexpr int at = S::template issue_after<FWD>();  // passes run before issue()
  if constexpr (FWD) {
    if constexpr (at == 0) issue();
    P0::template run<true>(x, tw, q, qi, tid);
    if constexpr (at == 1) issue();
    relayout<P0, P1>(lds, x, tid);
    P1::template run<true>(x, tw, q, qi, tid);
    if constexpr (at == 2) issue();
    relayout<P1, P2>(lds, x, tid);
    P2::template run<true>(x, tw, q, qi, tid);
    if constexpr (at == 3) issue();
    if constexpr (S::HAS3) {
      relayout<P2, P3>(lds, x, tid);
      P3::template run<true>(x, tw, q, qi, tid);
      if constexpr (at == 4) issue();
    }
  } else {
    // pass k of the inverse runs Pass index NP - 1 - k
    if constexpr (at == 0) issue();
    if constexpr (S::HAS3) {
      P3::template run<false>(x, tw, q, qi, tid);
      if constexpr (at == 1) issue();
      relayout<P3, P2>(lds, x, tid);
    }
    P2::template run<false>(x, tw, q, qi, tid);
    if constexpr (at == S::NP - 2) issue();
    relayout<P2, P1>(lds, x, tid);
    P1::template run<false>(x, tw, q, qi, tid);
    if constexpr (at == S::NP - 1) issue();
    relayout<P1, P0>(lds, x, tid);
    P0::template run<false>(x, tw, q, qi, tid);
    if constexpr (at == S::NP) issue();
  }
}

template <int LOGN, int PT, bool FWD, class LoadOp>
__device__ __forceinline__ void ntt_load(double (&x)[PT], const PolyDesc& d, const LoadOp& ld, double q, double qi, int tid) {
#pragma unroll
  for (int i = 0; i < PT; ++i) x[i] = ld(d, FirstPass<LOGN, PT, FWD>::idx(tid, i), q, qi);
}

// canonical results of the last pass to global memory (the inverse applies N^-1 here; the
// lazy passes leave |x| below ~2.5 q, which canon_full brings into [0, q))
template <int LOGN, int PT, bool FWD, class StoreOp>
__device__ __forceinline__ void ntt_store(double (&x)[PT], const PolyDesc& d, const StoreOp& st, double q, double qi, double ninv, int tid,
                                          double* lds) {
  if constexpr (StoreOp::kPack) {  // the epilogue takes all of a work-item's results at once
    int j[PT];
    double v[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      j[i] = LastPass<LOGN, PT, FWD>::idx(tid, i);
      v[i] = FWD ? canon(x[i], q) : canon_full(mulmod_s(x[i], ninv, q, qi), q, qi);
    }
    st.template put_all<LOGN, PT>(d, j, v, lds, tid);
    return;
  }
  st.template prepare<PT>(d, lds, tid);  // the epilogue may stage an operand in LDS (free after the last pass)
  // Every operand load of the epilogue is issued before the first store: vector-memory
  // completion is tracked in issue order, so a load issued after a store could only be
  // consumed once that store had completed.
  typename StoreOp::Operand e[PT];
#pragma unroll
  for (int i = 0; i < PT; ++i) e[i] = st.fetch(d, LastPass<LOGN, PT, FWD>::idx(tid, i));
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int j = LastPass<LOGN, PT, FWD>::idx(tid, i);
    const double v = FWD ? canon(x[i], q) : canon_full(mulmod_s(x[i], ninv, q, qi), q, qi);
    st.put(d, j, v, e[i], q, qi, lds);
  }
}

// waves per SIMD the launch bounds promise: 4 (PT 16: 16 waves per workgroup at N = 16384, up
// to 128 VGPRs each) or 2 (PT 32: up to 256 VGPRs, room for 32 values and their prefetch)
template <int PT>
constexpr int waves_per_eu() { return PT == 32 ? 2 : 4; }

// One workgroup per polynomial.
template <int LOGN, int PT, bool FWD, class LoadOp, class StoreOp>
__global__ __launch_bounds__((1 << LOGN) / PT) __attribute__((amdgpu_waves_per_eu(waves_per_eu<PT>()))) void k_ntt(
    NttSrc descs, const double* __restrict__ tw_all, ModTable mt, LoadOp ld, StoreOp st) {
  constexpr int N = 1 << LOGN;
  __shared__ double lds[N + N / 16];
  const PolyDesc d = descs.get(blockIdx.x);
  const double q = mt.m[d.mod].q, qi = mt.m[d.mod].qinv;
  const int tid = threadIdx.x;
  double x[PT];
  ntt_load<LOGN, PT, FWD>(x, d, ld, q, qi, tid);
  ntt_core<LOGN, PT, FWD>(lds, x, tw_all + (size_t)d.mod * N, q, qi, tid);
  ntt_store<LOGN, PT, FWD>(x, d, st, q, qi, mt.m[d.mod].ninv, tid, lds);
}

// Persistent, software-pipelined variant: a grid of resident workgroups walks the descriptor
// list with a grid stride; the next polynomial's operands are loaded into registers while the
// current one is transformed, hiding the global-memory latency that a one-shot workgroup (one
// per CU at N = 16384) exposes.
template <int LOGN, int PT, bool FWD, class LoadOp, class StoreOp>
__global__ __launch_bounds__((1 << LOGN) / PT) __attribute__((amdgpu_waves_per_eu(waves_per_eu<PT>()))) void k_ntt_pipe(
    NttSrc descs, const double* __restrict__ tw_all, ModTable mt, LoadOp ld, StoreOp st, int count) {
  constexpr int N = 1 << LOGN;
  constexpr int PF = PT;
  using First = FirstPass<LOGN, PT, FWD>;
  __shared__ double lds[N + N / 16];
  const int tid0 = threadIdx.x;
  int p = blockIdx.x;
  if (p >= count) return;
  // The next polynomial's words are prefetched raw (converted only when its iteration starts, so
  // nothing waits for them earlier).  Vector-memory completion is tracked in issue order,
  // stores included: the only wait in an iteration is for its own prefetch, issued before the
  // previous iteration's stores.
  uint64_t nx[PF];
  {
    const PolyDesc d = descs.get(p);
#pragma unroll
    for (int i = 0; i < PF; ++i) nx[i] = ld.raw(d, First::idx(tid0, i));
    // the first polynomial's loads complete before the loop: registers still pending on entry
    // would make the loop head wait for the previous iteration's stores as well
#pragma unroll
    for (int i = 0; i < PF; ++i) asm volatile("" : "+v"(nx[i]));
  }
  for (;;) {
    // an opaque copy of the work-item index: keeps the compiler from hoisting every
    // index computation of the loop body out of the loop (which would spill registers)
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const PolyDesc d = descs.get(p);
    const double q = mt.m[d.mod].q, qi = mt.m[d.mod].qinv;
    double x[PT];
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      uint64_t u = nx[i];
      asm volatile("" : "+v"(u));  // the conversion stays in this iteration
      x[i] = ld.cvt(d, u, q, qi);
    }
#pragma unroll
    for (int i = PF; i < PT; ++i) x[i] = ld(d, First::idx(tid, i), q, qi);
    const int pn = p + gridDim.x;
    auto prefetch = [&] {
      // unconditional (the last iteration re-reads its own polynomial), so the loads land in nx
      // directly and are only waited for when the next iteration starts
      const PolyDesc dn = descs.get(pn < count ? pn : p);
#pragma unroll
      for (int i = 0; i < PF; ++i) nx[i] = ld.raw(dn, First::idx(tid, i));
    };
    ntt_core<LOGN, PT, FWD>(lds, x, tw_all + (size_t)d.mod * N, q, qi, tid, prefetch);
    ntt_store<LOGN, PT, FWD>(x, d, st, q, qi, mt.m[d.mod].ninv, tid, lds);
    p = pn;
    if (p >= count) break;
  }
}

template <int PT, bool FWD, class LoadOp, class StoreOp>
void launch_ntt_pt(blb_ctx* c, NttSrc d_descs, int count, LoadOp ld, StoreOp st) {
  const double* tw = FWD ? c->d_tw_fwd : c->d_tw_inv;
  const int threads = c->n / PT;
  if constexpr (StoreOp::kPersistent) {
    if (c->ntt_variant == 1) {
      // resident workgroups: LDS per workgroup is 8.5 N bytes of 160 KiB per CU
      const int per_cu = std::max(1, (160 * 1024) / (int)((c->n + c->n / 16) * sizeof(double)));
      const int grid = std::min(count, c->n_cu * per_cu);
      switch (c->log_n) {
        case 12: k_ntt_pipe<12, PT, FWD><<<grid, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st, count); break;
        case 13: k_ntt_pipe<13, PT, FWD><<<grid, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st, count); break;
        case 14: k_ntt_pipe<14, PT, FWD><<<grid, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st, count); break;
        default: break;
      }
      return;
    }
  }
  switch (c->log_n) {
    case 12: k_ntt<12, PT, FWD><<<count, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st); break;
    case 13: k_ntt<13, PT, FWD><<<count, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st); break;
    case 14: k_ntt<14, PT, FWD><<<count, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st); break;
    default: break;
  }
}
template <bool FWD, class LoadOp, class StoreOp>
void launch_ntt_generic(blb_ctx* c, NttSrc d_descs, int count, LoadOp ld, StoreOp st) {
  if (count <= 0) return;
  if (c->ntt_radix == 32) launch_ntt_pt<kPT32, FWD>(c, d_descs, count, ld, st);
  else launch_ntt_pt<kPT16, FWD>(c, d_descs, count, ld, st);
}

}  // namespace

// ---------------------------------------------------------------------------------------
// Load / store variants.  Descriptor pointers are global memory; accessing them through the
// global address space (not generic) keeps the loads off the LDS counter, so the LDS-only
// barriers do not wait for them, and lets a uniform base pointer stay in scalar registers.
// ---------------------------------------------------------------------------------------
typedef __attribute__((address_space(1))) uint64_t gu64;
__device__ __forceinline__ uint64_t gld(const uint64_t* p, int j) { return ((const gu64*)p)[j]; }
__device__ __forceinline__ void gst(uint64_t* p, int j, uint64_t v) { ((gu64*)p)[j] = v; }

// Loads: raw(d, j) fetches word j, cvt() turns it into this pass's double operand.
struct LdPlain {
  __device__ uint64_t raw(const PolyDesc& d, int j) const { return gld(d.src, j); }
  __device__ double cvt(const PolyDesc&, uint64_t u, double, double) const { return u2d(u); }
  __device__ double operator()(const PolyDesc& d, int j, double q, double qi) const { return cvt(d, raw(d, j), q, qi); }
};
// Stores: prepare() may stage an operand in LDS, fetch(d, j) loads the epilogue's global
// operand for word j, put() writes word j.
// kPersistent: whether the persistent kernel may run this epilogue.  The ModDown epilogue
// stages an operand through registers into LDS; next to a register prefetch of the following
// polynomial that no longer fits 128 VGPRs, so it always runs one polynomial per workgroup.
struct StPlain {
  static constexpr bool kPersistent = true;
  static constexpr bool kPack = false;
  struct Operand {};
  template <int PT>
  __device__ void prepare(const PolyDesc&, double*, int) const {}
  __device__ Operand fetch(const PolyDesc&, int) const { return {}; }
  __device__ void put(const PolyDesc& d, int j, double v, Operand, double, double, const double*) const { gst(d.dst, j, d2u(v)); }
};
// load a residue of another modulus (aux = that modulus as double) and lift it centred into
// this modulus: used by rescale (last limb -> limb i)
struct LdCentredLift {
  __device__ uint64_t raw(const PolyDesc& d, int j) const { return gld(d.src, j); }
  __device__ double cvt(const PolyDesc& d, uint64_t u, double q, double qi) const {
    const double v = u2d(u);
    const double ql = d.aux;
    const double t = v > 0.5 * ql ? v - ql : v;  // centred, |t| < q_l / 2
    return reduce_s(t, q, qi);
  }
  __device__ double operator()(const PolyDesc& d, int j, double q, double qi) const { return cvt(d, raw(d, j), q, qi); }
};
// rescale epilogue: dst[j] <- (c_i[j] - v) * q_l^-1 mod q_i, c_i = d.src2, aux2 = q_l^-1 mod q_i
struct StRescale {
  static constexpr bool kPersistent = true;
  static constexpr bool kPack = false;
  using Operand = uint64_t;
  template <int PT>
  __device__ void prepare(const PolyDesc&, double*, int) const {}
  __device__ Operand fetch(const PolyDesc& d, int j) const { return gld(d.src2, j); }
  __device__ void put(const PolyDesc& d, int j, double v, Operand ci, double q, double qi, const double*) const {
    const double r = mulmod_s(u2d(ci) - v, d.aux2, q, qi);
    gst(d.dst, j, d2u(canon(r, q)));
  }
};
// ModDown epilogue: dst[j] <- (u_i[j] - v) * P^-1 (+ add[j] if src3), u_i = src2 (u64).
// For a rotation add = sigma_g(c0), a permuted read of src3.  src3 is staged in LDS with
// coalesced reads (then read there, at the permuted index for a rotation), which keeps the
// epilogue's global loads to one word per output.
struct StModDown {
  static constexpr bool kPersistent = false;
  static constexpr bool kPack = false;
  using Operand = uint64_t;
  template <int PT>
  __device__ void prepare(const PolyDesc& d, double* lds, int tid) const {
    if (!d.src3) return;  // uniform over the workgroup (one descriptor)
    const int T = (1 << d.log_n) / PT;
    lds_barrier();
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int j = tid + i * T;
      lds[pad_idx(j)] = u2d(gld(d.src3, j));
    }
    lds_barrier();
  }
  __device__ Operand fetch(const PolyDesc& d, int j) const { return gld(d.src2, j); }
  __device__ void put(const PolyDesc& d, int j, double v, Operand ui, double q, double qi, const double* lds) const {
    double r = canon(mulmod_s(u2d(ui) - v, d.aux2, q, qi), q);
    if (d.src3) {
      r += lds[pad_idx(d.gal ? (int)gal_perm((uint32_t)j, d.gal, d.log_n) : j)];
      r = r >= q ? r - q : r;
    }
    gst(d.dst, j, d2u(r));
  }
};

// Plan epilogue: canonical results of a regular batch written in the 50-bit plan format (low
// 32 bits, next 16, top 2 in u32 words of 16; see pt50_bytes) at out + (poly index) x
// pt50_bytes(N), the poly index recovered from the batch's source address.  The top-bit codes
// are gathered in LDS (free after the last pass), then each u32 of 16 codes written once.
struct StPack50 {
  static constexpr bool kPersistent = false;
  static constexpr bool kPack = true;
  struct Operand {};
  const uint64_t* base;  // source of the regular batch (poly p at base + p N)
  uint8_t* out;          // packed destination of poly 0
  template <int LOGN, int PT>
  __device__ void put_all(const PolyDesc& d, const int (&j)[PT], const double (&v)[PT], double* lds, int tid) const {
    constexpr int N = 1 << LOGN, T = N / PT;
    const size_t p = (size_t)(d.src - base) >> LOGN;
    uint8_t* o = out + p * pt50_bytes(N);
    uint32_t* lo = (uint32_t*)o;
    uint16_t* mid = (uint16_t*)(o + (size_t)4 * N);
    uint32_t* top = (uint32_t*)(o + (size_t)6 * N);
    uint8_t* codes = (uint8_t*)lds;
    lds_barrier();  // every work-item is past its reads of the last exchange
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const uint64_t w = d2u(v[i]);
      lo[j[i]] = (uint32_t)w;
      mid[j[i]] = (uint16_t)(w >> 32);
      codes[j[i]] = (uint8_t)((w >> 48) & 3u);
    }
    lds_barrier();
    for (int t = tid; t < N / 16; t += T) {
      const uint32_t* c4 = (const uint32_t*)(codes + 16 * t);
      uint32_t word = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t x = c4[b];  // codes of words 4b .. 4b + 3, one per byte
        const uint32_t c = (x & 3u) | ((x >> 6) & 0xCu) | ((x >> 12) & 0x30u) | ((x >> 18) & 0xC0u);
        word |= c << (8 * b);
      }
      top[t] = word;
    }
  }
  template <int PT>
  __device__ void prepare(const PolyDesc&, double*, int) const {}
  __device__ Operand fetch(const PolyDesc&, int) const { return {}; }
  __device__ void put(const PolyDesc&, int, double, Operand, double, double, const double*) const {}
};

// add-into epilogue: dst[j] <- src2[j] + v mod q  (mask added to c0 in evaluation form)
struct StAddTo {
  static constexpr bool kPersistent = true;
  static constexpr bool kPack = false;
  using Operand = uint64_t;
  template <int PT>
  __device__ void prepare(const PolyDesc&, double*, int) const {}
  __device__ Operand fetch(const PolyDesc& d, int j) const { return gld(d.src2, j); }
  __device__ void put(const PolyDesc& d, int j, double v, Operand a, double q, double, const double*) const {
    double r = u2d(a) + v;
    r = r >= q ? r - q : r;
    gst(d.dst, j, d2u(r));
  }
};

static NttSrc table(blb_ctx* c, const PolyDesc* d_descs) { return NttSrc{d_descs, nullptr, 1, c->log_n}; }
void launch_ntt_addto(blb_ctx* c, const PolyDesc* d_descs, int count) {
  launch_ntt_generic<true>(c, table(c, d_descs), count, LdPlain{}, StAddTo{});
}
void launch_ntt(blb_ctx* c, const PolyDesc* d_descs, int count, bool fwd) {
  if (fwd) launch_ntt_generic<true>(c, table(c, d_descs), count, LdPlain{}, StPlain{});
  else launch_ntt_generic<false>(c, table(c, d_descs), count, LdPlain{}, StPlain{});
}
void launch_ntt_rescale(blb_ctx* c, const PolyDesc* d_descs, int count) {
  launch_ntt_generic<true>(c, table(c, d_descs), count, LdCentredLift{}, StRescale{});
}
void launch_ntt_moddown(blb_ctx* c, const PolyDesc* d_descs, int count) {
  launch_ntt_generic<true>(c, table(c, d_descs), count, LdPlain{}, StModDown{});
}
void launch_ntt_regular(blb_ctx* c, uint64_t* base, int count, int nl, bool fwd) {
  const NttSrc src{nullptr, base, nl, c->log_n};
  if (fwd) launch_ntt_generic<true>(c, src, count, LdPlain{}, StPlain{});
  else launch_ntt_generic<false>(c, src, count, LdPlain{}, StPlain{});
}
void launch_ntt_pack50(blb_ctx* c, const uint64_t* base, uint8_t* out, int count, int nl) {
  const NttSrc src{nullptr, (uint64_t*)base, nl, c->log_n};
  launch_ntt_generic<true>(c, src, count, LdPlain{}, StPack50{base, out});
}
