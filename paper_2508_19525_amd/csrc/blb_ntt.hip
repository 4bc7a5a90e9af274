// Batched negacyclic NTT / inverse NTT for gfx950 on FP64 lanes.
//
// One workgroup transforms one N-word polynomial (N = 4096 / 8192 / 16384) held in LDS
// (N doubles + 1/16 padding, 136 KiB at N = 16384 against 160 KiB per CU).  Each of the N/16
// work-items keeps 16 values in registers and runs up to four radix-2 stages on them per
// pass, so a transform costs ceil(log2 N / 4) LDS round trips.  The forward transform is the
// Cooley-Tukey ordering with twiddles psi^brv(m+i) (natural in, bit-reversed out, value j is
// the evaluation at psi^(2 brv(j) + 1)); the inverse is the Gentleman-Sande ordering with
// psi^-brv(m+i) followed by N^-1.  Polys are addressed through a descriptor table so a
// launch can gather from arbitrary buffers and moduli.
#include "blb_internal.h"
#include "blb_kernels.h"
#include <algorithm>

namespace {

constexpr int kPerThread = 16;

__device__ __forceinline__ int pad_idx(int j) { return j + (j >> 4); }

// One pass of R_LOG radix-2 stages, starting at global stage s0.  FWD selects Cooley-Tukey
// (stages in increasing order) or Gentleman-Sande (decreasing order, inverse twiddles).
template <int LOGN, int R_LOG, bool FWD>
__device__ __forceinline__ void ntt_pass(double* lds, const double* __restrict__ tw, int s0, double q, double qi) {
  constexpr int N = 1 << LOGN;
  constexpr int T = N / kPerThread;
  constexpr int GS = 1 << R_LOG;
  constexpr int GPT = kPerThread / GS;
  const int tid = threadIdx.x;
  const int t_last = N >> (s0 + R_LOG);
  double x[kPerThread];
  int his[GPT];
#pragma unroll
  for (int h = 0; h < GPT; ++h) {
    const int g = tid + h * T;
    const int lo = g % t_last, hi = g / t_last;
    his[h] = hi;
    const int base = hi * (t_last << R_LOG) + lo;
#pragma unroll
    for (int k = 0; k < GS; ++k) x[h * GS + k] = lds[pad_idx(base + k * t_last)];
  }
#pragma unroll
  for (int uu = 0; uu < R_LOG; ++uu) {
    const int u = FWD ? uu : (R_LOG - 1 - uu);
    const int t_loc = GS >> (u + 1);
#pragma unroll
    for (int h = 0; h < GPT; ++h) {
#pragma unroll
      for (int k = 0; k < GS; ++k) {
        if (k & t_loc) continue;
        const int widx = (1 << (s0 + u)) + (his[h] << u) + (k >> (R_LOG - u));
        const double w = tw[widx];
        double& a = x[h * GS + k];
        double& b = x[h * GS + k + t_loc];
        // lazy reduction: values are brought back to |x| <= q/2 only after every second stage
        // (and at the end of the pass); in between they stay below ~3.1 q < 2^52, where every
        // FP64 operation on them is exact and mulmod_s keeps |result| < 1.3 q.
        const bool red = (u & 1) || (u == R_LOG - 1);
        if (FWD) {
          const double v = mulmod_s(b, w, q, qi);
          const double s = a + v, d = a - v;
          a = red ? reduce_s(s, q, qi) : s;
          b = red ? reduce_s(d, q, qi) : d;
        } else {
          const double s = a + b, d = a - b;
          a = red ? reduce_s(s, q, qi) : s;
          b = mulmod_s(d, w, q, qi);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < GPT; ++h) {
    const int base = his[h] * (t_last << R_LOG) + ((tid + h * T) % t_last);
#pragma unroll
    for (int k = 0; k < GS; ++k) lds[pad_idx(base + k * t_last)] = x[h * GS + k];
  }
  __syncthreads();
}

template <int LOGN, bool FWD>
__device__ __forceinline__ void ntt_all_passes(double* lds, const double* tw, double q, double qi) {
  // passes of 4 stages, the remainder last (forward order); the inverse runs them reversed
  constexpr int REM = LOGN - 12;
  if (FWD) {
    ntt_pass<LOGN, 4, true>(lds, tw, 0, q, qi);
    ntt_pass<LOGN, 4, true>(lds, tw, 4, q, qi);
    ntt_pass<LOGN, 4, true>(lds, tw, 8, q, qi);
    if constexpr (REM > 0) ntt_pass<LOGN, (REM > 0 ? REM : 1), true>(lds, tw, 12, q, qi);
  } else {
    if constexpr (REM > 0) ntt_pass<LOGN, (REM > 0 ? REM : 1), false>(lds, tw, 12, q, qi);
    ntt_pass<LOGN, 4, false>(lds, tw, 8, q, qi);
    ntt_pass<LOGN, 4, false>(lds, tw, 4, q, qi);
    ntt_pass<LOGN, 4, false>(lds, tw, 0, q, qi);
  }
}

// Generic transform: load (LoadOp) -> passes -> store (StoreOp).  The load/store functors
// receive the descriptor, coefficient index and value.
template <int LOGN, bool FWD, class LoadOp, class StoreOp>
__global__ __launch_bounds__((1 << LOGN) / kPerThread) void k_ntt(const PolyDesc* __restrict__ descs, const double* __restrict__ tw_all,
                                                                ModTable mt, LoadOp ld, StoreOp st) {
  constexpr int N = 1 << LOGN;
  constexpr int T = N / kPerThread;
  __shared__ double lds[N + N / 16];
  const PolyDesc d = descs[blockIdx.x];
  const double q = mt.m[d.mod].q, qi = mt.m[d.mod].qinv;
  const double* tw = tw_all + (size_t)d.mod * N;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int j = tid + i * T;
    lds[pad_idx(j)] = ld(d, j, q, qi);
  }
  __syncthreads();
  ntt_all_passes<LOGN, FWD>(lds, tw, q, qi);
  if (!FWD) {
    const double ninv = mt.m[d.mod].ninv;
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const int j = tid + i * T;
      st(d, j, canon_full(mulmod_s(lds[pad_idx(j)], ninv, q, qi), q, qi), q, qi);
    }
  } else {
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const int j = tid + i * T;
      st(d, j, canon(lds[pad_idx(j)], q), q, qi);
    }
  }
}

// Persistent, software-pipelined variant: a grid of resident workgroups walks the descriptor
// list with a grid stride; the next polynomial's values are loaded into registers while the
// current one is transformed in LDS, hiding the global-memory latency that a one-shot
// workgroup (one per CU at N = 16384) exposes.
template <int LOGN, bool FWD, class LoadOp, class StoreOp>
__global__ __launch_bounds__((1 << LOGN) / kPerThread) void k_ntt_pipe(const PolyDesc* __restrict__ descs, const double* __restrict__ tw_all,
                                                                     ModTable mt, LoadOp ld, StoreOp st, int count) {
  constexpr int N = 1 << LOGN;
  constexpr int T = N / kPerThread;
  __shared__ double lds[N + N / 16];
  const int tid = threadIdx.x;
  int p = blockIdx.x;
  if (p >= count) return;
  double nx[kPerThread];
  {
    const PolyDesc d = descs[p];
    const double q = mt.m[d.mod].q, qi = mt.m[d.mod].qinv;
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) nx[i] = ld(d, tid + i * T, q, qi);
  }
  for (;;) {
    const PolyDesc d = descs[p];
    const double q = mt.m[d.mod].q, qi = mt.m[d.mod].qinv;
    const double* tw = tw_all + (size_t)d.mod * N;
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) lds[pad_idx(tid + i * T)] = nx[i];
    __syncthreads();
    const int pn = p + gridDim.x;
    if (pn < count) {  // prefetch the next polynomial while this one is transformed
      const PolyDesc dn = descs[pn];
      const double qn = mt.m[dn.mod].q, qin = mt.m[dn.mod].qinv;
#pragma unroll
      for (int i = 0; i < kPerThread; ++i) nx[i] = ld(dn, tid + i * T, qn, qin);
    }
    ntt_all_passes<LOGN, FWD>(lds, tw, q, qi);
    if (!FWD) {
      const double ninv = mt.m[d.mod].ninv;
#pragma unroll
      for (int i = 0; i < kPerThread; ++i) {
        const int j = tid + i * T;
        st(d, j, canon_full(mulmod_s(lds[pad_idx(j)], ninv, q, qi), q, qi), q, qi);
      }
    } else {
#pragma unroll
      for (int i = 0; i < kPerThread; ++i) {
        const int j = tid + i * T;
        st(d, j, canon(lds[pad_idx(j)], q), q, qi);
      }
    }
    __syncthreads();  // LDS is rewritten by the next iteration
    p = pn;
    if (p >= count) break;
  }
}

template <bool FWD, class LoadOp, class StoreOp>
void launch_ntt_generic(blb_ctx* c, const PolyDesc* d_descs, int count, LoadOp ld, StoreOp st) {
  if (count <= 0) return;
  const double* tw = FWD ? c->d_tw_fwd : c->d_tw_inv;
  const int threads = c->n / kPerThread;
  if (c->ntt_variant == 1) {
    // resident workgroups: LDS per workgroup is 8.5 N bytes of 160 KiB per CU
    const int per_cu = std::max(1, (160 * 1024) / (int)((c->n + c->n / 16) * sizeof(double)));
    const int grid = std::min(count, c->n_cu * per_cu);
    switch (c->log_n) {
      case 12: k_ntt_pipe<12, FWD><<<grid, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st, count); break;
      case 13: k_ntt_pipe<13, FWD><<<grid, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st, count); break;
      case 14: k_ntt_pipe<14, FWD><<<grid, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st, count); break;
      default: break;
    }
    return;
  }
  switch (c->log_n) {
    case 12: k_ntt<12, FWD><<<count, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st); break;
    case 13: k_ntt<13, FWD><<<count, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st); break;
    case 14: k_ntt<14, FWD><<<count, threads, 0, c->stream>>>(d_descs, tw, c->mt, ld, st); break;
    default: break;
  }
}

}  // namespace

// ---------------------------------------------------------------------------------------
// Load / store variants
// ---------------------------------------------------------------------------------------
struct LdPlain {
  __device__ double operator()(const PolyDesc& d, int j, double, double) const { return u2d(d.src[j]); }
};
struct StPlain {
  __device__ void operator()(const PolyDesc& d, int j, double v, double, double) const { d.dst[j] = d2u(v); }
};
// load a residue of another modulus (aux = that modulus as double) and lift it centred into
// this modulus: used by rescale (last limb -> limb i)
struct LdCentredLift {
  __device__ double operator()(const PolyDesc& d, int j, double q, double qi) const {
    const double v = u2d(d.src[j]);
    const double ql = d.aux;
    const double t = v > 0.5 * ql ? v - ql : v;  // centred, |t| < q_l / 2
    return reduce_s(t, q, qi);
  }
};
// rescale epilogue: dst[j] <- (c_i[j] - v) * q_l^-1 mod q_i, c_i = d.src2, aux2 = q_l^-1 mod q_i
struct StRescale {
  __device__ void operator()(const PolyDesc& d, int j, double v, double q, double qi) const {
    const double ci = u2d(d.src2[j]);
    const double r = mulmod_s(ci - v, d.aux2, q, qi);
    d.dst[j] = d2u(canon(r, q));
  }
};
// ModDown epilogue: dst[j] <- (u_i[j] - v) * P^-1 (+ add[j] if src3), u_i = src2 (u64)
struct StModDown {
  __device__ void operator()(const PolyDesc& d, int j, double v, double q, double qi) const {
    const double ui = u2d(d.src2[j]);
    double r = canon(mulmod_s(ui - v, d.aux2, q, qi), q);
    if (d.src3) {
      const uint32_t jj = d.gal ? gal_perm((uint32_t)j, d.gal, d.log_n) : (uint32_t)j;
      r += u2d(d.src3[jj]);
      r = r >= q ? r - q : r;
    }
    d.dst[j] = d2u(r);
  }
};

// add-into epilogue: dst[j] <- src2[j] + v mod q  (mask added to c0 in evaluation form)
struct StAddTo {
  __device__ void operator()(const PolyDesc& d, int j, double v, double q, double) const {
    double r = u2d(d.src2[j]) + v;
    r = r >= q ? r - q : r;
    d.dst[j] = d2u(r);
  }
};

void launch_ntt_addto(blb_ctx* c, const PolyDesc* d_descs, int count) {
  launch_ntt_generic<true>(c, d_descs, count, LdPlain{}, StAddTo{});
}
void launch_ntt(blb_ctx* c, const PolyDesc* d_descs, int count, bool fwd) {
  if (fwd) launch_ntt_generic<true>(c, d_descs, count, LdPlain{}, StPlain{});
  else launch_ntt_generic<false>(c, d_descs, count, LdPlain{}, StPlain{});
}
void launch_ntt_rescale(blb_ctx* c, const PolyDesc* d_descs, int count) {
  launch_ntt_generic<true>(c, d_descs, count, LdCentredLift{}, StRescale{});
}
void launch_ntt_moddown(blb_ctx* c, const PolyDesc* d_descs, int count) {
  launch_ntt_generic<true>(c, d_descs, count, LdPlain{}, StModDown{});
}
