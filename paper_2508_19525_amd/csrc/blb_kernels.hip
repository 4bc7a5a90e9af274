// Elementwise, sampling, key-switching, matmul_cp and encoder kernels for gfx950.
// All modular arithmetic is the FP64 signed-lazy scheme of blb_internal.h.
#include "blb_internal.h"
#include "blb_kernels.h"
#include <algorithm>
#include <type_traits>

// ---------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): 10 rounds, multipliers 0xD2511F53 / 0xCD9E8D57,
// key schedule increments 0x9E3779B9 / 0xBB67AE85.  Counter = (coefficient, limb, object,
// tag), key = (seed low word, seed high word).
// ---------------------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };
__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}
#define LIMB_INTEGER 0xFFFFFFFFu

// (w3 2^96 + w2 2^64 + w1 2^32 + w0) mod q by Horner steps r <- r*2^32 + w (mod q) on FP64
__device__ __forceinline__ double u128_mod(U4 w, double q, double qi) {
  const double two32 = 4294967296.0;
  double r = (double)w.w;  // < 2^32 < q
  r = canon_full(mulmod_s(r, two32, q, qi) + (double)w.z, q, qi);
  r = canon_full(mulmod_s(r, two32, q, qi) + (double)w.y, q, qi);
  r = canon_full(mulmod_s(r, two32, q, qi) + (double)w.x, q, qi);
  return r;
}

// out[limb][k] = uniform residue mod the limb's modulus; limb counter = mod index
__global__ void k_sample_uniform(uint64_t* out, int n, ModMap map, ModTable mt, uint32_t k0, uint32_t k1, uint32_t obj, uint32_t tag) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int limb = blockIdx.y;
  if (k >= n) return;
  const int m = map.idx[limb % map.len];
  const U4 w = philox10((uint32_t)k, (uint32_t)m, obj, tag, k0, k1);
  out[(size_t)limb * n + k] = d2u(u128_mod(w, mt.m[m].q, mt.m[m].qinv));
}

// integer samples reduced into every limb of the map.  mode 0: ternary (w0 mod 3) - 1;
// mode 1: Gaussian (CDT); mode F in [32, 48]: uniform integer in [-2^F, 2^F] (the 128-bit
// block mod 2^(F+1) + 1, minus 2^F; |v| <= 2^48 stays below every modulus)
__constant__ uint64_t c_cdt[20];
__global__ void k_sample_int(uint64_t* out, int n, int n_limbs, ModMap map, ModTable mt, uint32_t k0, uint32_t k1, uint32_t obj,
                             uint32_t tag, int mode) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const U4 w = philox10((uint32_t)k, LIMB_INTEGER, obj, tag, k0, k1);
  double v;
  if (mode == 1) {
    const uint64_t r = ((((uint64_t)w.y) << 32) | w.x) >> 1;
    int x = 0;
    while (x < 19 && r >= c_cdt[x]) ++x;
    v = (w.z & 1u) ? -x : x;
  } else if (mode == 0) {
    v = (double)((int)(w.x % 3u) - 1);
  } else {
    const double m = (double)((2ull << mode) + 1ull);
    v = u128_mod(w, m, 1.0 / m) - (double)(1ull << mode);
  }
  for (int l = 0; l < n_limbs; ++l) {
    const double q = mt.m[map.idx[l % map.len]].q;
    out[(size_t)l * n + k] = d2u(v < 0 ? q + v : v);
  }
}

void upload_cdt(const uint64_t* table20) { (void)hipMemcpyToSymbol(HIP_SYMBOL(c_cdt), table20, 20 * sizeof(uint64_t)); }

void launch_sample_uniform(blb_ctx* c, uint64_t* out, int n_limbs, ModMap map, uint64_t seed, uint32_t obj, uint32_t tag) {
  dim3 grid((c->n + 255) / 256, n_limbs);
  k_sample_uniform<<<grid, 256, 0, c->stream>>>(out, c->n, map, c->mt, (uint32_t)seed, (uint32_t)(seed >> 32), obj, tag);
}
void launch_sample_int(blb_ctx* c, uint64_t* out, int n_limbs, ModMap map, uint64_t seed, uint32_t obj, uint32_t tag, bool gaussian) {
  k_sample_int<<<(c->n + 255) / 256, 256, 0, c->stream>>>(out, c->n, n_limbs, map, c->mt, (uint32_t)seed, (uint32_t)(seed >> 32), obj,
                                                          tag, gaussian ? 1 : 0);
}
void launch_sample_flood(blb_ctx* c, uint64_t* out, int n_limbs, ModMap map, uint64_t seed, uint32_t obj, uint32_t tag, int bits) {
  k_sample_int<<<(c->n + 255) / 256, 256, 0, c->stream>>>(out, c->n, n_limbs, map, c->mt, (uint32_t)seed, (uint32_t)(seed >> 32), obj,
                                                          tag, bits);
}

// ---------------------------------------------------------------------------------------
// Elementwise ops over [count][N] u64 arrays (evaluation or coefficient form alike)
// ---------------------------------------------------------------------------------------
__global__ void k_ew(int op, uint64_t* out, const uint64_t* a, const uint64_t* b, const uint64_t* cc, int n, ModMap map, ModTable mt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (k >= n) return;
  const ModEntry me = mt.m[map.idx[p % map.len]];
  const size_t o = (size_t)p * n + k;
  const double x = u2d(a[o]);
  double r;
  switch (op) {
    case EW_ADD: { r = x + u2d(b[o]); r = r >= me.q ? r - me.q : r; break; }
    case EW_SUB: { r = x - u2d(b[o]); r = r < 0 ? r + me.q : r; break; }
    case EW_MUL: { r = canon(mulmod_s(x, u2d(b[o]), me.q, me.qinv), me.q); break; }
    case EW_NEG: { r = x == 0.0 ? 0.0 : me.q - x; break; }
    case EW_MULADD: { r = mulmod_s(x, u2d(b[o]), me.q, me.qinv) + u2d(cc[o]); r = canon_full(r, me.q, me.qinv); break; }
    default: { r = x; break; }
  }
  out[o] = d2u(r);
}
void launch_ew(blb_ctx* c, int op, uint64_t* out, const uint64_t* a, const uint64_t* b, const uint64_t* cc, int count, ModMap map) {
  if (count <= 0) return;
  dim3 grid((c->n + 255) / 256, count);
  k_ew<<<grid, 256, 0, c->stream>>>(op, out, a, b, cc, c->n, map, c->mt);
}

// encryption / key combination in evaluation form:
//   out0 = -a*s + e + extra     (extra optional: plaintext or P*s' term, added modularly)
__global__ void k_rlwe_combine(uint64_t* out0, const uint64_t* a, const uint64_t* s, const uint64_t* e, const uint64_t* extra,
                               LimbVals extra_mul, int n, ModMap map, ModTable mt) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (k >= n) return;
  const ModEntry me = mt.m[map.idx[l % map.len]];
  const size_t o = (size_t)l * n + k;
  double r = u2d(e[o]) - mulmod_s(u2d(a[o]), u2d(s[o]), me.q, me.qinv);  // (-q, 2q)
  if (extra) {
    double x = u2d(extra[o]);
    if (extra_mul.use) x = mulmod_s(x, extra_mul.v[l], me.q, me.qinv);
    r += x;
  }
  out0[o] = d2u(canon_full(r, me.q, me.qinv));
}
void launch_rlwe_combine(blb_ctx* c, uint64_t* out0, const uint64_t* a, const uint64_t* s, const uint64_t* e, const uint64_t* extra,
                         LimbVals extra_mul, int n_limbs, ModMap map) {
  dim3 grid((c->n + 255) / 256, n_limbs);
  k_rlwe_combine<<<grid, 256, 0, c->stream>>>(out0, a, s, e, extra, extra_mul, c->n, map, c->mt);
}

// evaluation-form automorphism of `count` polys
__global__ void k_automorph(uint64_t* out, const uint64_t* in, int n, int log_n, uint32_t g) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (k >= n) return;
  out[(size_t)p * n + k] = in[(size_t)p * n + gal_perm((uint32_t)k, g, log_n)];
}
void launch_automorph(blb_ctx* c, uint64_t* out, const uint64_t* in, int count, uint32_t g) {
  dim3 grid((c->n + 255) / 256, count);
  k_automorph<<<grid, 256, 0, c->stream>>>(out, in, c->n, c->log_n, g);
}

// ---------------------------------------------------------------------------------------
// Key switching
// ---------------------------------------------------------------------------------------
// ModUp: fast basis conversion (no centring) of digit j of each source, coefficient form.
//   x_m = sum_{i in D} [d_i * Qhat_i^-1]_{q_i} * [Qhat_i]_m  (mod m), for every extended
//   modulus m outside the digit.  Writes X[s][j][e][k] for those e.
// Thread per (s, j, k).
__global__ void k_modup(const uint64_t* dcoef, uint64_t* X, const KsLevelConst* kc, int n, int nl, int n_ext, int n_digits) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y % n_digits;
  const int s = blockIdx.y / n_digits;
  if (k >= n) return;
  const int lo = kc->dlo[j], hi = kc->dhi[j];
  double y[8];
#pragma unroll 4
  for (int i = lo; i < hi; ++i) {
    const ModEntry mq = kc->ext[i];
    y[i - lo] = canon(mulmod_s(u2d(dcoef[((size_t)s * nl + i) * n + k]), kc->qhat_inv[j][i - lo], mq.q, mq.qinv), mq.q);
  }
  for (int e = 0; e < n_ext; ++e) {
    if (e >= lo && e < hi) continue;
    const ModEntry mm = kc->ext[e];
    double acc = 0.0;
    for (int i = lo; i < hi; ++i) acc += mulmod_s(y[i - lo], kc->qhat_mod[j][i - lo][e], mm.q, mm.qinv);
    X[(((size_t)s * n_digits + j) * n_ext + e) * n + k] = d2u(canon_full(acc, mm.q, mm.qinv));
  }
}
void launch_modup(blb_ctx* c, const uint64_t* dcoef, uint64_t* X, const KsLevelConst* kc_dev, int n_src, int nl, int n_ext, int n_digits) {
  dim3 grid((c->n + 255) / 256, n_src * n_digits);
  k_modup<<<grid, 256, 0, c->stream>>>(dcoef, X, kc_dev, c->n, nl, n_ext, n_digits);
}

// Operands reached through descriptors in memory are addressed as global memory explicitly
// (global, not flat, loads and stores: a flat access also counts against the LDS / scalar wait
// counter and takes a 64-bit vector address).
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// Inner product with the switching key, with the automorphism applied to the extended
// digits (hoisted order).  Thread per (o, e, two adjacent k); writes U[o][2][e][k] (evaluation
// form).  For one wave the permuted reads stay inside one aligned block of 64 words: sigma_g
// keeps the low log2(N) - 6 bits of the exponent index, which bit reversal maps to the high
// bits of k.
__global__ void k_ks_inner(const KsOut* __restrict__ outs, const uint64_t* __restrict__ X, const KsLevelConst* __restrict__ kc,
                           uint64_t* __restrict__ U, int n, int log_n, int nl, int n_ext, int n_digits, int n_q) {
  const int k0 = (blockIdx.x * blockDim.x + threadIdx.x) * 2;
  const int e = blockIdx.y % n_ext;
  const int o = blockIdx.y / n_ext;
  if (k0 >= n) return;
  const KsOut od = outs[o];
  uint32_t kk[2];
#pragma unroll
  for (int v = 0; v < 2; ++v) kk[v] = od.gal ? gal_perm((uint32_t)(k0 + v), od.gal, log_n) : (uint32_t)(k0 + v);
  const ModEntry mm = kc->ext[e];
  const int key_mod = e < nl ? e : n_q + (e - nl);
  double acc0[2] = {0.0, 0.0}, acc1[2] = {0.0, 0.0};
  for (int j = 0; j < n_digits; ++j) {
    const auto xs = gmem((e >= kc->dlo[j] && e < kc->dhi[j]) ? od.c1 + (size_t)e * n : X + (((size_t)od.src * n_digits + j) * n_ext + e) * n);
    const auto kb = gmem(od.key + (((size_t)j * 2 + 0) * kc->n_key_mod + key_mod) * n + k0);
    const auto ka = gmem(od.key + (((size_t)j * 2 + 1) * kc->n_key_mod + key_mod) * n + k0);
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      const double x = u2d(xs[kk[v]]);
      acc0[v] += mulmod_s(x, u2d(kb[v]), mm.q, mm.qinv);
      acc1[v] += mulmod_s(x, u2d(ka[v]), mm.q, mm.qinv);
    }
    if ((j & 3) == 3) {  // keep |acc| < 5q < 2^53
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        acc0[v] = reduce_s(acc0[v], mm.q, mm.qinv);
        acc1[v] = reduce_s(acc1[v], mm.q, mm.qinv);
      }
    }
  }
  uint64_t* u0 = U + (((size_t)o * 2 + 0) * n_ext + e) * n + k0;
  uint64_t* u1 = U + (((size_t)o * 2 + 1) * n_ext + e) * n + k0;
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    u0[v] = d2u(canon_full(acc0[v], mm.q, mm.qinv));
    u1[v] = d2u(canon_full(acc1[v], mm.q, mm.qinv));
  }
}
void launch_ks_inner(blb_ctx* c, const KsOut* outs_dev, int n_out, const uint64_t* X, const KsLevelConst* kc_dev, uint64_t* U, int nl,
                     int n_ext, int n_digits) {
  dim3 grid((c->n / 2 + 255) / 256, n_out * n_ext);
  k_ks_inner<<<grid, 256, 0, c->stream>>>(outs_dev, X, kc_dev, U, c->n, c->log_n, nl, n_ext, n_digits, c->n_q);
}

// The same inner product for a group of outputs that share a switching key and Galois element:
// the key words of the thread's two coefficients are loaded once (all digits, in registers) and
// applied to every output of the group; per output the arithmetic and its order are those of
// k_ks_inner, so the words are identical.
__global__ void k_ks_inner_grp(const KsOut* __restrict__ outs, const int* __restrict__ ord, const KsGroup* __restrict__ groups,
                               const uint64_t* __restrict__ X, const KsLevelConst* __restrict__ kc, uint64_t* __restrict__ U, int n,
                               int log_n, int nl, int n_ext, int n_digits, int n_q) {
  const int k0 = (blockIdx.x * blockDim.x + threadIdx.x) * 2;
  const int e = blockIdx.y % n_ext;
  const int gi = blockIdx.y / n_ext;
  if (k0 >= n) return;
  const KsGroup gr = groups[gi];
  const KsOut lead = outs[ord[gr.first]];
  uint32_t kk[2];
#pragma unroll
  for (int v = 0; v < 2; ++v) kk[v] = lead.gal ? gal_perm((uint32_t)(k0 + v), lead.gal, log_n) : (uint32_t)(k0 + v);
  const ModEntry mm = kc->ext[e];
  const int key_mod = e < nl ? e : n_q + (e - nl);
  double kb[kKsMaxDigits][2], ka[kKsMaxDigits][2];
#pragma unroll
  for (int j = 0; j < kKsMaxDigits; ++j) {
    if (j < n_digits) {
      const auto b = gmem(lead.key + (((size_t)j * 2 + 0) * kc->n_key_mod + key_mod) * n + k0);
      const auto a = gmem(lead.key + (((size_t)j * 2 + 1) * kc->n_key_mod + key_mod) * n + k0);
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        kb[j][v] = u2d(b[v]);
        ka[j][v] = u2d(a[v]);
      }
    }
  }
  for (int i = 0; i < gr.count; ++i) {
    const int o = ord[gr.first + i];
    const KsOut od = outs[o];
    double acc0[2] = {0.0, 0.0}, acc1[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < kKsMaxDigits; ++j) {
      if (j < n_digits) {
        const auto xs = gmem((e >= kc->dlo[j] && e < kc->dhi[j]) ? od.c1 + (size_t)e * n : X + (((size_t)od.src * n_digits + j) * n_ext + e) * n);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          const double x = u2d(xs[kk[v]]);
          acc0[v] += mulmod_s(x, kb[j][v], mm.q, mm.qinv);
          acc1[v] += mulmod_s(x, ka[j][v], mm.q, mm.qinv);
        }
        if ((j & 3) == 3) {
#pragma unroll
          for (int v = 0; v < 2; ++v) {
            acc0[v] = reduce_s(acc0[v], mm.q, mm.qinv);
            acc1[v] = reduce_s(acc1[v], mm.q, mm.qinv);
          }
        }
      }
    }
    uint64_t* u0 = U + (((size_t)o * 2 + 0) * n_ext + e) * n + k0;
    uint64_t* u1 = U + (((size_t)o * 2 + 1) * n_ext + e) * n + k0;
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      u0[v] = d2u(canon_full(acc0[v], mm.q, mm.qinv));
      u1[v] = d2u(canon_full(acc1[v], mm.q, mm.qinv));
    }
  }
}
void launch_ks_inner_grouped(blb_ctx* c, const KsOut* outs_dev, const int* ord_dev, const KsGroup* groups_dev, int n_groups,
                             const uint64_t* X, const KsLevelConst* kc_dev, uint64_t* U, int nl, int n_ext, int n_digits) {
  dim3 grid((c->n / 2 + 255) / 256, n_groups * n_ext);
  k_ks_inner_grp<<<grid, 256, 0, c->stream>>>(outs_dev, ord_dev, groups_dev, X, kc_dev, U, c->n, c->log_n, nl, n_ext, n_digits, c->n_q);
}

// ModDown conversion: corr_i = sum_t [u_{p_t} * Phat_t^-1]_{p_t} * [Phat_t]_{q_i}  (coefficient
// form; U's special limbs must already be in coefficient form).  Thread per (o, poly, k).
__global__ void k_moddown_conv(const uint64_t* U, uint64_t* Corr, const KsLevelConst* kc, int n, int nl, int n_ext, int n_sp) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int op = blockIdx.y;  // o * 2 + poly
  if (k >= n) return;
  double y[4];
  for (int t = 0; t < n_sp; ++t) {
    const ModEntry mp = kc->ext[nl + t];
    y[t] = canon(mulmod_s(u2d(U[((size_t)op * n_ext + nl + t) * n + k]), kc->phat_inv[t], mp.q, mp.qinv), mp.q);
  }
  for (int i = 0; i < nl; ++i) {
    const ModEntry mq = kc->ext[i];
    double acc = 0.0;
    for (int t = 0; t < n_sp; ++t) acc += mulmod_s(y[t], kc->phat_mod[t][i], mq.q, mq.qinv);
    Corr[((size_t)op * nl + i) * n + k] = d2u(canon_full(acc, mq.q, mq.qinv));
  }
}
void launch_moddown_conv(blb_ctx* c, const uint64_t* U, uint64_t* Corr, const KsLevelConst* kc_dev, int n_out, int nl, int n_ext) {
  dim3 grid((c->n + 255) / 256, n_out * 2);
  k_moddown_conv<<<grid, 256, 0, c->stream>>>(U, Corr, kc_dev, c->n, nl, n_ext, c->n_sp);
}

// ---------------------------------------------------------------------------------------
// matmul_cp inner sums:  inner[bj][p][limb] = sum_{ai} pt[bj][ai][limb] (.) RX[ai][p][limb]
// Thread per (coefficient k, limb) for a tile of TB outputs.  The plaintext stream is read
// exactly once; RX tiles are re-read per output tile (L2 / MALL resident).
// ---------------------------------------------------------------------------------------
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Words k .. k + CPT - 1 (k even when CPT = 2) of a plan limb-poly in the 50-bit format at p,
// fetched raw (nontemporal: the plan stream is read once per call) and rebuilt as doubles:
// 2^52 + w has the high word 0x43300000 | w >> 32 and the low word w & 0xFFFFFFFF.
template <int CPT>
struct Pt50Raw {
  uint32_t lo[CPT];
  uint32_t mid[(CPT + 1) / 2];  // bits 32..47 of two words per u32 (the even word in the low half)
  uint32_t top;
};
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// (p may come from a descriptor in memory: the planes are addressed as global memory explicitly,
// so the loads are global, not flat, ones)
template <int CPT>
__device__ __forceinline__ void pt50_fetch(const uint8_t* __restrict__ p, int n, int k, Pt50Raw<CPT>& r) {
  typedef __attribute__((address_space(1))) const uint32_t g32;
  typedef __attribute__((address_space(1))) const uint16_t g16;
  typedef __attribute__((address_space(1))) const u32x2 g32x2;
  typedef __attribute__((address_space(1))) const u32x4 g32x4;
  g32* lo = (g32*)p;
  g16* mid = (g16*)(p + (size_t)4 * n);
  g32* top = (g32*)(p + (size_t)6 * n);
  if constexpr (CPT == 4) {
    const u32x4 l = __builtin_nontemporal_load((g32x4*)(lo + k));
    r.lo[0] = l.x;
    r.lo[1] = l.y;
    r.lo[2] = l.z;
    r.lo[3] = l.w;
    const u32x2 m = __builtin_nontemporal_load((g32x2*)(mid + k));
    r.mid[0] = m.x;
    r.mid[1] = m.y;
  } else if constexpr (CPT == 2) {
    const u32x2 l = __builtin_nontemporal_load((g32x2*)(lo + k));
    r.lo[0] = l.x;
    r.lo[1] = l.y;
    r.mid[0] = __builtin_nontemporal_load((g32*)(mid + k));
  } else {
    r.lo[0] = __builtin_nontemporal_load(lo + k);
    r.mid[0] = __builtin_nontemporal_load(mid + k);
  }
  r.top = __builtin_nontemporal_load(top + (k >> 4));
}
__device__ __forceinline__ double pt50_make(uint32_t lo, uint32_t mid16, uint32_t top2) {
  return __hiloint2double((int)(0x43300000u | (top2 << 16) | mid16), (int)lo) - BLB_TWO52;
}
template <int CPT>
__device__ __forceinline__ void pt50_cvt(const Pt50Raw<CPT>& r, int k, double (&v)[CPT]) {
  const uint32_t t = r.top >> (2 * (k & 15));
#pragma unroll
  for (int j = 0; j < CPT; ++j) v[j] = pt50_make(r.lo[j], (j & 1) ? r.mid[j / 2] >> 16 : r.mid[j / 2] & 0xFFFFu, (t >> (2 * j)) & 3u);
}


// One block's (tile, k-chunk, limb): sums over the n_ai rotated inputs of plaintext x input,
// for `rows` output rows of the tile (FULL: rows == TB, no row clamping).
template <int TB, int CPT, int UNR, bool FULL, bool P50>
__device__ __forceinline__ void cp_mac_tile(const uint8_t* __restrict__ pbase, const uint64_t* const* __restrict__ rx_tab,
                                            size_t pt_stride_bj, size_t pt_stride_ai, int n, int nl, int n_ai, int limb, int k0, int rows,
                                            double q, double qi, double (&a0)[TB][CPT], double (&a1)[TB][CPT]) {
  typedef __attribute__((address_space(1))) const uint64_t gu64;
  typedef __attribute__((address_space(1))) const u64x2 gu64x2;
  // STREAM: non-temporal loads (the plaintexts, read once); the rotated inputs, re-read by
  // every tile, stay cached.  A compile-time choice: a select between the two forms of the load
  // is merged into one plain load by the optimizer, which drops the non-temporal hint.
  auto load2 = [&](auto stream, gu64* a, double (&v)[CPT]) {
    constexpr bool STREAM = decltype(stream)::value;
    if constexpr (CPT >= 2) {
#pragma unroll
      for (int h = 0; h < CPT; h += 2) {
        u64x2 w;
        if constexpr (STREAM) w = __builtin_nontemporal_load((gu64x2*)(a + h));
        else w = *(gu64x2*)(a + h);
        v[h] = u2d(w.x);
        v[h + 1] = u2d(w.y);
      }
    } else {
      if constexpr (STREAM) v[0] = u2d(__builtin_nontemporal_load(a));
      else v[0] = u2d(*a);
    }
  };
  using kStream = std::true_type;
  using kCached = std::false_type;
  // Row pointers: the rows past a partial tile's last re-read that row, so every row of the
  // body runs unconditionally (branch-free, loads of all rows in flight together); their sums
  // are never stored.
  const uint8_t* rowp[TB];
#pragma unroll
  for (int t = 0; t < TB; ++t) rowp[t] = pbase + (size_t)(FULL ? t : min(t, rows - 1)) * pt_stride_bj;
  // poly: the (tile row, term) plaintext limb-poly
  auto load_pt = [&](const uint8_t* poly, double (&v)[CPT]) {
    if constexpr (P50) {
      Pt50Raw<CPT> r;
      pt50_fetch<CPT>(poly, n, k0, r);
      pt50_cvt<CPT>(r, k0, v);
    } else {
      load2(kStream{}, (gu64*)poly + k0, v);
    }
  };
  auto reduce_all = [&]() {
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int c = 0; c < CPT; ++c) { a0[t][c] = reduce_s(a0[t][c], q, qi); a1[t][c] = reduce_s(a1[t][c], q, qi); }
  };
  int ai = 0;
  for (; ai + UNR <= n_ai; ai += UNR) {
    double x0[UNR][CPT], x1[UNR][CPT], w[UNR][TB][CPT];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      gu64* rx = (gu64*)rx_tab[ai + u];
      load2(kCached{}, rx + (size_t)limb * n + k0, x0[u]);
      load2(kCached{}, rx + (size_t)(nl + limb) * n + k0, x1[u]);
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int t = 0; t < TB; ++t) load_pt(rowp[t] + (size_t)(ai + u) * pt_stride_ai, w[u][t]);
#pragma unroll
    for (int u = 0; u < UNR; ++u)
#pragma unroll
      for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          a0[t][c] += mulmod_s(w[u][t][c], x0[u][c], q, qi);
          a1[t][c] += mulmod_s(w[u][t][c], x1[u][c], q, qi);
        }
    if (((ai + UNR) & 7) == 0) reduce_all();  // every 8 terms: |acc| stays below 2^53
  }
  for (; ai < n_ai; ++ai) {
    double x0[CPT], x1[CPT], w[TB][CPT];
    gu64* rx = (gu64*)rx_tab[ai];
    load2(kCached{}, rx + (size_t)limb * n + k0, x0);
    load2(kCached{}, rx + (size_t)(nl + limb) * n + k0, x1);
#pragma unroll
    for (int t = 0; t < TB; ++t) load_pt(rowp[t] + (size_t)ai * pt_stride_ai, w[t]);
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        a0[t][c] += mulmod_s(w[t][c], x0[c], q, qi);
        a1[t][c] += mulmod_s(w[t][c], x1[c], q, qi);
      }
    if ((ai & 7) == 7) reduce_all();
  }
}

// SPLIT: full tiles run a body without row clamping (separately compiled from the clamped
// body of the last, partial tile); otherwise the clamped body serves every tile.
template <int TB, int CPT, int UNR, bool SPLIT, bool P50>
__global__ __launch_bounds__(256) void k_cp_mac(const uint64_t* __restrict__ pt, const uint64_t* const* __restrict__ rx_tab,
                                                uint64_t* __restrict__ inner, int n, int nl, int n_ai, int n_bj, ModTable mt, int n_kblk,
                                                int n_tiles) {
  static_assert(CPT == 1 || CPT == 2 || CPT == 4, "coefficients per thread");
  static_assert(UNR == 1 || UNR == 2, "unroll of the input loop");
  // Block order: k-chunk fastest, then limb, then output tile.  Consecutive blocks stream
  // consecutive 4 KB pieces of one plaintext limb-poly (the dispatcher deals them round-robin
  // over the 8 XCDs), and the blocks of one (k-chunk, limb) -- the ones reading the same
  // rotated-input words -- lie n_kblk * nl apart, a multiple of 8 whenever n_kblk is: one XCD,
  // one L2.  (A tile-fastest order with those readers adjacent on one XCD misses L2 less often
  // but ran 4-5 % slower on the BERT-base operator.)
  const int kb = blockIdx.x % n_kblk;
  const int limb = (blockIdx.x / n_kblk) % nl;
  const int tile = blockIdx.x / (n_kblk * nl);
  (void)n_tiles;
  const int k0 = (kb * 256 + threadIdx.x) * CPT;
  if (k0 >= n) return;
  const ModEntry me = mt.m[limb];
  const double q = me.q, qi = me.qinv;
  const int bj0 = tile * TB;
  const int rows = min(TB, n_bj - bj0);
  double a0[TB][CPT], a1[TB][CPT];
#pragma unroll
  for (int t = 0; t < TB; ++t)
#pragma unroll
    for (int c = 0; c < CPT; ++c) { a0[t][c] = 0.0; a1[t][c] = 0.0; }
  const size_t pb = pt_poly_bytes(n, P50);
  const size_t pt_stride_ai = (size_t)nl * pb, pt_stride_bj = (size_t)n_ai * pt_stride_ai;
  const uint8_t* pbase = (const uint8_t*)pt + (size_t)bj0 * pt_stride_bj + (size_t)limb * pb;
  if (SPLIT && rows == TB)
    cp_mac_tile<TB, CPT, UNR, true, P50>(pbase, rx_tab, pt_stride_bj, pt_stride_ai, n, nl, n_ai, limb, k0, rows, q, qi, a0, a1);
  else cp_mac_tile<TB, CPT, UNR, false, P50>(pbase, rx_tab, pt_stride_bj, pt_stride_ai, n, nl, n_ai, limb, k0, rows, q, qi, a0, a1);
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    if (t < rows) {
      uint64_t* o0 = inner + (((size_t)(bj0 + t) * 2 + 0) * nl + limb) * n + k0;
      uint64_t* o1 = inner + (((size_t)(bj0 + t) * 2 + 1) * nl + limb) * n + k0;
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        o0[c] = d2u(canon_full(a0[t][c], q, qi));
        o1[c] = d2u(canon_full(a1[t][c], q, qi));
      }
    }
  }
}

// Tuning knob (does not change any result bit): outputs per block x coefficients per thread
// x unroll of the input loop x split full / partial tiles.
void launch_cp_mac(blb_ctx* c, const uint64_t* pt, const uint64_t* const* rx_tab, uint64_t* inner, int nl, int n_ai, int n_bj, int variant,
                   int p50) {
  struct Shape { int tb, cpt; };
  static const Shape shapes[BLB_MAC_VARIANTS] = {{8, 2}, {8, 1}, {16, 2}, {4, 2}, {12, 2}, {2, 2}, {4, 2}, {2, 2}, {4, 1}, {4, 1},
                                                 {4, 2}, {4, 2}, {8, 1}, {4, 1}, {2, 4}, {4, 4}, {2, 4}, {4, 4}};
  const Shape sh = shapes[(variant >= 0 && variant < BLB_MAC_VARIANTS) ? variant : 0];
  const int n_kblk = c->n / (256 * sh.cpt);
  const int n_tiles = (n_bj + sh.tb - 1) / sh.tb;
  const int blocks = n_kblk * nl * n_tiles;
#define CPMAC(tb, cpt, unr, split)                                                                                                 \
  do {                                                                                                                             \
    if (p50) k_cp_mac<tb, cpt, unr, split, true><<<blocks, 256, 0, c->stream>>>(pt, rx_tab, inner, c->n, nl, n_ai, n_bj, c->mt, n_kblk, n_tiles); \
    else k_cp_mac<tb, cpt, unr, split, false><<<blocks, 256, 0, c->stream>>>(pt, rx_tab, inner, c->n, nl, n_ai, n_bj, c->mt, n_kblk, n_tiles); \
  } while (0)
  switch (variant) {
    case 1: CPMAC(8, 1, 1, false); break;
    case 2: CPMAC(16, 2, 1, false); break;
    case 3: CPMAC(4, 2, 1, false); break;
    case 4: CPMAC(12, 2, 1, false); break;
    case 5: CPMAC(2, 2, 1, false); break;
    case 6: CPMAC(4, 2, 2, false); break;
    case 7: CPMAC(2, 2, 2, false); break;
    case 8: CPMAC(4, 1, 1, false); break;
    case 9: CPMAC(4, 1, 2, false); break;
    case 10: CPMAC(4, 2, 2, true); break;
    case 11: CPMAC(4, 2, 1, true); break;
    case 12: CPMAC(8, 1, 1, true); break;
    case 13: CPMAC(4, 1, 2, true); break;
    case 14: CPMAC(2, 4, 1, false); break;
    case 15: CPMAC(4, 4, 1, false); break;
    case 16: CPMAC(2, 4, 1, true); break;
    case 17: CPMAC(4, 4, 1, true); break;
    default: CPMAC(8, 2, 1, false); break;
  }
#undef CPMAC
}

// out[o] = sum_t src[o * n_terms + t] over whole ciphertexts ([2][nl][N] words), mod q_limb
__global__ void k_sum_cts(const uint64_t* const* __restrict__ srcs, uint64_t* const* __restrict__ dsts, int n_terms, int n, int nl,
                          ModTable mt) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int o = blockIdx.y;
  if (w >= 2 * nl * n) return;
  const ModEntry me = mt.m[(w / n) % nl];
  double acc = 0.0;
  for (int t = 0; t < n_terms; ++t) {
    acc += u2d(gmem(srcs[(size_t)o * n_terms + t])[w]);
    if ((t & 3) == 3) acc = reduce_s(acc, me.q, me.qinv);
  }
  gmem(dsts[o])[w] = d2u(canon_full(acc, me.q, me.qinv));
}
void launch_sum_cts(blb_ctx* c, const uint64_t* const* srcs, uint64_t* const* dsts, int n_out, int n_terms, int nl) {
  dim3 grid((2 * nl * c->n + 255) / 256, n_out);
  k_sum_cts<<<grid, 256, 0, c->stream>>>(srcs, dsts, n_terms, c->n, nl, c->mt);
}

// ---------------------------------------------------------------------------------------
// Mask-and-share: r uniform per limb in coefficient form (tag mask, object = ct index),
// share = -r mod q_i; the mask is added to c0 in evaluation form by the caller after an NTT.
// ---------------------------------------------------------------------------------------
__global__ void k_mask_sample(uint64_t* r_out, uint64_t* share, int n, int tl, ModTable mt, uint32_t k0, uint32_t k1,
                              const uint64_t* seed_dev, uint32_t tag) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y % tl;
  const int t = blockIdx.y / tl;
  if (k >= n) return;
  if (seed_dev) {
    const uint64_t sd = *seed_dev;
    k0 = (uint32_t)sd;
    k1 = (uint32_t)(sd >> 32);
  }
  const ModEntry me = mt.m[i];
  const U4 w = philox10((uint32_t)k, (uint32_t)i, (uint32_t)t, tag, k0, k1);
  const double r = u128_mod(w, me.q, me.qinv);
  const size_t o = ((size_t)t * tl + i) * n + k;
  r_out[o] = d2u(r);
  share[o] = d2u(r == 0.0 ? 0.0 : me.q - r);
}
void launch_mask_sample(blb_ctx* c, uint64_t* r_out, uint64_t* share, int n_ct, int tl, uint64_t seed, const uint64_t* seed_dev,
                        uint32_t tag) {
  dim3 grid((c->n + 255) / 256, n_ct * tl);
  k_mask_sample<<<grid, 256, 0, c->stream>>>(r_out, share, c->n, tl, c->mt, (uint32_t)seed, (uint32_t)(seed >> 32), seed_dev, tag);
}

__global__ void k_set_u64(uint64_t* dst, uint64_t v) { *dst = v; }
void launch_set_u64(blb_ctx* c, uint64_t* dst, uint64_t value) { k_set_u64<<<1, 1, 0, c->stream>>>(dst, value); }

__global__ void k_zero(uint64_t* dst, size_t words) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) dst[i] = 0;
}
void launch_zero(blb_ctx* c, uint64_t* dst, size_t words) {
  if (!words) return;
  k_zero<<<(unsigned)((words + 255) / 256), 256, 0, c->stream>>>(dst, words);
}

// ---------------------------------------------------------------------------------------
// Encoder (eq. ckks_encode) in double-double arithmetic.
//   Slot j sits at zeta^(e_j), e_j = 5^j mod 2N = 4 u_j + 1.  With w_k = p_k + i p_{k+M}
//   (M = N/2), p(zeta^(4u+1)) = sum_k zeta^k w_k eta^(uk), eta = exp(2 pi i / M), so
//   w_k = zeta^-k (1/M) sum_u v_u eta^(-uk) with v_u the (real) slot value at u.
//   Steps: DFT of size M (exp(-i...)) of the slot values placed at their positions u, then
//   finalize (twist, scale, round half away from zero, reduce into the limbs).
// ---------------------------------------------------------------------------------------
struct dd { double hi, lo; };
__device__ __forceinline__ dd two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  const double err = (a - (s - bb)) + (b - bb);
  return dd{s, err};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  const double s = a + b;
  return dd{s, b - (s - a)};
}
__device__ __forceinline__ dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  dd t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd x) { return dd{-x.hi, -x.lo}; }
__device__ __forceinline__ dd dd_mul(dd x, dd y) {
  const double p = x.hi * y.hi;
  double e = __builtin_fma(x.hi, y.hi, -p);
  e += x.hi * y.lo + x.lo * y.hi;
  return quick_two_sum(p, e);
}
__device__ __forceinline__ dd dd_mul_d(dd x, double y) {
  const double p = x.hi * y;
  double e = __builtin_fma(x.hi, y, -p);
  e += x.lo * y;
  return quick_two_sum(p, e);
}
struct cdd { dd re, im; };
__device__ __forceinline__ cdd cdd_mul(cdd a, cdd b) {
  return cdd{dd_add(dd_mul(a.re, b.re), dd_neg(dd_mul(a.im, b.im))), dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
}
__device__ __forceinline__ cdd cdd_add(cdd a, cdd b) { return cdd{dd_add(a.re, b.re), dd_add(a.im, b.im)}; }
__device__ __forceinline__ cdd cdd_sub(cdd a, cdd b) { return cdd{dd_add(a.re, dd_neg(b.re)), dd_add(a.im, dd_neg(b.im))}; }
__device__ __forceinline__ cdd ld_cdd(const double* p) { return cdd{dd{p[0], p[1]}, dd{p[2], p[3]}}; }
__device__ __forceinline__ void st_cdd(double* p, cdd v) { p[0] = v.re.hi; p[1] = v.re.lo; p[2] = v.im.hi; p[3] = v.im.lo; }

// Slot values.  Position u of the DFT input holds slot j = slot_inv[u] (u_j = (5^j mod 2N - 1) / 4).
// Dense source: vals[p][j], n_vals per plaintext, one plaintext per complex vector.
// begin(p) gathers what is uniform over complex vector p, (ctx, u) gives the value at u.
struct EncSrcDense {
  const double* vals;
  int n_vals;
  const int32_t* slot_inv;
  __device__ const double* begin(int p) const { return vals + (size_t)p * n_vals; }
  __device__ cdd operator()(const double* v, int u) const {
    const int j = slot_inv[u];
    return cdd{dd{j < n_vals ? v[j] : 0.0, 0.0}, dd{0.0, 0.0}};
  }
};

// matmul_cp diagonal plaintexts, two per complex vector (plaintext p0 + 2 pp in the real part,
// p0 + 2 pp + 1 in the imaginary part, split apart after the transform); with the complex-slot
// output packing (g.cplx) one plaintext per complex vector, whose slots hold the diagonal of
// output block 2b in the real and that of block 2b + 1 in the imaginary part; plaintext p = (bj, ai):
//   value at slot s = W{a c + ((u + t) mod c_eff), b c + (u mod c_out)}, u = ((s - r) mod S) / L',
//   t = jB + i, r = j B L' (plaintext pre-rotated right by r).
// L', c, c_eff, c_out and S are powers of two (lLp = log2 L').
// Plaintext diagonals of matmul_cp: diagonal (b, j, a, i) pre-rotated right by j B L' slots,
// block u of the unrotated vector holding W{row, b c + (u mod c_out)} where, with
// u' = (u + j B + i) mod c_eff, row = a c + u' for a spatial-first input (broadcast over the
// L' slots of the block) or, for a diagonal-packed input (dg.tab set), row = h d_v + (r + tau)
// mod d_v' at slot r of the block, (h, tau) being the head and diagonal that block u' of input
// a holds (0 for r >= L or a padded column).
struct EncSrcCp {
  const double* W;
  CpGeom g;
  int p0, count, M, lLp;
  const int32_t* slot_inv;
  CpDiag dg;
  struct Diag {
    int r, t, row0, col0;
    bool used;
    CpDiagIn in;
  };
  struct Pair {
    Diag x, y;
  };
  __device__ Diag diag(int p, int half) const {
    const int n_ai = g.n_in * g.B;
    const int bj = p / n_ai, ai = p % n_ai;
    const int b = g.cplx ? 2 * (bj / g.G) + half : bj / g.G, j = bj % g.G;
    const int a = ai / g.B, i = ai % g.B;
    const bool used = p < p0 + count;
    const CpDiagIn in = (dg.tab && used) ? dg.tab[a] : CpDiagIn{0, 0, 1, 0};
    return Diag{j * g.B * g.Lp, j * g.B + i, a * g.c, b * g.c, used, in};
  }
  __device__ double value(const Diag& d, int s) const {
    if (!d.used) return 0.0;
    const int sr = (s - d.r) & (M - 1);
    const int u = sr >> lLp;
    const int ub = (u + d.t) & (g.c_eff - 1);
    const int col = d.col0 + (u & (g.c_out - 1));
    int row = d.row0 + ub;
    if (dg.tab) {
      const int r = sr & (g.Lp - 1);
      const int h = d.in.h0 + (ub & ((1 << d.in.logH) - 1));
      const int jj = (r + d.in.o * d.in.cg + (ub >> d.in.logH)) & (dg.dvp - 1);
      if (r >= dg.L || jj >= dg.d_v) return 0.0;
      row = h * dg.d_v + jj;
    }
    return (row < g.d_in && col < g.d_out) ? W[(size_t)row * g.d_out + col] : 0.0;
  }
  __device__ Pair begin(int pp) const {
    return g.cplx ? Pair{diag(p0 + pp, 0), diag(p0 + pp, 1)} : Pair{diag(p0 + 2 * pp, 0), diag(p0 + 2 * pp + 1, 0)};
  }
  __device__ cdd operator()(const Pair& pr, int u) const {
    const int s = slot_inv[u];
    return cdd{dd{value(pr.x, s), 0.0}, dd{value(pr.y, s), 0.0}};
  }
};

// The size-M DFT (forward sign) in four steps, M = M1 M2 with M2 = 128, n = M2 n1 + n2,
// k = k1 + M1 k2:
//   Y[k1 + M1 k2] = sum_n2 e^(-2 pi i n2 k2 / M2) [ e^(-2 pi i n2 k1 / M) sum_n1 v[M2 n1 + n2] e^(-2 pi i n1 k1 / M1) ].
// The column pass does the inner M1-point DFTs and the twiddles (Z[k1][n2]), the row pass the
// outer M2-point DFTs, so the transform makes two passes over HBM.  Each small DFT is split once
// more into radix-8 DFTs held in registers (M1 = 8 R2 with R2 = 2, 4 or 8; M2 = 8 x 16), with one
// exchange through LDS in between.
constexpr int kEncM2 = 128;
constexpr int kEncCB = 16;     // columns (n2) per workgroup in the column pass
constexpr int kEncRB = 8;      // rows (k1) per workgroup in the row pass

// e^(-2 pi i e / M), 0 <= e < M, from the table of eta^k = e^(2 pi i k / M), k < M/2
__device__ __forceinline__ cdd enc_twiddle(const double* tw, int e, int M) {
  const int half = M / 2;
  cdd w = ld_cdd(tw + (size_t)(e >= half ? e - half : e) * 4);
  w.im = dd_neg(w.im);
  if (e >= half) {
    w.re = dd_neg(w.re);
    w.im = dd_neg(w.im);
  }
  return w;
}

// x (-i)
__device__ __forceinline__ cdd cdd_mul_mi(cdd a) { return cdd{a.im, dd_neg(a.re)}; }

// In-place DFT (forward sign) of R = 2, 4 or 8 values in natural order, decimation in frequency:
// stage spans R/2 .. 1, twiddles e^(-2 pi i j / span*2) (1, -i and w8 = e^(-i pi / 4)), then the
// bit-reversed results put back in natural order.
template <int R>
__device__ __forceinline__ void dft_small(cdd (&a)[R], cdd w8) {
#pragma unroll
  for (int span = R / 2; span >= 1; span /= 2) {
#pragma unroll
    for (int b = 0; b < R; b += 2 * span) {
#pragma unroll
      for (int j = 0; j < span; ++j) {
        const cdd x = a[b + j], y = a[b + j + span];
        a[b + j] = cdd_add(x, y);
        cdd d = cdd_sub(x, y);
        // twiddle e^(-2 pi i j / (2 span)) = w8^(j * 4 / span)
        const int e8 = j * (4 / span);  // in units of 1/8 turn: 0..3
        if (e8 & 1) d = cdd_mul(d, w8);
        if (e8 & 2) d = cdd_mul_mi(d);
        a[b + j + span] = d;
      }
    }
  }
  cdd t[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    int r = 0;
#pragma unroll
    for (int bit = 1; bit < R; bit <<= 1) r = (r << 1) | ((k & bit) ? 1 : 0);
    t[r] = a[k];
  }
#pragma unroll
  for (int k = 0; k < R; ++k) a[k] = t[k];
}

// Column pass: kEncCB columns n2 of complex vector p; writes Z[p][k1][n2] (rows of M2).
// M1 = 8 R2: n1 = na + R2 nb, k1 = kb + 8 ka,
//   X[kb + 8 ka] = sum_na e^(-2 pi i na ka / R2) e^(-2 pi i na kb / M1) DFT8_nb(x[na + R2 nb])[kb].
// Step 1 (work-item (c, na), na < R2): the DFT8 over nb and its twiddle, into LDS S[kb][na][c];
// step 2 (work-item (c, kb)): the DFT of size R2 over na, the four-step twiddle, the store.
template <class Src, int R2>
__global__ __launch_bounds__(kEncCB * 8) void k_enc_cols(Src src, double* zbuf, const double* tw, int M) {
  constexpr int M1 = 8 * R2;
  __shared__ cdd S[8 * R2 * kEncCB];
  const int n2_0 = blockIdx.x * kEncCB;
  const int p = blockIdx.y;
  const int t = threadIdx.x;
  const int c = t % kEncCB, q = t / kEncCB;  // q: na in step 1, kb in step 2
  const cdd w8 = enc_twiddle(tw, M / 8, M);
  const auto ctx = src.begin(p);
  if (q < R2) {
    cdd a[8];
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) a[nb] = src(ctx, kEncM2 * (q + R2 * nb) + n2_0 + c);
    dft_small<8>(a, w8);
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      const cdd v = kb == 0 || q == 0 ? a[kb] : cdd_mul(a[kb], enc_twiddle(tw, q * kb * (M / M1), M));
      S[(kb * R2 + q) * kEncCB + c] = v;
    }
  }
  __syncthreads();
  cdd b[R2];
#pragma unroll
  for (int na = 0; na < R2; ++na) b[na] = S[(q * R2 + na) * kEncCB + c];
  dft_small<R2>(b, w8);
  const int n2 = n2_0 + c;
#pragma unroll
  for (int ka = 0; ka < R2; ++ka) {
    const int k1 = q + 8 * ka;
    const cdd z = cdd_mul(b[ka], enc_twiddle(tw, n2 * k1, M));  // n2 k1 < M2 M1 = M
    st_cdd(zbuf + ((size_t)p * M + (size_t)k1 * kEncM2 + n2) * 4, z);
  }
}

// Row pass: kEncRB rows k1 of vector p; writes Y[p][k1 + M1 k2].  M2 = 128: n2 = na + 16 nb,
// k2 = kb + 8 ka (na, ka < 16; nb, kb < 8),
//   X[kb + 8 ka] = DFT16_na(s_kb)[ka],  s_kb[na] = e^(-2 pi i na kb / 128) DFT8_nb(x[na + 16 nb])[kb].
// Step 1 (work-item (na, r)): the DFT8 over nb and its twiddle, into LDS; step 2 (work-item
// (r, kb, h)): the first decimation-in-frequency stage of the DFT16 (h = 0: s[n] + s[n + 8] for the
// even ka; h = 1: (s[n] - s[n + 8]) e^(-2 pi i n / 16) for the odd ka), then a DFT8.
constexpr int kEncRowPad = kEncRB + 1;  // LDS row stride (in cdd) of S[kb][na][r]
__global__ __launch_bounds__(kEncRB * 16) void k_enc_rows(const double* zbuf, double* ybuf, const double* tw, int M, int M1) {
  __shared__ cdd S[8 * 16 * kEncRowPad];
  const int k1_0 = blockIdx.x * kEncRB;
  const int p = blockIdx.y;
  const int t = threadIdx.x;
  const cdd w8 = enc_twiddle(tw, M / 8, M);
  {
    const int na = t % 16, r = t / 16;
    const double* row = zbuf + ((size_t)p * M + (size_t)(k1_0 + r) * kEncM2) * 4;
    cdd a[8];
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) a[nb] = ld_cdd(row + (size_t)(na + 16 * nb) * 4);
    dft_small<8>(a, w8);
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      const cdd v = kb == 0 || na == 0 ? a[kb] : cdd_mul(a[kb], enc_twiddle(tw, na * kb * (M / kEncM2), M));
      S[(kb * 16 + na) * kEncRowPad + r] = v;
    }
  }
  __syncthreads();
  const int r = t % kEncRB, q = t / kEncRB;
  const int kb = q % 8, h = q / 8;
  cdd b[8];
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    const cdd s0 = S[(kb * 16 + n) * kEncRowPad + r], s8 = S[(kb * 16 + n + 8) * kEncRowPad + r];
    b[n] = h == 0 ? cdd_add(s0, s8) : (n == 0 ? cdd_sub(s0, s8) : cdd_mul(cdd_sub(s0, s8), enc_twiddle(tw, n * (M / 16), M)));
  }
  dft_small<8>(b, w8);
  const int k1 = k1_0 + r;
#pragma unroll
  for (int kp = 0; kp < 8; ++kp) {
    const int k2 = kb + 8 * (2 * kp + h);
    st_cdd(ybuf + ((size_t)p * M + k1 + (size_t)M1 * k2) * 4, b[kp]);
  }
}

__device__ __forceinline__ long long rhaz_dd(dd x, int* overflow) {
  const bool neg = x.hi < 0.0;
  if (neg) x = dd_neg(x);
  if (!(x.hi < 4.0e18)) { *overflow = 1; return 0; }
  const double f = floor(x.hi);
  const double frac = (x.hi - f) + x.lo;
  long long r = (long long)f + (long long)floor(frac + 0.5);
  return neg ? -r : r;
}

// finalize: w_k = zeta^-k * y_k * (Delta / M); p_k = RHAZ(Re w_k), p_{k+M} = RHAZ(Im w_k);
// residues into limbs 0..level of out[p][limb][N]
// r mod q for |r| < 2^62 without a 64-bit division: quotient from FP64 (off by at most one),
// exact remainder in integers, one correction
__device__ __forceinline__ uint64_t mod_i64(long long r, long long q, double qinv) {
  const long long t = (long long)rint((double)r * qinv);
  long long m = r - t * q;
  if (m < 0) m += q;
  if (m >= q) m -= q;
  return (uint64_t)m;
}

// rounding and residues of one transformed value y_k: w = zeta^-k y_k (Delta / M),
// p_k = RHAZ(Re w), p_{k+M} = RHAZ(Im w) into limbs 0..nl-1 of out_p[limb][N]
__device__ __forceinline__ void enc_round_store(cdd y, const double* twist, double scale_over_m, int M, int k, int nl, const ModTable& mt,
                                                const uint64_t* mods, uint64_t* out_p, int* overflow) {
  const cdd w = cdd_mul(y, ld_cdd(twist + (size_t)k * 4));
  int of = 0;
  const long long pr = rhaz_dd(dd_mul_d(w.re, scale_over_m), &of);
  const long long pi = rhaz_dd(dd_mul_d(w.im, scale_over_m), &of);
  if (of) atomicOr(overflow, 1);
  const int n = 2 * M;
  for (int i = 0; i < nl; ++i) {
    const long long q = (long long)mods[i];
    const double qinv = mt.m[i].qinv;
    out_p[(size_t)i * n + k] = mod_i64(pr, q, qinv);
    out_p[(size_t)i * n + k + M] = mod_i64(pi, q, qinv);
  }
}

// finalize: w_k = zeta^-k * y_k * (Delta / M); p_k = RHAZ(Re w_k), p_{k+M} = RHAZ(Im w_k);
// residues into limbs 0..level of out[p][limb][N]
__global__ void k_enc_final(const double* ybuf, const double* twist /* [M][4] zeta^-k */, double scale_over_m, int M, int nl,
                            ModTable mt, const uint64_t* mods, uint64_t* out, int* overflow) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (k >= M) return;
  const cdd y = ld_cdd(ybuf + ((size_t)p * M + k) * 4);
  enc_round_store(y, twist, scale_over_m, M, k, nl, mt, mods, out + (size_t)p * nl * 2 * M, overflow);
}

// paired finalize: buffer pp holds FFT(x_{2pp} + i x_{2pp+1}) of two real inputs; their
// transforms are X1_k = (Y_k + conj Y_{M-k}) / 2 and X2_k = (Y_k - conj Y_{M-k}) / (2i)
__global__ void k_enc_final_pair(const double* ybuf, const double* twist, double scale_over_m, int M, int nl, ModTable mt,
                                 const uint64_t* mods, uint64_t* out, int count, int* overflow) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int pp = blockIdx.y;
  if (k >= M) return;
  const cdd y = ld_cdd(ybuf + ((size_t)pp * M + k) * 4);
  const cdd yc = ld_cdd(ybuf + ((size_t)pp * M + (k == 0 ? 0 : M - k)) * 4);
  const dd half_re1 = dd_add(y.re, yc.re), half_im1 = dd_add(y.im, dd_neg(yc.im));  // Y + conj(Yc)
  const dd half_re2 = dd_add(y.im, yc.im), half_im2 = dd_add(yc.re, dd_neg(y.re));  // (Y - conj(Yc)) / i
  const cdd x1 = cdd{dd_mul_d(half_re1, 0.5), dd_mul_d(half_im1, 0.5)};
  const cdd x2 = cdd{dd_mul_d(half_re2, 0.5), dd_mul_d(half_im2, 0.5)};
  const size_t stride = (size_t)nl * 2 * M;
  enc_round_store(x1, twist, scale_over_m, M, k, nl, mt, mods, out + (size_t)(2 * pp) * stride, overflow);
  if (2 * pp + 1 < count) enc_round_store(x2, twist, scale_over_m, M, k, nl, mt, mods, out + (size_t)(2 * pp + 1) * stride, overflow);
}

// Encodes `count` plaintexts into coefficient-form residues out[count][nl][N] (the DFT of the
// slot values from src, then twist, scale, rounding and residues).  bufA, bufB: [count][M][4].
template <class Src>
int encode_with(blb_ctx* c, const Src& src, int count, double* bufA, double* bufB, double scale, int nl, uint64_t* out, int* d_overflow,
                bool paired) {
  const int M = c->n / 2, M1 = M / kEncM2;
  if (M1 != 16 && M1 != 32 && M1 != 64) return BLB_EINVAL;  // M1 = 8 R2, R2 = 2, 4, 8; M1 >= kEncRB
  const int n_vec = paired ? (count + 1) / 2 : count;  // complex vectors transformed
  const dim3 gc(kEncM2 / kEncCB, n_vec);
  if (M1 == 64) k_enc_cols<Src, 8><<<gc, kEncCB * 8, 0, c->stream>>>(src, bufB, c->d_enc_tw, M);
  else if (M1 == 32) k_enc_cols<Src, 4><<<gc, kEncCB * 8, 0, c->stream>>>(src, bufB, c->d_enc_tw, M);
  else k_enc_cols<Src, 2><<<gc, kEncCB * 8, 0, c->stream>>>(src, bufB, c->d_enc_tw, M);
  k_enc_rows<<<dim3(M1 / kEncRB, n_vec), kEncRB * 16, 0, c->stream>>>(bufB, bufA, c->d_enc_tw, M, M1);
  dim3 grid((M + 255) / 256, n_vec);
  if (paired)
    k_enc_final_pair<<<grid, 256, 0, c->stream>>>(bufA, c->d_enc_twist, scale / (double)M, M, nl, c->mt, c->d_mods, out, count, d_overflow);
  else
    k_enc_final<<<grid, 256, 0, c->stream>>>(bufA, c->d_enc_twist, scale / (double)M, M, nl, c->mt, c->d_mods, out, d_overflow);
  return BLB_OK;
}
int run_encode_dense(blb_ctx* c, const double* vals, int n_vals, int count, double* bufA, double* bufB, double scale, int nl, uint64_t* out,
                     int* d_overflow) {
  return encode_with(c, EncSrcDense{vals, n_vals, c->d_slot_inv}, count, bufA, bufB, scale, nl, out, d_overflow, false);
}
int run_encode_cp(blb_ctx* c, const double* W, CpGeom g, int p0, int count, double* bufA, double* bufB, double scale, int nl, uint64_t* out,
                  int* d_overflow, CpDiag dg) {
  int lLp = 0;
  while ((1 << lLp) < g.Lp) ++lLp;
  return encode_with(c, EncSrcCp{W, g, p0, count, c->n / 2, lLp, c->d_slot_inv, dg}, count, bufA, bufB, scale, nl, out, d_overflow,
                     !g.cplx);
}

// ---------------------------------------------------------------------------------------
// matmul_cc helpers
// ---------------------------------------------------------------------------------------
// out = x (.) mx + y (.) my over a whole degree-1 ciphertext ([2][nl][N]); masks are
// evaluation-form plaintexts [nl][N] shared by both polys; y may be null.
__global__ void k_mask_pair(const CcPair* __restrict__ pairs, int nl, int n, ModTable mt) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= 2 * nl * n) return;
  const CcPair pr = pairs[blockIdx.y];
  const int mw = w % (nl * n);
  const ModEntry me = mt.m[mw / n];
  double r = mulmod_s(u2d(gmem(pr.x)[w]), u2d(gmem(pr.mx)[mw]), me.q, me.qinv);
  if (pr.y) r += mulmod_s(u2d(gmem(pr.y)[w]), u2d(gmem(pr.my)[mw]), me.q, me.qinv);
  gmem(pr.out)[w] = d2u(canon_full(r, me.q, me.qinv));
}
void launch_mask_pair(blb_ctx* c, const CcPair* pairs_dev, int n_pairs, int nl) {
  if (n_pairs <= 0) return;
  dim3 grid((2 * nl * c->n + 255) / 256, n_pairs);
  k_mask_pair<<<grid, 256, 0, c->stream>>>(pairs_dev, nl, c->n, c->mt);
}

// T3[t] = sum_a A_a (x) R[t][a]: degree-2 output (d0, d1, d2) at nl2 limbs.  A_a is at a
// higher level (nlA limbs per poly) and is used through its first nl2 limbs.
__global__ void k_tensor_sum(const uint64_t* const* __restrict__ A_tab, const uint64_t* const* __restrict__ R_tab,
                             uint64_t* __restrict__ T3, int n_ct, int nlA, int nl2, int n, ModTable mt, int a_per_t) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int limb = blockIdx.y % nl2;
  const int t = blockIdx.y / nl2;
  if (k >= n) return;
  const ModEntry me = mt.m[limb];
  const double q = me.q, qi = me.qinv;
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  for (int a = 0; a < n_ct; ++a) {
    const auto A = gmem(A_tab[a_per_t ? (size_t)t * n_ct + a : (size_t)a]);
    const auto R = gmem(R_tab[(size_t)t * n_ct + a]);
    const double a0 = u2d(A[(size_t)limb * n + k]), a1 = u2d(A[(size_t)(nlA + limb) * n + k]);
    const double r0 = u2d(R[(size_t)limb * n + k]), r1 = u2d(R[(size_t)(nl2 + limb) * n + k]);
    d0 += mulmod_s(a0, r0, q, qi);
    d1 += mulmod_s(a0, r1, q, qi) + mulmod_s(a1, r0, q, qi);
    d2 += mulmod_s(a1, r1, q, qi);
    if ((a & 1) == 1) {
      d0 = reduce_s(d0, q, qi);
      d1 = reduce_s(d1, q, qi);
      d2 = reduce_s(d2, q, qi);
    }
  }
  uint64_t* o = T3 + (size_t)t * 3 * nl2 * n;
  o[(size_t)limb * n + k] = d2u(canon_full(d0, q, qi));
  o[(size_t)(nl2 + limb) * n + k] = d2u(canon_full(d1, q, qi));
  o[(size_t)(2 * nl2 + limb) * n + k] = d2u(canon_full(d2, q, qi));
}
void launch_tensor_sum(blb_ctx* c, const uint64_t* const* A_tab, const uint64_t* const* R_tab, uint64_t* T3, int n_t, int n_ct, int nlA,
                       int nl2, bool a_per_t) {
  dim3 grid((c->n + 255) / 256, n_t * nl2);
  k_tensor_sum<<<grid, 256, 0, c->stream>>>(A_tab, R_tab, T3, n_ct, nlA, nl2, c->n, c->mt, a_per_t ? 1 : 0);
}

// out[o] (+)= sum over its terms of ct (.) mask, whole degree-1 ciphertexts at nl limbs
__global__ void k_masked_acc(const CcTerm* __restrict__ terms, const int* __restrict__ off, uint64_t* const* __restrict__ outs, int nl,
                             int n, ModTable mt, int accumulate) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int o = blockIdx.y;
  if (w >= 2 * nl * n) return;
  const int mw = w % (nl * n);
  const ModEntry me = mt.m[mw / n];
  const auto out = gmem(outs[o]);
  double acc = accumulate ? u2d(out[w]) : 0.0;
  int cnt = 0;
  for (int i = off[o]; i < off[o + 1]; ++i) {
    acc += mulmod_s(u2d(gmem(terms[i].ct)[w]), u2d(gmem(terms[i].mask)[mw]), me.q, me.qinv);
    if ((++cnt & 3) == 0) acc = reduce_s(acc, me.q, me.qinv);
  }
  out[w] = d2u(canon_full(acc, me.q, me.qinv));
}
void launch_masked_acc(blb_ctx* c, const CcTerm* terms, const int* off, uint64_t* const* outs, int n_out, int nl, bool accumulate) {
  if (n_out <= 0) return;
  dim3 grid((2 * nl * c->n + 255) / 256, n_out);
  k_masked_acc<<<grid, 256, 0, c->stream>>>(terms, off, outs, nl, c->n, c->mt, accumulate ? 1 : 0);
}

// ---------------------------------------------------------------------------------------
// Batched matmul_cp MAC over many independent instances (uneven lengths, several plans).
// Work item = (plan group, IB consecutive instances of the group, TB outputs, 256*CPT
// coefficients, one limb).  A persistent grid walks the item list with a grid stride; each
// plaintext word loaded is applied to IB instances' rotated inputs, so instances sharing a
// plan read its diagonals once per IB instances.
// ---------------------------------------------------------------------------------------
// The tile's tail (outputs past n_bj, instances past the group's last) is computed on clamped,
// in-bounds operands and not stored, so the inner loop has no branches.  Operands go through
// the global address space (pointer tables through scalar loads) and the next term's words are
// loaded while the current term is multiplied.
template <int TB, int IB, int CPT, bool P50>
__global__ __launch_bounds__(256) void k_cp_mac_batch(const MacGroup* __restrict__ groups, const MacItem* __restrict__ items, int n_items,
                                                      int n, ModTable mt) {
  typedef __attribute__((address_space(1))) const uint64_t gu64c;
  typedef __attribute__((address_space(1))) const u64x2 gu64x2c;
  typedef __attribute__((address_space(1))) uint64_t gu64;
  typedef __attribute__((address_space(4))) const uint64_t ku64;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const MacItem item = items[it];
    const MacGroup gr = groups[item.group];
    const int k0 = (item.kb * 256 + threadIdx.x) * CPT;
    if (k0 >= n) continue;
    for (int limb = item.limb; limb < item.limb + item.n_limb; ++limb) {
    const int nl = gr.nl, n_ai = gr.n_ai, n_bj = gr.n_bj;
    const ModEntry me = mt.m[limb];
    const double q = me.q, qi = me.qinv;
    const int bj0 = item.tile * TB;
    const int ninst = min(IB, gr.n_inst - item.inst0);
    const size_t pb = pt_poly_bytes(n, P50);
    const size_t term = (size_t)nl * pb;  // bytes per (bj, ai) plaintext
    const uint8_t* pt[TB];
#pragma unroll
    for (int t = 0; t < TB; ++t) pt[t] = (const uint8_t*)gr.pt + (size_t)min(bj0 + t, n_bj - 1) * n_ai * term + (size_t)limb * pb;
    const ku64* rxtab[IB];  // row of rotated-input pointers of each instance
#pragma unroll
    for (int u = 0; u < IB; ++u) rxtab[u] = (const ku64*)(gr.rx + (size_t)(item.inst0 + min(u, ninst - 1)) * n_ai);
    Pt50Raw<CPT> rw[TB];
    uint64_t rq[TB][CPT];
    uint64_t rx0[IB][CPT], rx1[IB][CPT];  // raw words of the term in flight
    auto fetch = [&](int ai) {
#pragma unroll
      for (int t = 0; t < TB; ++t) {
        if constexpr (P50) {
          pt50_fetch<CPT>(pt[t] + (size_t)ai * term, n, k0, rw[t]);
        } else {
          const gu64c* a = (const gu64c*)(pt[t] + (size_t)ai * term) + k0;
          if constexpr (CPT >= 2) {
#pragma unroll
            for (int c = 0; c < CPT; c += 2) {
              const u64x2 w = __builtin_nontemporal_load((const gu64x2c*)(a + c));
              rq[t][c] = w.x;
              rq[t][c + 1] = w.y;
            }
          } else {
            rq[t][0] = __builtin_nontemporal_load(a);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < IB; ++u) {
        const gu64c* x = (const gu64c*)rxtab[u][ai];
        if constexpr (CPT >= 2) {
#pragma unroll
          for (int c = 0; c < CPT; c += 2) {
            const u64x2 w0 = *(const gu64x2c*)(x + (size_t)limb * n + k0 + c);
            const u64x2 w1 = *(const gu64x2c*)(x + (size_t)(nl + limb) * n + k0 + c);
            rx0[u][c] = w0.x;
            rx0[u][c + 1] = w0.y;
            rx1[u][c] = w1.x;
            rx1[u][c + 1] = w1.y;
          }
        } else {
          rx0[u][0] = x[(size_t)limb * n + k0];
          rx1[u][0] = x[(size_t)(nl + limb) * n + k0];
        }
      }
    };
    double a0[IB][TB][CPT], a1[IB][TB][CPT];
#pragma unroll
    for (int u = 0; u < IB; ++u)
#pragma unroll
      for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int c = 0; c < CPT; ++c) { a0[u][t][c] = 0.0; a1[u][t][c] = 0.0; }
    fetch(0);
    for (int ai = 0; ai < n_ai; ++ai) {
      double w[TB][CPT], x0[IB][CPT], x1[IB][CPT];
#pragma unroll
      for (int t = 0; t < TB; ++t) {
        if constexpr (P50) {
          pt50_cvt<CPT>(rw[t], k0, w[t]);
        } else {
#pragma unroll
          for (int c = 0; c < CPT; ++c) w[t][c] = u2d(rq[t][c]);
        }
      }
#pragma unroll
      for (int u = 0; u < IB; ++u)
#pragma unroll
        for (int c = 0; c < CPT; ++c) { x0[u][c] = u2d(rx0[u][c]); x1[u][c] = u2d(rx1[u][c]); }
      fetch(min(ai + 1, n_ai - 1));  // the last term re-reads itself
#pragma unroll
      for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int u = 0; u < IB; ++u)
#pragma unroll
          for (int c = 0; c < CPT; ++c) {
            a0[u][t][c] += mulmod_s(w[t][c], x0[u][c], q, qi);
            a1[u][t][c] += mulmod_s(w[t][c], x1[u][c], q, qi);
          }
      if ((ai & 7) == 7) {  // 8 products below 0.875q each on a reduced |acc| <= q/2: |acc| < 7.5q < 2^53
#pragma unroll
        for (int u = 0; u < IB; ++u)
#pragma unroll
          for (int t = 0; t < TB; ++t)
#pragma unroll
            for (int c = 0; c < CPT; ++c) { a0[u][t][c] = reduce_s(a0[u][t][c], q, qi); a1[u][t][c] = reduce_s(a1[u][t][c], q, qi); }
      }
    }
#pragma unroll
    for (int u = 0; u < IB; ++u) {
      if (u >= ninst) continue;
      gu64* out = (gu64*)gr.inner[item.inst0 + u];
#pragma unroll
      for (int t = 0; t < TB; ++t) {
        if (bj0 + t < n_bj) {
          gu64* o0 = out + (((size_t)(bj0 + t) * 2 + 0) * nl + limb) * n + k0;
          gu64* o1 = out + (((size_t)(bj0 + t) * 2 + 1) * nl + limb) * n + k0;
#pragma unroll
          for (int c = 0; c < CPT; ++c) {
            o0[c] = d2u(canon_full(a0[u][t][c], q, qi));
            o1[c] = d2u(canon_full(a1[u][t][c], q, qi));
          }
        }
      }
    }
    }  // limbs of the item
  }
}

int batch_mac_shape(int variant, int* tb, int* ib, int* cpt) {
  switch (variant) {
    case 1: *tb = 4; *ib = 1; *cpt = 2; break;
    case 2: *tb = 2; *ib = 4; *cpt = 2; break;
    case 3: *tb = 4; *ib = 4; *cpt = 1; break;
    case 4: *tb = 8; *ib = 2; *cpt = 1; break;
    case 5: *tb = 8; *ib = 4; *cpt = 1; break;
    case 6: *tb = 4; *ib = 8; *cpt = 1; break;
    case 7: *tb = 4; *ib = 4; *cpt = 2; break;
    case 8: *tb = 8; *ib = 2; *cpt = 2; break;
    default: *tb = 4; *ib = 2; *cpt = 2; break;
  }
  return 0;
}

void launch_cp_mac_batch(blb_ctx* c, const MacGroup* groups, const MacItem* items, int n_items, int variant, int grid, int p50) {
  if (n_items <= 0) return;
  int tb, ib, cpt;
  batch_mac_shape(variant, &tb, &ib, &cpt);
  const int blocks = std::min(n_items, grid);
#define MB(a, b, d)                                                                                   \
  do {                                                                                                \
    if (p50) k_cp_mac_batch<a, b, d, true><<<blocks, 256, 0, c->stream>>>(groups, items, n_items, c->n, c->mt);  \
    else k_cp_mac_batch<a, b, d, false><<<blocks, 256, 0, c->stream>>>(groups, items, n_items, c->n, c->mt); \
  } while (0)
  if (tb == 4 && ib == 1) MB(4, 1, 2);
  else if (tb == 2 && ib == 4) MB(2, 4, 2);
  else if (tb == 4 && ib == 4 && cpt == 1) MB(4, 4, 1);
  else if (tb == 8 && ib == 2 && cpt == 1) MB(8, 2, 1);
  else if (tb == 8 && ib == 4) MB(8, 4, 1);
  else if (tb == 4 && ib == 8) MB(4, 8, 1);
  else if (tb == 4 && ib == 4) MB(4, 4, 2);
  else if (tb == 8 && ib == 2) MB(8, 2, 2);
  else MB(4, 2, 2);
#undef MB
}

// out[o] = sum of its terms (offsets per output), whole ciphertexts of `words` u64 each
__global__ void k_sum_var(const uint64_t* const* __restrict__ srcs, const int* __restrict__ off, uint64_t* const* __restrict__ dsts,
                          int n, int nl, ModTable mt) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int o = blockIdx.y;
  if (w >= 2 * nl * n) return;
  const ModEntry me = mt.m[(w / n) % nl];
  double acc = 0.0;
  int cnt = 0;
  for (int t = off[o]; t < off[o + 1]; ++t) {
    acc += u2d(gmem(srcs[t])[w]);
    if ((++cnt & 3) == 0) acc = reduce_s(acc, me.q, me.qinv);
  }
  gmem(dsts[o])[w] = d2u(canon_full(acc, me.q, me.qinv));
}
void launch_sum_var(blb_ctx* c, const uint64_t* const* srcs, const int* off, uint64_t* const* dsts, int n_out, int nl) {
  if (n_out <= 0) return;
  dim3 grid((2 * nl * c->n + 255) / 256, n_out);
  k_sum_var<<<grid, 256, 0, c->stream>>>(srcs, off, dsts, c->n, nl, c->mt);
}

// out[t] = k * in[t] for whole degree-1 ciphertexts (exact integer scalar, every limb); in[t]
// may hold more limbs per poly (nl_in) than out keeps (nl): the extra limbs are dropped
__global__ void k_scale_cts(const uint64_t* const* __restrict__ in, uint64_t* __restrict__ out, int n, int nl, int nl_in, double k,
                            ModTable mt) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (w >= 2 * nl * n) return;
  const int limb = (w / n) % nl, poly = w / (nl * n);
  const ModEntry me = mt.m[limb];
  const size_t src = ((size_t)poly * nl_in + limb) * n + (w % n);
  out[(size_t)t * 2 * nl * n + w] = d2u(canon(mulmod_s(u2d(gmem(in[t])[src]), k, me.q, me.qinv), me.q));
}
void launch_scale_cts(blb_ctx* c, const uint64_t* const* in, uint64_t* out, int count, int nl, double k, int nl_in) {
  if (count <= 0) return;
  dim3 grid((2 * nl * c->n + 255) / 256, count);
  k_scale_cts<<<grid, 256, 0, c->stream>>>(in, out, c->n, nl, nl_in > nl ? nl_in : nl, k, c->mt);
}
