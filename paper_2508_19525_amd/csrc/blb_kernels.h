// Kernel-side shared structures and launcher declarations.
#pragma once
#include "blb_internal.h"

// Per-poly descriptor for batched transforms.  Fields beyond src/dst/mod are used by the
// fused prologue / epilogue variants (rescale, ModDown).
struct PolyDesc {
  const uint64_t* src;
  uint64_t* dst;
  const uint64_t* src2;
  const uint64_t* src3;
  double aux;   // prologue constant (e.g. the modulus whose residues are lifted)
  double aux2;  // epilogue constant (e.g. q_l^-1 or P^-1 mod this modulus)
  int32_t mod;  // modulus index of this poly
  uint32_t gal; // Galois element applied to src3 (0 = none)
  int32_t log_n;
  int32_t pad;
};

// Bit-reversal of j over log_n bits
__device__ __forceinline__ uint32_t brv_bits(uint32_t j, int log_n) { return __brev(j) >> (32 - log_n); }

// Evaluation-form automorphism: value j of sigma_g(x) is value perm(j) of x, where slot j
// holds the evaluation at psi^(2 brv(j) + 1).
__device__ __forceinline__ uint32_t gal_perm(uint32_t j, uint32_t g, int log_n) {
  const uint32_t two_n_mask = (2u << log_n) - 1u;
  const uint32_t r = 2u * brv_bits(j, log_n) + 1u;
  const uint32_t rg = (r * g) & two_n_mask;  // g < 2N, r < 2N: product < 2^30 for N <= 2^14
  return brv_bits((rg - 1u) >> 1, log_n);
}

void launch_ntt(blb_ctx* c, const PolyDesc* d_descs, int count, bool fwd);
void launch_ntt_rescale(blb_ctx* c, const PolyDesc* d_descs, int count);
void launch_ntt_moddown(blb_ctx* c, const PolyDesc* d_descs, int count);
void launch_ntt_addto(blb_ctx* c, const PolyDesc* d_descs, int count);
// in-place transform of `count` limb-polys stored back to back at base ([item][nl][N]), no
// descriptor table
void launch_ntt_regular(blb_ctx* c, uint64_t* base, int count, int nl, bool fwd);
