/*
 * blb_oracle.c -- plain, slow CPU reference ("the oracle") for the server-side RNS-CKKS
 * path of "Breaking the Layer Barrier" (BLB, arXiv 2508.19525).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load this library.  It shares no code, header, table or constant
 * generator with the HIP library: every constant here (primes, roots, CRT factors, the
 * Gaussian CDT, Philox) is computed or written out independently in this file.
 *
 * Representation: every polynomial is kept in COEFFICIENT form as residues in [0, q_i),
 * limb-major: ct[poly][limb][N].  Ring products are exact negacyclic convolutions computed
 * with a textbook NTT (twist by psi^k, cyclic radix-2 DFT, pointwise, inverse); all modular
 * arithmetic uses unsigned __int128 and '%'.
 *
 * What it follows (sections of the paper):
 *   - CKKS primitives (Preliminaries, "Cryptographic Primitives"): ciphertext = pair of ring
 *     elements, rescale, homomorphic add/mult, left/right rotation.
 *   - Encoding (eq. ckks_encode, "CKKS Approximate HE and Message Encoding"): real slots only.
 *   - matmul_cp with BSGS (Section "Efficient Protocol for Fused MatMuls" and Appendix
 *     "BSGS Optimization"), spatial-first packing ("Consistent Packing for Single Operator").
 *   - matmul_cc steps 1-3 with multi-head packing ("Building Blocks", Multi-Head Optimization).
 *   - the column reordering of W_Q / W_K that makes matmul_cp emit the multi-head packing.
 *   - Softmax x V_h with zero padding and the dense diagonal packing, and the matmul_cp variant
 *     with diagonal-packed input for Concat(Att_h) W_O ("Efficient Fused Computations in
 *     Multi-Head Attention"; Appendix "Diagonal Ciphertext-Plaintext MatMul").
 *   - rotate-and-sum summation / broadcast ("Consistent Packing for Single Operator").
 *   - CKKS-to-MPC mask-and-share, step 1 of Algorithm ckks2mpc and F_C2M; the server's
 *     homomorphic addition of its share in Algorithm mpc2ckks.
 * Where the paper is silent (primes, randomness, key switching variant, schedules) the
 * readings are documented with the function that implements them.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <quadmath.h>

typedef unsigned __int128 u128;
typedef __float128 f128;

#define MAXL 16 /* max primes (q's + p's) */

/* ------------------------------------------------------------------------------------ */
/* integer helpers                                                                       */
/* ------------------------------------------------------------------------------------ */
static inline uint64_t mulm(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)(((u128)a * b) % q); }
static inline uint64_t addm(uint64_t a, uint64_t b, uint64_t q) { uint64_t s = a + b; return s >= q ? s - q : s; }
static inline uint64_t subm(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }
static uint64_t powm(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q; a %= q;
  while (e) { if (e & 1) r = mulm(r, a, q); a = mulm(a, a, q); e >>= 1; }
  return r;
}
static inline uint64_t invm(uint64_t a, uint64_t q) { return powm(a, q - 2, q); } /* q prime */
/* reduce a signed integer into [0,q) */
static inline uint64_t smod(int64_t v, uint64_t q) {
  int64_t r = v % (int64_t)q; if (r < 0) r += (int64_t)q; return (uint64_t)r;
}

/* deterministic Miller-Rabin for 64-bit n (bases 2..37 suffice below 3.3e24) */
static int is_prime_u64(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) { if (n == bases[i]) return 1; if (n % bases[i] == 0) return 0; }
  uint64_t d = n - 1; int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = powm(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int comp = 1;
    for (int r = 1; r < s; ++r) { x = mulm(x, x, n); if (x == n - 1) { comp = 0; break; } }
    if (comp) return 0;
  }
  return 1;
}

/* Prime rule (the paper fixes only that parameters are RNS chains of NTT-friendly primes):
 * scan q = k*2N + 1 downward from the largest such value below 2^50; the first n_q primes
 * found are q_0, q_1, ... and the next n_special are p_0, p_1, ... */
int orc_primes(int log_n, int count, uint64_t* out) {
  uint64_t two_n = 2ull << log_n;
  uint64_t k = ((1ull << 50) - 2) / two_n;
  int found = 0;
  for (; k > 0 && found < count; --k) {
    uint64_t q = k * two_n + 1;
    if (is_prime_u64(q)) out[found++] = q;
  }
  return found == count ? 0 : -1;
}

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",  */
/* SC'11): 10 rounds of the 4x32 Philox S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and   */
/* Weyl key increments 0x9E3779B9 / 0xBB67AE85.                                            */
/* ------------------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Randomness reading (the paper is silent): counter = (coefficient k, limb, object id,
 * domain tag), key = the 64-bit seed split into (low, high) 32-bit words.  Integer-valued
 * samples (secret, errors) use limb = 0xFFFFFFFF and are reduced into every limb. */
enum { TAG_SK = 1, TAG_ENC_A = 2, TAG_ENC_E = 3, TAG_KEY_A = 4, TAG_KEY_E = 5, TAG_MASK = 6 };
#define LIMB_INT 0xFFFFFFFFu

static void philox_at(uint64_t seed, uint32_t k, uint32_t limb, uint32_t obj, uint32_t tag, uint32_t out[4]) {
  uint32_t ctr[4] = {k, limb, obj, tag};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* uniform mod q: the 128-bit Philox block (word 0 least significant) reduced mod q */
static uint64_t sample_uniform(uint64_t seed, uint32_t k, uint32_t limb, uint32_t obj, uint32_t tag, uint64_t q) {
  uint32_t w[4]; philox_at(seed, k, limb, obj, tag, w);
  u128 x = ((u128)w[3] << 96) | ((u128)w[2] << 64) | ((u128)w[1] << 32) | (u128)w[0];
  return (uint64_t)(x % q);
}
/* ternary secret coefficient: (word0 mod 3) - 1 */
static int sample_ternary(uint64_t seed, uint32_t k) {
  uint32_t w[4]; philox_at(seed, k, LIMB_INT, 0, TAG_SK, w);
  return (int)(w[0] % 3u) - 1;
}

/* Gaussian error: discrete Gaussian rho(x) = exp(-x^2/(2 sigma^2)), sigma = 3.2, support
 * |x| <= 19 = floor(6 sigma), sampled by a cumulative distribution table on |x| with 63-bit
 * thresholds T_k = floor(2^63 * P(|x| <= k)) and a separate sign bit.  The table is computed
 * here in quad precision. */
#define CDT_MAX 19
static uint64_t g_cdt[CDT_MAX + 1];
static int g_cdt_ready = 0;
static void cdt_init(void) {
  if (g_cdt_ready) return;
  const f128 sigma = 3.2Q;
  f128 rho[CDT_MAX + 1], z = 0;
  for (int x = 0; x <= CDT_MAX; ++x) {
    rho[x] = expq(-(f128)(x * x) / (2 * sigma * sigma));
    z += (x == 0 ? 1 : 2) * rho[x];
  }
  f128 cum = 0;
  for (int x = 0; x <= CDT_MAX; ++x) {
    cum += (x == 0 ? 1 : 2) * rho[x] / z;
    f128 t = floorq(cum * 9223372036854775808.0Q); /* 2^63 */
    if (t >= 9223372036854775808.0Q) t = 9223372036854775807.0Q;
    g_cdt[x] = (uint64_t)t;
  }
  g_cdt[CDT_MAX] = 0x7FFFFFFFFFFFFFFFull; /* the last bucket takes the remainder */
  g_cdt_ready = 1;
}
void orc_cdt_table(uint64_t out[CDT_MAX + 1]) { cdt_init(); memcpy(out, g_cdt, sizeof(g_cdt)); }

static int sample_gauss(uint64_t seed, uint32_t k, uint32_t obj, uint32_t tag) {
  cdt_init();
  uint32_t w[4]; philox_at(seed, k, LIMB_INT, obj, tag, w);
  uint64_t r = (((uint64_t)w[1] << 32) | w[0]) >> 1; /* 63 uniform bits */
  int x = 0;
  while (x < CDT_MAX && r >= g_cdt[x]) ++x;
  return (w[2] & 1u) ? -x : x;
}

/* exported samplers (used by the statistical pins) */
void orc_sample_uniform_poly(uint64_t seed, uint32_t limb, uint32_t obj, uint32_t tag, uint64_t q, int n, uint64_t* out) {
  for (int k = 0; k < n; ++k) out[k] = sample_uniform(seed, (uint32_t)k, limb, obj, tag, q);
}
void orc_sample_ternary_poly(uint64_t seed, int n, int32_t* out) {
  for (int k = 0; k < n; ++k) out[k] = sample_ternary(seed, (uint32_t)k);
}
void orc_sample_gauss_poly(uint64_t seed, uint32_t obj, uint32_t tag, int n, int32_t* out) {
  for (int k = 0; k < n; ++k) out[k] = sample_gauss(seed, (uint32_t)k, obj, tag);
}

/* ------------------------------------------------------------------------------------ */
/* context: primes, textbook NTT tables, CRT constants                                   */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  int log_n, n, n_q, n_sp, dnum, alpha;
  uint64_t mod[MAXL];      /* q_0..q_{n_q-1}, p_0..p_{n_sp-1} */
  uint64_t* psi_pow[MAXL]; /* psi^k, k < N */
  uint64_t* ipsi_pow[MAXL];/* psi^-k */
  uint64_t* omega[MAXL];   /* omega^k = psi^(2k), k < N */
  uint64_t* iomega[MAXL];
  uint64_t n_inv[MAXL];
  f128* cw_re; f128* cw_im; /* zeta^j = exp(i pi j / N), j < 2N, quad precision */
} orc_ctx;

static uint64_t find_psi(uint64_t q, int log_n) {
  uint64_t two_n = 2ull << log_n;
  for (uint64_t g = 2;; ++g) {
    uint64_t psi = powm(g, (q - 1) / two_n, q);
    if (powm(psi, two_n >> 1, q) == q - 1) return psi; /* order exactly 2N */
  }
}

orc_ctx* orc_ctx_create(int log_n, int n_q, int n_special, int dnum) {
  if (log_n < 2 || log_n > 16 || n_q < 1 || n_special < 0 || n_q + n_special > MAXL || dnum < 1) return NULL;
  orc_ctx* c = (orc_ctx*)calloc(1, sizeof(orc_ctx));
  c->log_n = log_n; c->n = 1 << log_n; c->n_q = n_q; c->n_sp = n_special; c->dnum = dnum;
  c->alpha = (n_q + dnum - 1) / dnum;
  if (orc_primes(log_n, n_q + n_special, c->mod) != 0) { free(c); return NULL; }
  int n = c->n;
  for (int m = 0; m < n_q + n_special; ++m) {
    uint64_t q = c->mod[m], psi = find_psi(q, log_n), ipsi = invm(psi, q);
    c->psi_pow[m] = (uint64_t*)malloc(8 * n); c->ipsi_pow[m] = (uint64_t*)malloc(8 * n);
    c->omega[m] = (uint64_t*)malloc(8 * n); c->iomega[m] = (uint64_t*)malloc(8 * n);
    uint64_t a = 1, b = 1;
    for (int k = 0; k < n; ++k) { c->psi_pow[m][k] = a; c->ipsi_pow[m][k] = b; a = mulm(a, psi, q); b = mulm(b, ipsi, q); }
    uint64_t w = mulm(psi, psi, q), iw = invm(w, q);
    a = 1; b = 1;
    for (int k = 0; k < n; ++k) { c->omega[m][k] = a; c->iomega[m][k] = b; a = mulm(a, w, q); b = mulm(b, iw, q); }
    c->n_inv[m] = invm((uint64_t)n % q, q);
  }
  c->cw_re = (f128*)malloc(sizeof(f128) * 2 * n); c->cw_im = (f128*)malloc(sizeof(f128) * 2 * n);
  for (int j = 0; j < 2 * n; ++j) {
    f128 ang = M_PIq * (f128)j / (f128)n;
    c->cw_re[j] = cosq(ang); c->cw_im[j] = sinq(ang);
  }
  return c;
}
void orc_ctx_destroy(orc_ctx* c) {
  if (!c) return;
  for (int m = 0; m < c->n_q + c->n_sp; ++m) { free(c->psi_pow[m]); free(c->ipsi_pow[m]); free(c->omega[m]); free(c->iomega[m]); }
  free(c->cw_re); free(c->cw_im); free(c);
}
void orc_ctx_moduli(const orc_ctx* c, uint64_t* out) { memcpy(out, c->mod, 8 * (c->n_q + c->n_sp)); }

/* ---- textbook negacyclic NTT: A[t] = sum_k a_k psi^((2t+1)k) mod q, natural order t ---- */
static void bitrev_perm(uint64_t* a, int n) {
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
  }
}
/* cyclic DFT with root table w[k] = root^k (iterative radix-2 Cooley-Tukey) */
static void cyclic_dft(uint64_t* a, int n, const uint64_t* w, uint64_t q) {
  bitrev_perm(a, n);
  for (int len = 2; len <= n; len <<= 1) {
    int step = n / len;
    for (int s = 0; s < n; s += len)
      for (int j = 0; j < len / 2; ++j) {
        uint64_t u = a[s + j], v = mulm(a[s + j + len / 2], w[j * step], q);
        a[s + j] = addm(u, v, q); a[s + j + len / 2] = subm(u, v, q);
      }
  }
}
static void ntt_fwd(const orc_ctx* c, int m, uint64_t* a) {
  uint64_t q = c->mod[m];
  for (int k = 0; k < c->n; ++k) a[k] = mulm(a[k], c->psi_pow[m][k], q);
  cyclic_dft(a, c->n, c->omega[m], q);
}
static void ntt_inv(const orc_ctx* c, int m, uint64_t* a) {
  uint64_t q = c->mod[m];
  cyclic_dft(a, c->n, c->iomega[m], q);
  for (int k = 0; k < c->n; ++k) a[k] = mulm(mulm(a[k], c->n_inv[m], q), c->ipsi_pow[m][k], q);
}
/* exported for the pins */
void orc_ntt_forward(const orc_ctx* c, int m, uint64_t* a) { ntt_fwd(c, m, a); }
void orc_ntt_inverse(const orc_ctx* c, int m, uint64_t* a) { ntt_inv(c, m, a); }

/* negacyclic product r = a*b mod (X^N+1, modulus index m); r may alias a or b */
static void polymul(const orc_ctx* c, int m, const uint64_t* a, const uint64_t* b, uint64_t* r) {
  int n = c->n; uint64_t q = c->mod[m];
  uint64_t* fa = (uint64_t*)malloc(8 * n); uint64_t* fb = (uint64_t*)malloc(8 * n);
  memcpy(fa, a, 8 * n); memcpy(fb, b, 8 * n);
  ntt_fwd(c, m, fa); ntt_fwd(c, m, fb);
  for (int k = 0; k < n; ++k) fa[k] = mulm(fa[k], fb[k], q);
  ntt_inv(c, m, fa);
  memcpy(r, fa, 8 * n);
  free(fa); free(fb);
}
void orc_polymul(const orc_ctx* c, int m, const uint64_t* a, const uint64_t* b, uint64_t* r) { polymul(c, m, a, b, r); }

/* Galois automorphism sigma_g: X^k -> X^(kg mod 2N), negated when kg mod 2N >= N */
static void automorph(const orc_ctx* c, int m, const uint64_t* a, uint64_t g, uint64_t* r) {
  int n = c->n; uint64_t q = c->mod[m]; uint64_t two_n = 2ull * n;
  for (int k = 0; k < n; ++k) {
    uint64_t e = ((uint64_t)k * g) % two_n;
    if (e < (uint64_t)n) r[e] = a[k]; else r[e - n] = a[k] ? q - a[k] : 0;
  }
}
void orc_automorphism(const orc_ctx* c, int m, const uint64_t* a, uint64_t g, uint64_t* r) { automorph(c, m, a, g, r); }

/* slot index -> exponent: slot j sits at zeta^(5^j mod 2N) */
static uint64_t galois_left(const orc_ctx* c, int64_t t) {
  int64_t s = c->n / 2;
  int64_t tt = ((t % s) + s) % s;
  return powm(5, (uint64_t)tt, 2ull * c->n);
}
uint64_t orc_galois_elt(const orc_ctx* c, int64_t left_steps) { return galois_left(c, left_steps); }

/* ------------------------------------------------------------------------------------ */
/* encode / decode (eq. ckks_encode, real slots)                                         */
/* ------------------------------------------------------------------------------------ */
/* complex quad FFT in place, unnormalised: y[t] = sum_k x[k] * zeta^(2*sgn*t*k) */
static void fft_quad(const orc_ctx* c, f128* re, f128* im, int sgn) {
  int n = c->n;
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) { f128 t = re[i]; re[i] = re[j]; re[j] = t; t = im[i]; im[i] = im[j]; im[j] = t; }
  }
  for (int len = 2; len <= n; len <<= 1) {
    int step = n / len; /* omega^(j*step) = zeta^(2*j*step) */
    for (int s = 0; s < n; s += len)
      for (int j = 0; j < len / 2; ++j) {
        int e = (2 * j * step) % (2 * n);
        f128 wr = c->cw_re[e], wi = sgn > 0 ? c->cw_im[e] : -c->cw_im[e];
        f128 xr = re[s + j + len / 2], xi = im[s + j + len / 2];
        f128 vr = xr * wr - xi * wi, vi = xr * wi + xi * wr;
        f128 ur = re[s + j], ui = im[s + j];
        re[s + j] = ur + vr; im[s + j] = ui + vi;
        re[s + j + len / 2] = ur - vr; im[s + j + len / 2] = ui - vi;
      }
  }
}

/* Encode: p_k = round_half_away( (2*Delta/N) * sum_j m_j cos(pi * e_j * k / N) ), e_j = 5^j mod 2N.
 * Computed as the inverse transform over all odd exponents r: slot values sit at r = e_j
 * and (real slots) at r = -e_j; p_k = (Delta/N) Re( zeta^(-k) sum_t z_t omega^(-t k) ) with
 * r = 2t + 1.  Slots beyond n_vals are zero.  Output: signed integer coefficients.
 * With mi (complex slots, the full space the encoding map covers): slot j holds
 * z_j = m_j + i mi_j at r = e_j and its conjugate at r = -e_j, so that
 * p_k = round_half_away( (2*Delta/N) * sum_j [m_j cos(pi e_j k / N) + mi_j sin(pi e_j k / N)] ). */
static int encode_slots(const orc_ctx* c, const double* m, const double* mi, int64_t n_vals, double delta, int64_t* out) {
  int n = c->n, s = n / 2;
  if (n_vals > s || n_vals < 0) return -1;
  f128* re = (f128*)calloc(n, sizeof(f128)); f128* im = (f128*)calloc(n, sizeof(f128));
  uint64_t e = 1, two_n = 2ull * n;
  for (int j = 0; j < s; ++j) {
    f128 v = j < n_vals ? (f128)m[j] : 0;
    re[(e - 1) / 2] = v;
    re[(two_n - e - 1) / 2] = v;
    if (mi) {
      f128 w = j < n_vals ? (f128)mi[j] : 0;
      im[(e - 1) / 2] = w;
      im[(two_n - e - 1) / 2] = -w;
    }
    e = (e * 5) % two_n;
  }
  fft_quad(c, re, im, -1);
  int rc = 0;
  for (int k = 0; k < n; ++k) {
    int ek = (2 * n - k) % (2 * n); /* zeta^(-k) */
    f128 v = (re[k] * c->cw_re[ek] - im[k] * c->cw_im[ek]) * (f128)delta / (f128)n;
    f128 r = v >= 0 ? floorq(v + 0.5Q) : -floorq(-v + 0.5Q);
    if (fabsq(r) > 9.0e18Q) { rc = -2; r = 0; }
    out[k] = (int64_t)r;
  }
  free(re); free(im);
  return rc;
}
int orc_encode(const orc_ctx* c, const double* m, int64_t n_vals, double delta, int64_t* out) {
  return encode_slots(c, m, NULL, n_vals, delta, out);
}
int orc_encode_cplx(const orc_ctx* c, const double* m_re, const double* m_im, int64_t n_vals, double delta, int64_t* out) {
  return encode_slots(c, m_re, m_im, n_vals, delta, out);
}

/* residues of a signed integer polynomial in limbs 0..n_limbs-1 */
static void to_rns(const orc_ctx* c, const int64_t* p, int n_limbs, uint64_t* out) {
  for (int i = 0; i < n_limbs; ++i)
    for (int k = 0; k < c->n; ++k) out[(size_t)i * c->n + k] = smod(p[k], c->mod[i]);
}
int orc_encode_rns(const orc_ctx* c, const double* m, int64_t n_vals, double delta, int level, uint64_t* out) {
  int64_t* p = (int64_t*)malloc(8 * c->n);
  int rc = orc_encode(c, m, n_vals, delta, p);
  if (rc == 0) to_rns(c, p, level + 1, out);
  free(p);
  return rc;
}
int orc_encode_rns_cplx(const orc_ctx* c, const double* m_re, const double* m_im, int64_t n_vals, double delta, int level,
                        uint64_t* out) {
  int64_t* p = (int64_t*)malloc(8 * c->n);
  int rc = orc_encode_cplx(c, m_re, m_im, n_vals, delta, p);
  if (rc == 0) to_rns(c, p, level + 1, out);
  free(p);
  return rc;
}

/* centred CRT lift of residues r[0..nl-1] (moduli c->mod[0..nl-1]) as a quad value, via
 * Garner's mixed-radix digits; the lift is the representative in (-Q/2, Q/2]. */
static f128 crt_centered(const orc_ctx* c, const uint64_t* r, int nl) {
  uint64_t v[MAXL], vn[MAXL];
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->mod[i];
    uint64_t t = r[i] % q, tn = (q - r[i] % q) % q;
    for (int j = 0; j < i; ++j) {
      uint64_t inv = invm(c->mod[j] % q, q);
      t = mulm(subm(t, v[j] % q, q), inv, q);
      tn = mulm(subm(tn, vn[j] % q, q), inv, q);
    }
    v[i] = t; vn[i] = tn;
  }
  f128 x = 0, xn = 0;
  for (int i = nl - 1; i >= 0; --i) { x = x * (f128)c->mod[i] + (f128)v[i]; xn = xn * (f128)c->mod[i] + (f128)vn[i]; }
  return x <= xn ? x : -xn;
}
void orc_crt_centered(const orc_ctx* c, const uint64_t* poly, int level, double* out) {
  int nl = level + 1;
  for (int k = 0; k < c->n; ++k) {
    uint64_t r[MAXL];
    for (int i = 0; i < nl; ++i) r[i] = poly[(size_t)i * c->n + k];
    out[k] = (double)crt_centered(c, r, nl);
  }
}

/* Decode: m_j = Delta^-1 * Re( p~(zeta^(e_j)) ), p~ = centred CRT lift (no rounding before
 * the embedding; see the reading of eq. ckks_encode in the design notes).  With out_im the
 * imaginary parts Delta^-1 * Im( p~(zeta^(e_j)) ) too (complex slots). */
static void decode_slots(const orc_ctx* c, const uint64_t* poly, int level, double delta, int64_t n_vals, double* out, double* out_im) {
  int n = c->n, nl = level + 1;
  f128* re = (f128*)calloc(n, sizeof(f128)); f128* im = (f128*)calloc(n, sizeof(f128));
  for (int k = 0; k < n; ++k) {
    uint64_t r[MAXL];
    for (int i = 0; i < nl; ++i) r[i] = poly[(size_t)i * n + k];
    f128 pk = crt_centered(c, r, nl);
    re[k] = pk * c->cw_re[k]; im[k] = pk * c->cw_im[k]; /* twist by zeta^k */
  }
  fft_quad(c, re, im, +1);
  uint64_t e = 1, two_n = 2ull * n;
  for (int64_t j = 0; j < n_vals && j < n / 2; ++j) {
    out[j] = (double)(re[(e - 1) / 2] / (f128)delta);
    if (out_im) out_im[j] = (double)(im[(e - 1) / 2] / (f128)delta);
    e = (e * 5) % two_n;
  }
  free(re); free(im);
}
void orc_decode(const orc_ctx* c, const uint64_t* poly, int level, double delta, int64_t n_vals, double* out) {
  decode_slots(c, poly, level, delta, n_vals, out, NULL);
}
void orc_decode_cplx(const orc_ctx* c, const uint64_t* poly, int level, double delta, int64_t n_vals, double* out_re,
                     double* out_im) {
  decode_slots(c, poly, level, delta, n_vals, out_re, out_im);
}

/* ------------------------------------------------------------------------------------ */
/* keys                                                                                  */
/* ------------------------------------------------------------------------------------ */
/* switching key for target s': for digit j, (b_j, a_j) over all n_q + n_sp moduli.
 * Hybrid key switching reading (the paper relies on a library for it): digits
 * D_j = {q_{j*alpha}, ..., q_{min((j+1)alpha, n_q)-1}}; b_j = -a_j s + e_j + [P]_{q_i} s' 1{i in D_j}
 * (mod q_i), b_j = -a_j s + e_j (mod p_k); a_j uniform mod each prime. */
typedef struct {
  uint64_t id;      /* 0 = relinearisation (s^2), otherwise the Galois element g */
  uint64_t* data;   /* [digit][2 (b,a)][modulus][N] */
} orc_swk;

typedef struct {
  const orc_ctx* c;
  uint64_t seed;
  int32_t* s;       /* ternary secret, N coefficients */
  uint64_t* s_rns;  /* secret residues for all moduli [modulus][N] */
  int n_keys;
  orc_swk* keys;
} orc_keys;

static size_t swk_words(const orc_ctx* c) { return (size_t)c->dnum * 2 * (c->n_q + c->n_sp) * c->n; }
static uint64_t* swk_ptr(const orc_ctx* c, const orc_swk* k, int j, int ba, int m) {
  return k->data + (((size_t)j * 2 + ba) * (c->n_q + c->n_sp) + m) * c->n;
}

static void make_swk(const orc_ctx* c, const orc_keys* K, const int32_t* s_target, uint64_t id, orc_swk* out) {
  int n = c->n, nm = c->n_q + c->n_sp;
  out->id = id;
  out->data = (uint64_t*)calloc(swk_words(c), 8);
  /* P mod q_i */
  for (int j = 0; j < c->dnum; ++j) {
    uint32_t obj = (uint32_t)(id * 64 + (uint64_t)j);
    int32_t* e = (int32_t*)malloc(4 * n);
    for (int k = 0; k < n; ++k) e[k] = sample_gauss(K->seed, (uint32_t)k, obj, TAG_KEY_E);
    #pragma omp parallel for schedule(dynamic)
    for (int m = 0; m < nm; ++m) {
      uint64_t q = c->mod[m];
      uint64_t* b = swk_ptr(c, out, j, 0, m);
      uint64_t* a = swk_ptr(c, out, j, 1, m);
      for (int k = 0; k < n; ++k) a[k] = sample_uniform(K->seed, (uint32_t)k, (uint32_t)m, obj, TAG_KEY_A, q);
      polymul(c, m, a, K->s_rns + (size_t)m * n, b); /* a*s */
      for (int k = 0; k < n; ++k) b[k] = subm(smod(e[k], q), b[k], q); /* -a s + e */
      if (m < c->n_q && m / c->alpha == j) {
        uint64_t pmod = 1;
        for (int t = 0; t < c->n_sp; ++t) pmod = mulm(pmod, c->mod[c->n_q + t] % q, q);
        for (int k = 0; k < n; ++k) b[k] = addm(b[k], mulm(pmod, smod(s_target[k], q), q), q);
      }
    }
    free(e);
  }
}

/* integer (not reduced) products: s^2 and sigma_g(s) as integer polynomials */
static void int_sq_secret(const orc_ctx* c, const int32_t* s, int32_t* out) {
  /* negacyclic square of a ternary polynomial: |coeff| <= N, computed exactly with the
   * first modulus (|value| < q/2) and centred. */
  int n = c->n; uint64_t q = c->mod[0];
  uint64_t* a = (uint64_t*)malloc(8 * n);
  for (int k = 0; k < n; ++k) a[k] = smod(s[k], q);
  polymul(c, 0, a, a, a);
  for (int k = 0; k < n; ++k) out[k] = a[k] > q / 2 ? -(int32_t)(q - a[k]) : (int32_t)a[k];
  free(a);
}
static void int_automorph(const orc_ctx* c, const int32_t* s, uint64_t g, int32_t* out) {
  int n = c->n; uint64_t two_n = 2ull * n;
  for (int k = 0; k < n; ++k) {
    uint64_t e = ((uint64_t)k * g) % two_n;
    if (e < (uint64_t)n) out[e] = s[k]; else out[e - n] = -s[k];
  }
}

/* Key generation: secret s (tag sk), relinearisation key (id 0), Galois keys for the given
 * Galois elements. */
orc_keys* orc_keygen(const orc_ctx* c, uint64_t seed, const uint64_t* galois, int n_galois) {
  int n = c->n, nm = c->n_q + c->n_sp;
  orc_keys* K = (orc_keys*)calloc(1, sizeof(orc_keys));
  K->c = c; K->seed = seed;
  K->s = (int32_t*)malloc(4 * n);
  for (int k = 0; k < n; ++k) K->s[k] = sample_ternary(seed, (uint32_t)k);
  K->s_rns = (uint64_t*)malloc(8 * (size_t)nm * n);
  for (int m = 0; m < nm; ++m)
    for (int k = 0; k < n; ++k) K->s_rns[(size_t)m * n + k] = smod(K->s[k], c->mod[m]);
  K->n_keys = 1 + n_galois;
  K->keys = (orc_swk*)calloc(K->n_keys, sizeof(orc_swk));
  int32_t* tgt = (int32_t*)malloc(4 * n);
  int_sq_secret(c, K->s, tgt);
  make_swk(c, K, tgt, 0, &K->keys[0]);
  for (int i = 0; i < n_galois; ++i) {
    int_automorph(c, K->s, galois[i], tgt);
    make_swk(c, K, tgt, galois[i], &K->keys[1 + i]);
  }
  free(tgt);
  return K;
}
void orc_keys_destroy(orc_keys* K) {
  if (!K) return;
  for (int i = 0; i < K->n_keys; ++i) free(K->keys[i].data);
  free(K->keys); free(K->s); free(K->s_rns); free(K);
}
void orc_keys_secret(const orc_keys* K, int32_t* out) { memcpy(out, K->s, 4 * K->c->n); }
/* copy out a switching key ([digit][2][modulus][N]); returns -1 if absent */
int orc_keys_swk(const orc_keys* K, uint64_t id, uint64_t* out) {
  for (int i = 0; i < K->n_keys; ++i)
    if (K->keys[i].id == id) { memcpy(out, K->keys[i].data, 8 * swk_words(K->c)); return 0; }
  return -1;
}
static const orc_swk* find_key(const orc_keys* K, uint64_t id) {
  for (int i = 0; i < K->n_keys; ++i) if (K->keys[i].id == id) return &K->keys[i];
  return NULL;
}

/* ------------------------------------------------------------------------------------ */
/* encrypt / decrypt (secret-key form; the paper does not say which)                     */
/* ------------------------------------------------------------------------------------ */
/* ct = (-a s + e + pt, a) mod Q_level; a uniform per limb (tag enc-a), e Gaussian (tag
 * enc-e), object id = ct_id.  pt: residues [limb][N]. ct: [2][limb][N]. */
void orc_encrypt(const orc_keys* K, const uint64_t* pt, int level, uint64_t seed, uint32_t ct_id, uint64_t* ct) {
  const orc_ctx* c = K->c; int n = c->n, nl = level + 1;
  int32_t* e = (int32_t*)malloc(4 * n);
  for (int k = 0; k < n; ++k) e[k] = sample_gauss(seed, (uint32_t)k, ct_id, TAG_ENC_E);
  #pragma omp parallel for
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->mod[i];
    uint64_t* c0 = ct + (size_t)i * n;
    uint64_t* c1 = ct + ((size_t)nl + i) * n;
    for (int k = 0; k < n; ++k) c1[k] = sample_uniform(seed, (uint32_t)k, (uint32_t)i, ct_id, TAG_ENC_A, q);
    polymul(c, i, c1, K->s_rns + (size_t)i * n, c0);
    for (int k = 0; k < n; ++k) c0[k] = addm(subm(smod(e[k], q), c0[k], q), pt[(size_t)i * n + k], q);
  }
  free(e);
}
/* m = c0 + c1 s (+ c2 s^2) ; degree = number of polys - 1 */
void orc_decrypt(const orc_keys* K, const uint64_t* ct, int level, int degree, uint64_t* pt) {
  const orc_ctx* c = K->c; int n = c->n, nl = level + 1;
  #pragma omp parallel for
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->mod[i];
    const uint64_t* s = K->s_rns + (size_t)i * n;
    uint64_t* acc = pt + (size_t)i * n;
    uint64_t* t = (uint64_t*)malloc(8 * n);
    uint64_t* sp = (uint64_t*)malloc(8 * n);
    memcpy(acc, ct + (size_t)i * n, 8 * n);
    memcpy(sp, s, 8 * n);
    for (int d = 1; d <= degree; ++d) {
      polymul(c, i, ct + ((size_t)d * nl + i) * n, sp, t);
      for (int k = 0; k < n; ++k) acc[k] = addm(acc[k], t[k], q);
      if (d < degree) polymul(c, i, sp, s, sp);
    }
    free(t); free(sp);
  }
}

/* ------------------------------------------------------------------------------------ */
/* key switching, rotation, relinearisation, rescale                                     */
/* ------------------------------------------------------------------------------------ */
/* KeySwitch of d (coefficient form, limbs 0..level) with key `k`; if g != 1 the Galois
 * automorphism sigma_g is applied to the extended digits after ModUp (hoisted order).
 * Output u0, u1 at `level` ([limb][N] each).
 *   ModUp (fast basis conversion, no centring), digit j over D = D_j cap {0..level}:
 *     x_m = sum_{i in D} [d_i * (Q_D/q_i)^-1]_{q_i} * [(Q_D/q_i)]_m  (mod m)
 *   inner product: u = sum_j x_j * (b_j, a_j) over {q_0..q_level} u {p_k}
 *   ModDown (no centring): u_i <- (u_i - sum_k [u_{p_k} (P/p_k)^-1]_{p_k} [P/p_k]_{q_i}) * [P^-1]_{q_i} */
static void key_switch(const orc_ctx* c, const orc_swk* key, const uint64_t* d, int level, uint64_t g,
                       uint64_t* u0, uint64_t* u1) {
  int n = c->n, nl = level + 1, nsp = c->n_sp;
  int n_ext = nl + nsp;
  int ext_mod[MAXL];
  for (int i = 0; i < nl; ++i) ext_mod[i] = i;
  for (int t = 0; t < nsp; ++t) ext_mod[nl + t] = c->n_q + t;
  uint64_t* acc0 = (uint64_t*)calloc((size_t)n_ext * n, 8);
  uint64_t* acc1 = (uint64_t*)calloc((size_t)n_ext * n, 8);
  int n_digits = (nl + c->alpha - 1) / c->alpha;
  for (int j = 0; j < n_digits; ++j) {
    int lo = j * c->alpha, hi = (j + 1) * c->alpha; if (hi > nl) hi = nl;
    /* per-digit CRT factors */
    uint64_t qhat_inv[MAXL];
    for (int i = lo; i < hi; ++i) {
      uint64_t q = c->mod[i], prod = 1;
      for (int i2 = lo; i2 < hi; ++i2) if (i2 != i) prod = mulm(prod, c->mod[i2] % q, q);
      qhat_inv[i] = invm(prod, q);
    }
    #pragma omp parallel for schedule(dynamic)
    for (int e = 0; e < n_ext; ++e) {
      int m = ext_mod[e]; uint64_t mm = c->mod[m];
      uint64_t* x = (uint64_t*)calloc(n, 8);
      uint64_t* t = (uint64_t*)malloc(8 * n);
      for (int i = lo; i < hi; ++i) {
        uint64_t q = c->mod[i];
        uint64_t qhat_m = 1; /* (Q_D / q_i) mod m */
        for (int i2 = lo; i2 < hi; ++i2) if (i2 != i) qhat_m = mulm(qhat_m, c->mod[i2] % mm, mm);
        const uint64_t* di = d + (size_t)i * n;
        for (int k = 0; k < n; ++k) {
          uint64_t y = mulm(di[k], qhat_inv[i], q);
          x[k] = addm(x[k], mulm(y % mm, qhat_m, mm), mm);
        }
      }
      if (g != 1) { automorph(c, m, x, g, t); memcpy(x, t, 8 * n); }
      polymul(c, m, x, swk_ptr(c, key, j, 0, m), t);
      for (int k = 0; k < n; ++k) acc0[(size_t)e * n + k] = addm(acc0[(size_t)e * n + k], t[k], mm);
      polymul(c, m, x, swk_ptr(c, key, j, 1, m), t);
      for (int k = 0; k < n; ++k) acc1[(size_t)e * n + k] = addm(acc1[(size_t)e * n + k], t[k], mm);
      free(x); free(t);
    }
  }
  /* ModDown */
  uint64_t phat_inv[MAXL];
  for (int t = 0; t < nsp; ++t) {
    uint64_t p = c->mod[c->n_q + t], prod = 1;
    for (int t2 = 0; t2 < nsp; ++t2) if (t2 != t) prod = mulm(prod, c->mod[c->n_q + t2] % p, p);
    phat_inv[t] = invm(prod, p);
  }
  for (int pass = 0; pass < 2; ++pass) {
    uint64_t* acc = pass == 0 ? acc0 : acc1;
    uint64_t* u = pass == 0 ? u0 : u1;
    #pragma omp parallel for
    for (int i = 0; i < nl; ++i) {
      uint64_t q = c->mod[i];
      uint64_t pinv = 1, phat_q[MAXL];
      for (int t = 0; t < nsp; ++t) pinv = mulm(pinv, c->mod[c->n_q + t] % q, q);
      pinv = invm(pinv, q);
      for (int t = 0; t < nsp; ++t) {
        phat_q[t] = 1;
        for (int t2 = 0; t2 < nsp; ++t2) if (t2 != t) phat_q[t] = mulm(phat_q[t], c->mod[c->n_q + t2] % q, q);
      }
      for (int k = 0; k < n; ++k) {
        uint64_t corr = 0;
        for (int t = 0; t < nsp; ++t) {
          uint64_t p = c->mod[c->n_q + t];
          uint64_t y = mulm(acc[((size_t)nl + t) * n + k], phat_inv[t], p);
          corr = addm(corr, mulm(y % q, phat_q[t], q), q);
        }
        u[(size_t)i * n + k] = mulm(subm(acc[(size_t)i * n + k], corr, q), pinv, q);
      }
    }
  }
  free(acc0); free(acc1);
}

/* Key switches performed since the last reset (rotations with g != 1, relinearisations): the
 * schedules' operation counts are checked against their closed forms through these. */
static long g_n_rot = 0, g_n_relin = 0;
void orc_ks_counts(int64_t out[2], int reset) {
  out[0] = g_n_rot; out[1] = g_n_relin;
  if (reset) g_n_rot = g_n_relin = 0;
}

/* rotate left by `steps` slots: (sigma_g(c0) + u0, u1), (u0,u1) = KS_hoisted(c1) */
int orc_rotate(const orc_keys* K, const uint64_t* ct, int level, int64_t steps, uint64_t* out) {
  const orc_ctx* c = K->c; int n = c->n, nl = level + 1;
  uint64_t g = galois_left(c, steps);
  if (g == 1) { memcpy(out, ct, 8 * (size_t)2 * nl * n); return 0; }
  const orc_swk* key = find_key(K, g);
  if (!key) return -1;
  ++g_n_rot;
  uint64_t* u0 = (uint64_t*)malloc(8 * (size_t)nl * n);
  uint64_t* u1 = (uint64_t*)malloc(8 * (size_t)nl * n);
  key_switch(c, key, ct + (size_t)nl * n, level, g, u0, u1);
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->mod[i];
    uint64_t* t = (uint64_t*)malloc(8 * n);
    automorph(c, i, ct + (size_t)i * n, g, t);
    for (int k = 0; k < n; ++k) out[(size_t)i * n + k] = addm(t[k], u0[(size_t)i * n + k], q);
    memcpy(out + ((size_t)nl + i) * n, u1 + (size_t)i * n, 8 * n);
    free(t);
  }
  free(u0); free(u1);
  return 0;
}

/* relinearise (d0, d1, d2) -> (d0 + u0, d1 + u1), (u0,u1) = KS(d2) with the s^2 key */
int orc_relinearize(const orc_keys* K, const uint64_t* ct3, int level, uint64_t* out) {
  const orc_ctx* c = K->c; int n = c->n, nl = level + 1;
  const orc_swk* key = find_key(K, 0);
  if (!key) return -1;
  ++g_n_relin;
  uint64_t* u0 = (uint64_t*)malloc(8 * (size_t)nl * n);
  uint64_t* u1 = (uint64_t*)malloc(8 * (size_t)nl * n);
  key_switch(c, key, ct3 + (size_t)2 * nl * n, level, 1, u0, u1);
  for (int i = 0; i < nl; ++i)
    for (int k = 0; k < n; ++k) {
      size_t o = (size_t)i * n + k;
      out[o] = addm(ct3[o], u0[o], c->mod[i]);
      out[(size_t)nl * n + o] = addm(ct3[(size_t)nl * n + o], u1[o], c->mod[i]);
    }
  free(u0); free(u1);
  return 0;
}

/* Rescale (Preliminaries, "Rescaling"): c'_i = (c_i - [t]_{q_i}) * q_l^-1 mod q_i where t is the
 * centred lift of the last limb; equals round(c / q_l) mod Q_{l-1}.  n_poly polys. */
void orc_rescale(const orc_ctx* c, const uint64_t* ct, int level, int n_poly, uint64_t* out) {
  int n = c->n, nl = level + 1;
  uint64_t ql = c->mod[level];
  for (int p = 0; p < n_poly; ++p)
    for (int i = 0; i < level; ++i) {
      uint64_t q = c->mod[i], inv = invm(ql % q, q);
      const uint64_t* last = ct + ((size_t)p * nl + level) * n;
      for (int k = 0; k < n; ++k) {
        uint64_t v = last[k];
        uint64_t tm = v <= ql / 2 ? v % q : subm(0, (ql - v) % q, q); /* centred lift mod q */
        out[((size_t)p * level + i) * n + k] = mulm(subm(ct[((size_t)p * nl + i) * n + k], tm, q), inv, q);
      }
    }
}

/* ------------------------------------------------------------------------------------ */
/* ciphertext-level helpers used by the schedules                                         */
/* ------------------------------------------------------------------------------------ */
/* acc += pt * ct  (pt: [limb][N], ct: [2][limb][N]) */
static void mac_pt(const orc_ctx* c, uint64_t* acc, const uint64_t* pt, const uint64_t* ct, int nl) {
  int n = c->n;
  #pragma omp parallel for
  for (int i = 0; i < 2 * nl; ++i) {
    int limb = i % nl;
    uint64_t q = c->mod[limb];
    uint64_t* t = (uint64_t*)malloc(8 * n);
    polymul(c, limb, pt + (size_t)limb * n, ct + (size_t)i * n, t);
    for (int k = 0; k < n; ++k) acc[(size_t)i * n + k] = addm(acc[(size_t)i * n + k], t[k], q);
    free(t);
  }
}
static void add_ct(const orc_ctx* c, uint64_t* acc, const uint64_t* x, int nl, int n_poly) {
  int n = c->n;
  for (int p = 0; p < n_poly; ++p)
    for (int i = 0; i < nl; ++i)
      for (int k = 0; k < n; ++k) {
        size_t o = ((size_t)p * nl + i) * n + k;
        acc[o] = addm(acc[o], x[o], c->mod[i]);
      }
}

static int ceil_log2(int64_t v) { int r = 0; while ((1ll << r) < v) ++r; return r; }

/* Noise boost applied before key-switched rotations inside the matmuls (reading: the paper
 * gives no noise management; 2^10 keeps key-switch noise ~2^-27 of a 2^40-scaled message). */
#define NOISE_BOOST 1024.0

/* out = k * ct (integer scalar, every limb of both polys) */
static void scale_ct(const orc_ctx* c, const uint64_t* ct, uint64_t k, int nl, uint64_t* out) {
  int n = c->n;
  for (int p = 0; p < 2; ++p)
    for (int i = 0; i < nl; ++i)
      for (int j = 0; j < n; ++j) {
        size_t o = ((size_t)p * nl + i) * n + j;
        out[o] = mulm(ct[o], k % c->mod[i], c->mod[i]);
      }
}

/* ------------------------------------------------------------------------------------ */
/* matmul_cp (pinned schedule)                                                           */
/* ------------------------------------------------------------------------------------ */
/* Geometry of the spatial-first packing ("Consistent Packing for Single Operator"): element
 * (i, j) of an L x D matrix sits in ciphertext j / c at slot i + L' * (j mod c), L' = 2^ceil(log2 L),
 * c = S / L'.  When D' * L' < S (D' = 2^ceil(log2 D)) the D' columns are replicated c / D' times. */
void orc_cp_geometry(const orc_ctx* c, int L, int d_in, int d_out, int32_t* out /* [8] */) {
  int s = c->n / 2;
  int lp = 1 << ceil_log2(L);
  int cc = s / lp;
  int din_p = 1 << ceil_log2(d_in), dout_p = 1 << ceil_log2(d_out);
  int c_eff = cc < din_p ? cc : din_p;
  int c_out = cc < dout_p ? cc : dout_p;
  int n_in = (d_in + cc - 1) / cc, n_out = (d_out + cc - 1) / cc;
  int b = 1 << ((ceil_log2(c_eff) + 1) / 2);
  int g = c_eff / b;
  out[0] = lp; out[1] = cc; out[2] = c_eff; out[3] = c_out; out[4] = n_in; out[5] = n_out; out[6] = b; out[7] = g;
}

/* spatial-first slot vector of ciphertext a (length S) for an L x D row-major matrix */
void orc_pack_spatial(const orc_ctx* c, const double* X, int L, int D, int a, double* out) {
  int32_t g[8]; orc_cp_geometry(c, L, D, D, g);
  int lp = g[0], cc = g[1];
  int dp = 1 << ceil_log2(D);
  int s = c->n / 2;
  for (int slot = 0; slot < s; ++slot) {
    int i = slot % lp, u = slot / lp;
    int col = (dp < cc) ? (u % dp) : a * cc + u;
    out[slot] = (i < L && col < D) ? X[(size_t)i * D + col] : 0.0;
  }
}

/* The schedule of matmul_cp ("Diagonal Ciphertext-Plaintext MatMul", BSGS over the c_eff
 * diagonals, t = jB + i):
 *   Y_b = rescale( sum_{j<G} Rot_l^{jBL'}( sum_a sum_{i<B} Encode_{q_l}(Rot_r^{jBL'}(d_{a,b,t})) * Rot_l^{iL'}(X_a) ) ).
 * diag(geo, a, b, t, vec) writes the slot vector of diagonal d_{a,b,t} (before its pre-rotation;
 * all zero for an output block b past the last).  With cplx (complex-slot output packing) output
 * ciphertext b carries block 2b in the real and block 2b + 1 in the imaginary part of each slot:
 * its plaintexts encode d_{a,2b,t} + i d_{a,2b+1,t}.  The inputs are real, the rotations move
 * whole complex slots and the products are slot-wise, so the result decodes to Y_{2b} + i Y_{2b+1}. */
typedef void (*cp_diag_fn)(const void* geo, int a, int b, int t, double* vec);

static int cp_schedule(const orc_keys* K, const uint64_t* X, int level, int lp, int n_in, int n_out_ct, int B, int G,
                       cp_diag_fn diag, const void* geo, int cplx, const uint8_t* out_mask, uint64_t* Y) {
  const orc_ctx* c = K->c;
  int n = c->n, s = n / 2, nl = level + 1;
  size_t ctw = (size_t)2 * nl * n;
  /* noise boost: the inputs are multiplied by the integer 2^10 before their rotations (the
   * key-switch noise is absolute, so it shrinks by 2^10 relative to the message) and the
   * diagonals are encoded at q_l / 2^10, which leaves the product's scale Delta_X * q_l */
  double delta_w = (double)c->mod[level] / NOISE_BOOST;
  uint64_t* xs = (uint64_t*)malloc(8 * ctw * (size_t)n_in);
  for (int a = 0; a < n_in; ++a) scale_ct(c, X + ctw * a, (uint64_t)NOISE_BOOST, nl, xs + ctw * a);
  /* baby steps: Rot_l^{iL'}(X_a) */
  uint64_t* rx = (uint64_t*)malloc(8 * ctw * (size_t)n_in * B);
  for (int a = 0; a < n_in; ++a)
    for (int i = 0; i < B; ++i)
      if (orc_rotate(K, xs + ctw * a, level, (int64_t)i * lp, rx + ctw * ((size_t)a * B + i)) != 0) { free(rx); free(xs); return -1; }
  free(xs);
  double* vec = (double*)malloc(8 * s);
  double* vrot = (double*)malloc(8 * s);
  double* vec_im = (double*)malloc(8 * s);
  double* vrot_im = (double*)malloc(8 * s);
  uint64_t* pt = (uint64_t*)malloc(8 * (size_t)nl * n);
  uint64_t* inner = (uint64_t*)malloc(8 * ctw);
  uint64_t* rot = (uint64_t*)malloc(8 * ctw);
  uint64_t* acc = (uint64_t*)malloc(8 * ctw);
  int rc = 0;
  for (int b = 0; b < n_out_ct && rc == 0; ++b) {
    if (out_mask && !out_mask[b]) continue;
    memset(acc, 0, 8 * ctw);
    for (int j = 0; j < G && rc == 0; ++j) {
      memset(inner, 0, 8 * ctw);
      for (int a = 0; a < n_in; ++a)
        for (int i = 0; i < B; ++i) {
          int t = j * B + i;
          int r = j * B * lp; /* Rot_r^r: out[slot] = in[slot - r] */
          diag(geo, a, cplx ? 2 * b : b, t, vec);
          for (int slot = 0; slot < s; ++slot) vrot[slot] = vec[((slot - r) % s + s) % s];
          if (cplx) {
            diag(geo, a, 2 * b + 1, t, vec_im);
            for (int slot = 0; slot < s; ++slot) vrot_im[slot] = vec_im[((slot - r) % s + s) % s];
            orc_encode_rns_cplx(c, vrot, vrot_im, s, delta_w, level, pt);
          } else {
            orc_encode_rns(c, vrot, s, delta_w, level, pt);
          }
          mac_pt(c, inner, pt, rx + ctw * ((size_t)a * B + i), nl);
        }
      if (j == 0) add_ct(c, acc, inner, nl, 2);
      else {
        if (orc_rotate(K, inner, level, (int64_t)j * B * lp, rot) != 0) { rc = -1; break; }
        add_ct(c, acc, rot, nl, 2);
      }
    }
    if (rc == 0) orc_rescale(c, acc, level, 2, Y + (size_t)b * 2 * level * n);
  }
  free(rx); free(vec); free(vrot); free(vec_im); free(vrot_im); free(pt); free(inner); free(rot); free(acc);
  return rc;
}

/* spatial-first input: d_{a,b,t}[u L' + i] = W{a c + ((u + t) mod c_eff), b c + (u mod c_out)}
 * (0 out of range), broadcast over the L' slots of block u */
typedef struct {
  int s, lp, cc, c_eff, c_out, d_in, d_out;
  const double* W;
} cp_sf_geo;
static void cp_sf_diag(const void* geo, int a, int b, int t, double* vec) {
  const cp_sf_geo* g = (const cp_sf_geo*)geo;
  for (int slot = 0; slot < g->s; ++slot) {
    int u = slot / g->lp;
    int row = a * g->cc + (u + t) % g->c_eff, col = b * g->cc + u % g->c_out;
    vec[slot] = (row < g->d_in && col < g->d_out) ? g->W[(size_t)row * g->d_out + col] : 0.0;
  }
}

/* Inputs X: n_in cts at `level` ([ct][2][limb][N]); W: d_in x d_out row-major.  Outputs Y:
 * n_out cts at level-1 ([ct][2][level][N]); with cplx, ceil(n_out / 2) of them, output b holding
 * blocks 2b (real part) and 2b + 1 (imaginary part).  out_mask selects which outputs to compute
 * (NULL = all; skipped outputs are left untouched).  Returns 0, or -1 on a missing key. */
int orc_matmul_cp_pack(const orc_keys* K, const uint64_t* X, int level, const double* W, int L, int d_in, int d_out, int cplx,
                       const uint8_t* out_mask, uint64_t* Y) {
  const orc_ctx* c = K->c;
  int32_t g[8]; orc_cp_geometry(c, L, d_in, d_out, g);
  cp_sf_geo geo = {c->n / 2, g[0], g[1], g[2], g[3], d_in, d_out, W};
  int n_out_ct = cplx ? (g[5] + 1) / 2 : g[5];
  return cp_schedule(K, X, level, g[0], g[4], n_out_ct, g[6], g[7], cp_sf_diag, &geo, cplx, out_mask, Y);
}
int orc_matmul_cp(const orc_keys* K, const uint64_t* X, int level, const double* W, int L, int d_in, int d_out,
                  const uint8_t* out_mask, uint64_t* Y) {
  return orc_matmul_cp_pack(K, X, level, W, L, d_in, d_out, 0, out_mask, Y);
}

/* Galois elements needed by matmul_cp at this geometry (baby and giant steps) */
int orc_cp_galois(const orc_ctx* c, int L, int d_in, int d_out, uint64_t* out) {
  int32_t g[8]; orc_cp_geometry(c, L, d_in, d_out, g);
  int lp = g[0], B = g[6], G = g[7], cnt = 0;
  for (int i = 1; i < B; ++i) out[cnt++] = galois_left(c, (int64_t)i * lp);
  for (int j = 1; j < G; ++j) out[cnt++] = galois_left(c, (int64_t)j * B * lp);
  return cnt;
}

/* ------------------------------------------------------------------------------------ */
/* matmul_cp with diagonal-packed input (Appendix "Diagonal Ciphertext-Plaintext MatMul")  */
/* ------------------------------------------------------------------------------------ */
/* E = Concat_h(Att_h) W for Att_h (L x d_v) in the dense diagonal packing that Softmax x V_h
 * produces (heads split into power-of-two groups, largest first, group outputs concatenated):
 * input ciphertext a, the o-th output of a group of H_g heads starting at head h0 with
 * c_g = S / (L' H_g), holds at slot i + L' u the value Att_h{i, (i + tau) mod d_v'} with
 * h = h0 + (u mod H_g) and tau = o c_g + floor(u / H_g).  Row r of E's column k is then
 * sum over (h, tau) of Att_h{i, (i + tau) mod d_v'} W{h d_v + (i + tau) mod d_v', k}: the input
 * blocks meet the weights of a "duplicated" spatial-first plaintext (figure diag (c)).  The
 * schedule is the one of orc_matmul_cp with c_eff = c = S / L' and the diagonals
 *   d_{a,b,t}[u L' + i] = W{h d_v + j, b c + (u mod c_out)},  (h, tau) = block (u + t) mod c of
 *   input a, j = (i + tau) mod d_v', and 0 when i >= L, j >= d_v or the column is >= d_out;
 * the output Y_b is spatial-first (column b c + u at slots u L' + i).  Geometry and Galois
 * elements are those of orc_cp_geometry / orc_cp_galois at d_in = n_heads d_v'. */
static void diag_block(const orc_ctx* c, int lp, int n_heads, int dvp, int a, int u, int* h, int* tau) {
  int s = c->n / 2, rem = n_heads, h0 = 0, idx = 0;
  while (rem > 0) {
    int hg = 1;
    while (hg * 2 <= rem) hg *= 2;
    int cg = s / (lp * hg), nd = dvp / cg;
    if (a < idx + nd) {
      int o = a - idx;
      *h = h0 + u % hg;
      *tau = o * cg + u / hg;
      return;
    }
    idx += nd; h0 += hg; rem -= hg;
  }
  *h = -1; *tau = 0;
}

/* diagonal-packed input: the diagonal of the block comment above, for input a */
typedef struct {
  const orc_ctx* c;
  int s, lp, cc, c_eff, c_out, L, n_heads, d_v, dvp, d_out;
  const double* W;
} cp_dg_geo;
static void cp_dg_diag(const void* geo, int a, int b, int t, double* vec) {
  const cp_dg_geo* g = (const cp_dg_geo*)geo;
  for (int slot = 0; slot < g->s; ++slot) {
    int u = slot / g->lp, row_i = slot % g->lp, h, tau;
    diag_block(g->c, g->lp, g->n_heads, g->dvp, a, (u + t) % g->c_eff, &h, &tau);
    int jj = (row_i + tau) % g->dvp, col = b * g->cc + u % g->c_out;
    vec[slot] = (row_i < g->L && jj < g->d_v && col < g->d_out) ? g->W[(size_t)(h * g->d_v + jj) * g->d_out + col] : 0.0;
  }
}

int orc_matmul_cp_diag_pack(const orc_keys* K, const uint64_t* X, int level, const double* W, int L, int n_heads, int d_v, int d_out,
                            int cplx, const uint8_t* out_mask, uint64_t* Y) {
  const orc_ctx* c = K->c;
  int s = c->n / 2;
  int dvp = 1 << ceil_log2(d_v);
  int32_t g[8]; orc_cp_geometry(c, L, n_heads * dvp, d_out, g);
  int lp = g[0], cc = g[1], c_eff = g[2];
  if (c_eff != cc || dvp > lp) return -3;
  for (int rem = n_heads; rem > 0;) {
    int hg = 1;
    while (hg * 2 <= rem) hg *= 2;
    if (s / (lp * hg) > dvp) return -3;
    rem -= hg;
  }
  cp_dg_geo geo = {c, s, lp, cc, c_eff, g[3], L, n_heads, d_v, dvp, d_out, W};
  int n_out_ct = cplx ? (g[5] + 1) / 2 : g[5];
  return cp_schedule(K, X, level, lp, g[4], n_out_ct, g[6], g[7], cp_dg_diag, &geo, cplx, out_mask, Y);
}
int orc_matmul_cp_diag(const orc_keys* K, const uint64_t* X, int level, const double* W, int L, int n_heads, int d_v, int d_out,
                       const uint8_t* out_mask, uint64_t* Y) {
  return orc_matmul_cp_diag_pack(K, X, level, W, L, n_heads, d_v, d_out, 0, out_mask, Y);
}

/* ------------------------------------------------------------------------------------ */
/* CKKS-to-MPC mask-and-share (Algorithm ckks2mpc step 1; F_C2M item 1)                   */
/* ------------------------------------------------------------------------------------ */
/* r ~ U(R_{Q_l}) in the coefficient domain, one independent uniform residue per limb
 * (uniform mod Q_l by CRT); masked = (c0 + r, c1); share_1 = -r mod q_i.  If
 * target_level < level the ciphertext is first reduced to target_level (top limbs dropped).
 * ct: [2][level+1][N] in; masked: [2][target+1][N]; share: [target+1][N]. */
void orc_mask_to_share(const orc_ctx* c, const uint64_t* ct, int level, int target_level, uint64_t seed, uint32_t ct_id,
                       uint64_t* masked, uint64_t* share) {
  int n = c->n, nl = level + 1, tl = target_level + 1;
  for (int i = 0; i < tl; ++i) {
    uint64_t q = c->mod[i];
    for (int k = 0; k < n; ++k) {
      uint64_t r = sample_uniform(seed, (uint32_t)k, (uint32_t)i, ct_id, TAG_MASK, q);
      masked[(size_t)i * n + k] = addm(ct[(size_t)i * n + k], r, q);
      masked[((size_t)tl + i) * n + k] = ct[((size_t)nl + i) * n + k];
      share[(size_t)i * n + k] = (q - r) % q;
    }
  }
}

/* ------------------------------------------------------------------------------------ */
/* Rotate-and-sum summation and broadcast (Section "Consistent Packing for Single Operator": */
/* Expansion and Reduction operators)                                                      */
/* ------------------------------------------------------------------------------------ */
/* m^0 = m, m^i = m^{i-1} + Rot^{2^{i-1} block}(m^{i-1}) for i = 1 .. log2 n_blocks, with left
 * rotations (direction 0: summation) or right rotations (direction 1: broadcast).  Summation then
 * keeps the first `block` slots: mask [1 x block, 0, ...] encoded at scale q_level, product
 * rescaled (output at level-1, the input scale kept); without the mask (mask = 0), or for a
 * broadcast, the output is m^{log2 n_blocks} at the input level.  ct, out: [2][nl][N].
 * Returns 0, -1 on a missing key, -3 on bad arguments. */
static void mac_vec(const orc_ctx* c, uint64_t* acc, const double* vec, double delta, const uint64_t* ct, int level);

int orc_rotate_sum(const orc_keys* K, const uint64_t* ct, int level, int block, int n_blocks, int direction, int mask, uint64_t* out) {
  const orc_ctx* c = K->c;
  int n = c->n, s = n / 2, nl = level + 1;
  if (block < 1 || n_blocks < 1 || (n_blocks & (n_blocks - 1)) || (int64_t)block * n_blocks > s) return -3;
  if (mask && (direction != 0 || level < 1)) return -3;
  size_t w = (size_t)2 * nl * n;
  uint64_t* cur = (uint64_t*)malloc(8 * w);
  uint64_t* rot = (uint64_t*)malloc(8 * w);
  memcpy(cur, ct, 8 * w);
  int rc = 0;
  for (int64_t step = block; step < (int64_t)block * n_blocks; step *= 2) {
    if (orc_rotate(K, cur, level, direction == 0 ? step : -step, rot) != 0) { rc = -1; break; }
    add_ct(c, cur, rot, nl, 2);
  }
  if (rc == 0) {
    if (mask) {
      double* v = (double*)malloc(8 * s);
      for (int j = 0; j < s; ++j) v[j] = j < block ? 1.0 : 0.0;
      uint64_t* acc = (uint64_t*)calloc(w, 8);
      mac_vec(c, acc, v, (double)c->mod[level], cur, level);
      orc_rescale(c, acc, level, 2, out);
      free(acc); free(v);
    } else {
      memcpy(out, cur, 8 * w);
    }
  }
  free(cur); free(rot);
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* MPC-to-CKKS, the server's step (Algorithm mpc2ckks, last step)                          */
/* ------------------------------------------------------------------------------------ */
/* The client encrypts its field share tmp_0 and the server adds its own share tmp_1 (a ring
 * element mod Q_level in coefficient form, one residue per limb in [0, q_i)) as a plaintext:
 * out = (c0 + tmp_1, c1) mod q_i.  ct, out: [2][level+1][N]; share: [level+1][N]. */
void orc_add_share(const orc_ctx* c, const uint64_t* ct, int level, const uint64_t* share, uint64_t* out) {
  int n = c->n, nl = level + 1;
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->mod[i];
    for (int k = 0; k < n; ++k) {
      out[(size_t)i * n + k] = addm(ct[(size_t)i * n + k], share[(size_t)i * n + k] % q, q);
      out[((size_t)nl + i) * n + k] = ct[((size_t)nl + i) * n + k];
    }
  }
}

/* ------------------------------------------------------------------------------------ */
/* Identity and Expansion operators (Table "opertors": element-wise ewadd / ewmul of ct-ct */
/* and ct-pt, scalar sadd / smul by broadcast; Section "Consistent Packing for Single      */
/* Operator": a summation followed by a scalar operator skips the mask and the broadcast)  */
/* ------------------------------------------------------------------------------------ */
static void tensor_acc(const orc_ctx* c, uint64_t* acc3, const uint64_t* a, const uint64_t* r, int nl);

/* ewadd_cc: a + b (both polys, every limb) */
void orc_ew_add(const orc_ctx* c, const uint64_t* a, const uint64_t* b, int level, uint64_t* out) {
  size_t w = (size_t)2 * (level + 1) * c->n;
  memcpy(out, a, 8 * w);
  add_ct(c, out, b, level + 1, 2);
}

/* ewadd_cp: (c0 + pt, c1), pt a coefficient-form plaintext at the ciphertext's level and scale */
void orc_ew_add_plain(const orc_ctx* c, const uint64_t* a, const uint64_t* pt, int level, uint64_t* out) {
  orc_add_share(c, a, level, pt, out);
}

/* ewmul_cp: (c0 pt, c1 pt) in R_{Q_level}; the scale becomes the product of the two scales */
void orc_ew_mul_plain(const orc_ctx* c, const uint64_t* a, const uint64_t* pt, int level, uint64_t* out) {
  size_t w = (size_t)2 * (level + 1) * c->n;
  memset(out, 0, 8 * w);
  mac_pt(c, out, pt, a, level + 1);
}

/* ewmul_cc: the tensor (a0 b0, a0 b1 + a1 b0, a1 b1), then relinearised with the s^2 key */
int orc_ew_mul_relin(const orc_keys* K, const uint64_t* a, const uint64_t* b, int level, uint64_t* out) {
  const orc_ctx* c = K->c;
  uint64_t* t3 = (uint64_t*)calloc((size_t)3 * (level + 1) * c->n, 8);
  tensor_acc(c, t3, a, b, level + 1);
  int rc = orc_relinearize(K, t3, level, out);
  free(t3);
  return rc;
}

/* sadd / smul with a ciphertext scalar column (op 0: add, 1: multiply and relinearise).
 * from_sum = 0: s holds the scalar column in its first block of `block` slots (zero elsewhere)
 *   and is broadcast to n_blocks blocks by the right rotate-and-sum (log2 n_blocks rotations);
 * from_sum = 1: s is the input of a summation over its n_blocks blocks (block * n_blocks = N/2),
 *   whose unmasked left rotate-and-sum already holds the sum in every block: the mask and the
 *   broadcast are skipped (log2 n_blocks rotations, no product, no level).
 * a and s at `level`; out = a (op) that vector. */
int orc_scalar_op(const orc_keys* K, const uint64_t* a, const uint64_t* s_ct, int level, int block, int n_blocks, int op, int from_sum,
                  uint64_t* out) {
  const orc_ctx* c = K->c;
  if ((op != 0 && op != 1) || (from_sum != 0 && from_sum != 1)) return -3;
  if (from_sum && (int64_t)block * n_blocks != c->n / 2) return -3;
  size_t w = (size_t)2 * (level + 1) * c->n;
  uint64_t* v = (uint64_t*)malloc(8 * w);
  int rc = orc_rotate_sum(K, s_ct, level, block, n_blocks, from_sum ? 0 : 1, 0, v);
  if (rc == 0) {
    if (op == 0) orc_ew_add(c, a, v, level, out);
    else rc = orc_ew_mul_relin(K, a, v, level, out);
  }
  free(v);
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Re-randomisation before mask-to-share (opt-in; the paper leaves c1 as the evaluation    */
/* produced it, and c1 depends on the server's weights)                                    */
/* ------------------------------------------------------------------------------------ */
/* Public key over the ciphertext primes: p1 = a (uniform per limb, tag pk-a, object 0, key
 * seed), p0 = -a s + e (e Gaussian, tag pk-e).  Re-randomised ciphertext:
 *   (c0 + v p0 + e0, c1 + v p1 + e1) mod Q_level,
 * v ternary (tag rr-v), e1 Gaussian (tag rr-e1), e0 a uniform integer in [-2^F, 2^F] (tag
 * rr-e0: the 128-bit Philox block mod 2^(F+1) + 1, minus 2^F), object id ct_id, key `seed`;
 * it decrypts to m + v e + e0 + e1 s, so the flooding term e0 hides the evaluation noise. */
enum { TAG_PK_A = 7, TAG_PK_E = 8, TAG_RR_V = 9, TAG_RR_E0 = 10, TAG_RR_E1 = 11 };
static int64_t sample_flood(uint64_t seed, uint32_t k, uint32_t obj, int bits) {
  uint32_t w[4]; philox_at(seed, k, LIMB_INT, obj, TAG_RR_E0, w);
  u128 x = ((u128)w[3] << 96) | ((u128)w[2] << 64) | ((u128)w[1] << 32) | (u128)w[0];
  u128 m = ((u128)2 << bits) + 1;
  return (int64_t)(uint64_t)(x % m) - ((int64_t)1 << bits);
}
int orc_rerandomize(const orc_keys* K, const uint64_t* ct, int level, uint64_t seed, uint32_t ct_id, int flood_bits, uint64_t* out) {
  const orc_ctx* c = K->c;
  if (flood_bits < 32 || flood_bits > 48 || level < 0 || level >= c->n_q) return -1;
  int n = c->n, nl = level + 1;
  int32_t* v = (int32_t*)malloc(4 * n);
  int32_t* epk = (int32_t*)malloc(4 * n);
  int32_t* e1 = (int32_t*)malloc(4 * n);
  int64_t* e0 = (int64_t*)malloc(8 * n);
  for (int k = 0; k < n; ++k) {
    uint32_t w[4]; philox_at(seed, (uint32_t)k, LIMB_INT, ct_id, TAG_RR_V, w);
    v[k] = (int)(w[0] % 3u) - 1;
    epk[k] = sample_gauss(K->seed, (uint32_t)k, 0, TAG_PK_E);
    e1[k] = sample_gauss(seed, (uint32_t)k, ct_id, TAG_RR_E1);
    e0[k] = sample_flood(seed, (uint32_t)k, ct_id, flood_bits);
  }
  #pragma omp parallel for
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->mod[i];
    uint64_t* a = (uint64_t*)malloc(8 * n);
    uint64_t* p0 = (uint64_t*)malloc(8 * n);
    uint64_t* vq = (uint64_t*)malloc(8 * n);
    uint64_t* t = (uint64_t*)malloc(8 * n);
    for (int k = 0; k < n; ++k) a[k] = sample_uniform(K->seed, (uint32_t)k, (uint32_t)i, 0, TAG_PK_A, q);
    polymul(c, i, a, K->s_rns + (size_t)i * n, p0);
    for (int k = 0; k < n; ++k) { p0[k] = subm(smod(epk[k], q), p0[k], q); vq[k] = smod(v[k], q); }
    polymul(c, i, vq, p0, t);
    for (int k = 0; k < n; ++k) out[(size_t)i * n + k] = addm(addm(ct[(size_t)i * n + k], t[k], q), smod(e0[k], q), q);
    polymul(c, i, vq, a, t);
    for (int k = 0; k < n; ++k)
      out[((size_t)nl + i) * n + k] = addm(addm(ct[((size_t)nl + i) * n + k], t[k], q), smod(e1[k], q), q);
    free(a); free(p0); free(vq); free(t);
  }
  free(v); free(epk); free(e1); free(e0);
  return 0;
}

/* number of OpenMP threads the oracle's parallel loops use */
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
/* thread count of the parallel loops from now on (n >= 1); returns the previous count */
int orc_set_threads(int n) {
  int prev = omp_get_max_threads();
  if (n >= 1) omp_set_num_threads(n);
  return prev;
}

/* ------------------------------------------------------------------------------------ */
/* matmul_cc (Section "Efficient Protocol for Fused MatMuls", "Building Blocks": observations */
/* 1-2, steps 1-3, and the Multi-Head Optimization), one head group, B pre-rotated        */
/* ------------------------------------------------------------------------------------ */
/* Packing of a group of H_g heads (reading of the multi-head packing, the layout figure is not
 * available): with L' = 2^ceil(log2 L), c = S / (L' H_g) columns per ciphertext and n = d/c
 * ciphertexts per operand, ciphertext a holds at slot i + L'(h + H_g kappa):
 *   A_h{i, a c + kappa}                      (A = Q_h, spatial-first per head)
 *   B_h{a c + kappa, (i + kappa) mod L'}     (B = K_h^T rows, reduce-first, pre-rotated by kappa)
 * Output ciphertext g (g < L'/c) holds at slot i + L'(h + H_g kappa'):
 *   C_h{i, (i + g c + kappa') mod L'}        (diagonal packing: diagonal g c + kappa')       */
void orc_cc_geometry(const orc_ctx* c, int H_g, int L, int d, int32_t* out /* [4] */) {
  int s = c->n / 2;
  int lp = 1 << ceil_log2(L);
  int cc = s / (lp * H_g);
  out[0] = lp; out[1] = cc; out[2] = (d + cc - 1) / cc; out[3] = lp / cc;
}

/* slot vectors of the masks */
static void mask_lo(int s, int lp, int t, double* v) { for (int j = 0; j < s; ++j) v[j] = (j % lp) < lp - t ? 1.0 : 0.0; }
static void mask_hi(int s, int lp, int t, double* v) { for (int j = 0; j < s; ++j) v[j] = (j % lp) >= lp - t ? 1.0 : 0.0; }
static void mask_blk_ge(int s, int blk, int tau, double* v) { for (int j = 0; j < s; ++j) v[j] = (j / blk) >= tau ? 1.0 : 0.0; }
static void mask_blk_lt(int s, int blk, int tau, double* v) { for (int j = 0; j < s; ++j) v[j] = (j / blk) < tau ? 1.0 : 0.0; }

/* acc (+)= pt (.) ct  for a degree-1 ct at nl limbs (pt encoded from a slot vector) */
static void mac_vec(const orc_ctx* c, uint64_t* acc, const double* vec, double delta, const uint64_t* ct, int level) {
  int n = c->n, nl = level + 1;
  uint64_t* pt = (uint64_t*)malloc(8 * (size_t)nl * n);
  orc_encode_rns(c, vec, n / 2, delta, level, pt);
  mac_pt(c, acc, pt, ct, nl);
  free(pt);
}

/* tensor product accumulation: acc3 += (a0 r0, a0 r1 + a1 r0, a1 r1), all at nl limbs */
static void tensor_acc(const orc_ctx* c, uint64_t* acc3, const uint64_t* a, const uint64_t* r, int nl) {
  int n = c->n;
  #pragma omp parallel for
  for (int i = 0; i < nl; ++i) {
    uint64_t q = c->mod[i];
    uint64_t* t = (uint64_t*)malloc(8 * n);
    const uint64_t *a0 = a + (size_t)i * n, *a1 = a + ((size_t)nl + i) * n;
    const uint64_t *r0 = r + (size_t)i * n, *r1 = r + ((size_t)nl + i) * n;
    uint64_t *d0 = acc3 + (size_t)i * n, *d1 = acc3 + ((size_t)nl + i) * n, *d2 = acc3 + ((size_t)2 * nl + i) * n;
    polymul(c, i, a0, r0, t); for (int k = 0; k < n; ++k) d0[k] = addm(d0[k], t[k], q);
    polymul(c, i, a0, r1, t); for (int k = 0; k < n; ++k) d1[k] = addm(d1[k], t[k], q);
    polymul(c, i, a1, r0, t); for (int k = 0; k < n; ++k) d1[k] = addm(d1[k], t[k], q);
    polymul(c, i, a1, r1, t); for (int k = 0; k < n; ++k) d2[k] = addm(d2[k], t[k], q);
    free(t);
  }
}

/* Pinned schedule, inputs at `level` (A_a and pre-rotated B'_a, n_ct each, [ct][2][level+1][N]):
 *  step 2 (for t < L'): B''_a = 2^10 B'_a (noise boost, an exact integer scalar), then
 *          R_{a,t} = Rescale( Rot_l^t(B''_a) (.) M^lo_t + Rot_r^{L'-t}(B''_a) (.) M^hi_t ),
 *          masks encoded at q_level * 2^10 (t = 0: B''_a times the all-ones mask);
 *          T_t = Rescale( Relin( sum_a Drop(A_a) (x) R_{a,t} ) )   (summed before relinearising)
 *  step 3 (t = g c + tau): V_t = Rot_r^{tau H_g L'}(T_t);
 *          O_g += V_t (.) M^{>=tau};  O_{(g+1) mod (L'/c)} += V_t (.) M^{<tau}  (masks at q_{level-2} / 2^10);
 *          O_g = Rescale(O_g).
 * Output: L'/c cts at level-3, [g][2][level-2][N].  out_mask (NULL = all) selects the outputs;
 * only the t that feed them are computed.
 * n_dense < L'/c (Softmax x V_h with zero-padded columns): output g' < n_dense gathers the
 * accumulators O_g of every g with g mod n_dense = g' (the sum of those ciphertexts, taken before
 * their common rescale), so n_dense outputs come out. */
static int cc_steps23(const orc_keys* K, const uint64_t* A, const uint64_t* Bp, int n_ct, int level, int H_g, int L, int d,
                      int n_dense, const uint8_t* out_mask, uint64_t* O) {
  const orc_ctx* c = K->c;
  int n = c->n, s = n / 2;
  if (level < 3) return -2;
  int32_t geo[4]; orc_cc_geometry(c, H_g, L, d, geo);
  int lp = geo[0], cc = geo[1], n_out = geo[3];
  if (n_ct != geo[2] || cc < 1 || cc > lp || lp * H_g * cc != s) return -3;
  if (n_dense < 1 || n_out % n_dense) return -3;
  int nl = level + 1, l2 = level - 1, l1 = level - 2;
  size_t w3 = (size_t)2 * nl * n, w2 = (size_t)2 * (l2 + 1) * n, w1 = (size_t)2 * (l1 + 1) * n;
  double dm2 = (double)c->mod[level] * 1024.0, dm3 = (double)c->mod[l1] / NOISE_BOOST;
  uint64_t* bs = (uint64_t*)malloc(8 * w3 * (size_t)n_ct);
  for (int a = 0; a < n_ct; ++a) scale_ct(c, Bp + (size_t)a * w3, (uint64_t)NOISE_BOOST, nl, bs + (size_t)a * w3);
  double* v = (double*)malloc(8 * s);
  uint64_t* rot = (uint64_t*)malloc(8 * w3);
  uint64_t* racc = (uint64_t*)malloc(8 * w3);
  uint64_t* R = (uint64_t*)malloc(8 * w2);
  uint64_t* Ad = (uint64_t*)malloc(8 * w2);
  uint64_t* T3 = (uint64_t*)malloc(8 * (size_t)3 * (l2 + 1) * n);
  uint64_t* T = (uint64_t*)malloc(8 * w2);
  uint64_t* Tr = (uint64_t*)malloc(8 * w1);
  uint64_t* V = (uint64_t*)malloc(8 * w1);
  uint64_t* acc = (uint64_t*)calloc((size_t)n_dense * w1, 8);
  int rc = 0;
  for (int t = 0; t < lp && rc == 0; ++t) {
    int g = (t / cc) % n_dense, tau = t % cc, g2 = ((t / cc + 1) % n_out) % n_dense;
    int need = !out_mask || out_mask[g] || (tau > 0 && out_mask[g2]);
    if (!need) continue;
    memset(T3, 0, 8 * (size_t)3 * (l2 + 1) * n);
    for (int a = 0; a < n_ct && rc == 0; ++a) {
      const uint64_t* b = bs + (size_t)a * w3;
      memset(racc, 0, 8 * w3);
      if (t == 0) {
        mask_lo(s, lp, 0, v); mac_vec(c, racc, v, dm2, b, level);
      } else {
        if (orc_rotate(K, b, level, t, rot) != 0) { rc = -1; break; }
        mask_lo(s, lp, t, v); mac_vec(c, racc, v, dm2, rot, level);
        if (orc_rotate(K, b, level, -(int64_t)(lp - t), rot) != 0) { rc = -1; break; }
        mask_hi(s, lp, t, v); mac_vec(c, racc, v, dm2, rot, level);
      }
      orc_rescale(c, racc, level, 2, R);
      /* drop A_a to level-1: keep limbs 0..l2 of each poly */
      const uint64_t* aa = A + (size_t)a * w3;
      for (int p = 0; p < 2; ++p) memcpy(Ad + (size_t)p * (l2 + 1) * n, aa + (size_t)p * nl * n, 8 * (size_t)(l2 + 1) * n);
      tensor_acc(c, T3, Ad, R, l2 + 1);
    }
    if (rc) break;
    if (orc_relinearize(K, T3, l2, T) != 0) { rc = -1; break; }
    orc_rescale(c, T, l2, 2, Tr);
    if (tau == 0) memcpy(V, Tr, 8 * w1);
    else if (orc_rotate(K, Tr, l1, -(int64_t)tau * H_g * lp, V) != 0) { rc = -1; break; }
    int blk = lp * H_g;
    if (!out_mask || out_mask[g]) { mask_blk_ge(s, blk, tau, v); mac_vec(c, acc + (size_t)g * w1, v, dm3, V, l1); }
    if (tau > 0 && (!out_mask || out_mask[g2])) { mask_blk_lt(s, blk, tau, v); mac_vec(c, acc + (size_t)g2 * w1, v, dm3, V, l1); }
  }
  if (rc == 0)
    for (int g = 0; g < n_dense; ++g)
      if (!out_mask || out_mask[g]) orc_rescale(c, acc + (size_t)g * w1, l1, 2, O + (size_t)g * 2 * l1 * n);
  free(v); free(rot); free(racc); free(R); free(Ad); free(T3); free(T); free(Tr); free(V); free(acc); free(bs);
  return rc;
}

/* slot vector of the step-1 mask for class kappa: slot i + L' beta (class beta / H_g) is 1 when
 * its class is kappa and lo <= i < hi */
static void mask_cls(int s, int lp, int H_g, int kap, int lo, int hi, double* v) {
  for (int j = 0; j < s; ++j) {
    int i = j % lp, cls = (j / lp) / H_g;
    v[j] = (cls == kap && i >= lo && i < hi) ? 1.0 : 0.0;
  }
}

/* Step 1 (B row pre-rotation by kappa) in homomorphic form, for B_a that the client did not
 * pre-rotate: with B''_a = 2^10 B_a (noise boost, an exact integer scalar),
 *   B'_a = Rescale( B''_a (.) M^0 + sum_{kappa=1}^{c-1} [ Rot_l^kappa(B''_a) (.) M^1_kappa
 *                                                   + Rot_r^{L'-kappa}(B''_a) (.) M^2_kappa ] ),
 * masks encoded at q_level / 2^10: M^0 selects the blocks of class 0, M^1_kappa the slots of
 * class kappa with i < L' - kappa, M^2_kappa those with i >= L' - kappa.  Block (h, kappa) of
 * B'_a then holds B_h{a c + kappa, (i + kappa) mod L'} at scale Delta_B, one level down; A_a is
 * dropped to the same level and steps 2-3 follow.  Output: L'/c cts at level-4. */
static int cc_step1(const orc_keys* K, const uint64_t* A, const uint64_t* B, int n_ct, int level, int H_g, int L, int d,
                    uint64_t* Ad, uint64_t* Bq) {
  const orc_ctx* c = K->c;
  int n = c->n, s = n / 2;
  int32_t geo[4]; orc_cc_geometry(c, H_g, L, d, geo);
  int lp = geo[0], cc = geo[1];
  int nl = level + 1;
  size_t w = (size_t)2 * nl * n, wq = (size_t)2 * level * n;
  double dm1 = (double)c->mod[level] / NOISE_BOOST;
  double* v = (double*)malloc(8 * s);
  uint64_t* bs = (uint64_t*)malloc(8 * w);
  uint64_t* rot = (uint64_t*)malloc(8 * w);
  uint64_t* acc = (uint64_t*)malloc(8 * w);
  int rc = 0;
  for (int a = 0; a < n_ct && rc == 0; ++a) {
    scale_ct(c, B + (size_t)a * w, (uint64_t)NOISE_BOOST, nl, bs);
    memset(acc, 0, 8 * w);
    mask_cls(s, lp, H_g, 0, 0, lp, v); mac_vec(c, acc, v, dm1, bs, level);
    for (int kap = 1; kap < cc; ++kap) {
      if (orc_rotate(K, bs, level, kap, rot) != 0) { rc = -1; break; }
      mask_cls(s, lp, H_g, kap, 0, lp - kap, v); mac_vec(c, acc, v, dm1, rot, level);
      if (orc_rotate(K, bs, level, -(int64_t)(lp - kap), rot) != 0) { rc = -1; break; }
      mask_cls(s, lp, H_g, kap, lp - kap, lp, v); mac_vec(c, acc, v, dm1, rot, level);
    }
    if (rc) break;
    orc_rescale(c, acc, level, 2, Bq + (size_t)a * wq);
    const uint64_t* aa = A + (size_t)a * w;
    for (int p = 0; p < 2; ++p) memcpy(Ad + (size_t)a * wq + (size_t)p * level * n, aa + (size_t)p * nl * n, 8 * (size_t)level * n);
  }
  free(v); free(bs); free(rot); free(acc);
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* matmul_cc with BSGS (Appendix "BSGS Optimization", figure bsgs): baby-step inner       */
/* rotations of B', giant-step inner rotations of A, and the giant step's own rotation     */
/* postponed into step 3                                                                   */
/* ------------------------------------------------------------------------------------ */
/* Split of the L' inner rotations of step 2 and of the c row classes of step 1: a fixed rule
 * (it changes bits), B = 2^ceil(log2(L')/2), G = L'/B; b1 = 2^ceil(log2(c)/2), g1 = c/b1. */
void orc_cc_bsgs_split(const orc_ctx* c, int H_g, int L, int d, int32_t* out /* [4] */) {
  int32_t geo[4]; orc_cc_geometry(c, H_g, L, d, geo);
  int lb = ceil_log2(geo[0]), lc = ceil_log2(geo[1]);
  out[0] = 1 << ((lb + 1) / 2); out[1] = geo[0] / out[0];
  out[2] = 1 << ((lc + 1) / 2); out[3] = geo[1] / out[2];
}

/* slot vector v rotated left by r slots (out[k] = v[(k + r) mod S]); r may be negative */
static void rot_vec(int s, const double* v, int64_t r, double* out) {
  int64_t rr = ((r % s) + s) % s;
  for (int k = 0; k < s; ++k) out[k] = v[(k + rr) % s];
}

/* Inner rotation of a ciphertext: every block of L' slots rotated left by t within itself,
 *   Rescale( Rot_l^t(x) (.) M^lo_t + Rot_r^{L'-t}(x) (.) M^hi_t )   (t = 0: x (.) M^lo_0),
 * masks encoded at `dm`; x at `level`, result at level-1. */
static int inner_rot(const orc_keys* K, const uint64_t* x, int level, int lp, int t, double dm, uint64_t* out) {
  const orc_ctx* c = K->c;
  int n = c->n, s = n / 2, nl = level + 1;
  size_t w = (size_t)2 * nl * n;
  double* v = (double*)malloc(8 * s);
  uint64_t* rot = (uint64_t*)malloc(8 * w);
  uint64_t* acc = (uint64_t*)calloc(w, 8);
  int rc = 0;
  if (t == 0) {
    mask_lo(s, lp, 0, v); mac_vec(c, acc, v, dm, x, level);
  } else if (orc_rotate(K, x, level, t, rot) != 0) {
    rc = -1;
  } else {
    mask_lo(s, lp, t, v); mac_vec(c, acc, v, dm, rot, level);
    if (orc_rotate(K, x, level, -(int64_t)(lp - t), rot) != 0) rc = -1;
    else { mask_hi(s, lp, t, v); mac_vec(c, acc, v, dm, rot, level); }
  }
  if (rc == 0) orc_rescale(c, acc, level, 2, out);
  free(v); free(rot); free(acc);
  return rc;
}

/* Steps 2-3 with BSGS.  Inputs at `level` (A_a and pre-rotated B'_a).  With t = j B + i:
 *   T_t = sum_a A_a (x) InnerRot_t(B'_a) = InnerRot_{jB}( sum_a InnerRot_{-jB}(A_a) (x) InnerRot_i(B'_a) ),
 * because an inner rotation is the same slot permutation in every block and the elementwise
 * product commutes with it.  So
 *   Y_{a,i}  = InnerRot_i(2^10 B'_a), masks at q_level 2^10               (baby steps, i < B)
 *   A'_{a,j} = InnerRot_{L'-jB}(2^10 A_a), masks at q_level / 2^10 (j >= 1),  Drop(A_a) for j = 0
 *   U_t      = Rescale( Relin( sum_a A'_{a,j} (x) Y_{a,i} ) ),  V_t = Rot_r^{tau H_g L'}(U_t)
 * and InnerRot_{jB} commutes with the step-3 block rotation and block masks.  Step 3 therefore
 * splits each V_t of giant step j >= 1 with the product masks M^{>=tau} H_j, M^{>=tau} Lo_j (into
 * O_g) and M^{<tau} H_j, M^{<tau} Lo_j (into O_{g+1}), where H_j keeps the in-block positions
 * >= jB and Lo_j the others; every accumulator (g, j, H) is rotated left by jB and every (g, j, Lo)
 * right by L' - jB before it joins O_g (one extra mask product per V_t and one rotation per
 * accumulator: the giant step of step 2 done once per output instead of once per ciphertext).
 * j = 0 accumulates straight into O_g as in the plain schedule.  Step-3 masks at q_{level-2} / 2^10;
 * O_g = Rescale(O_g).  Outputs and folding (n_dense) as in cc_steps23. */
static int cc_steps23_bsgs(const orc_keys* K, const uint64_t* A, const uint64_t* Bp, int n_ct, int level, int H_g, int L, int d,
                           int n_dense, const uint8_t* out_mask, uint64_t* O) {
  const orc_ctx* c = K->c;
  int n = c->n, s = n / 2;
  if (level < 3) return -2;
  int32_t geo[4]; orc_cc_geometry(c, H_g, L, d, geo);
  int lp = geo[0], cc = geo[1], n_out = geo[3];
  if (n_ct != geo[2] || cc < 1 || cc > lp || lp * H_g * cc != s) return -3;
  if (n_dense < 1 || n_out % n_dense) return -3;
  int32_t sp[4]; orc_cc_bsgs_split(c, H_g, L, d, sp);
  int Bb = sp[0], Gg = sp[1];
  int nl = level + 1, l2 = level - 1, l1 = level - 2;
  size_t w3 = (size_t)2 * nl * n, w2 = (size_t)2 * (l2 + 1) * n, w1 = (size_t)2 * (l1 + 1) * n;
  double dmB = (double)c->mod[level] * 1024.0, dmA = (double)c->mod[level] / NOISE_BOOST, dm3 = (double)c->mod[l1] / NOISE_BOOST;
  int blk = lp * H_g;
  /* which t feed a selected output */
  uint8_t* need_t = (uint8_t*)calloc(lp, 1);
  uint8_t* need_i = (uint8_t*)calloc(Bb, 1);
  uint8_t* need_j = (uint8_t*)calloc(Gg, 1);
  for (int t = 0; t < lp; ++t) {
    int g = (t / cc) % n_dense, tau = t % cc, g2 = ((t / cc + 1) % n_out) % n_dense;
    if (!out_mask || out_mask[g] || (tau > 0 && out_mask[g2])) { need_t[t] = 1; need_i[t % Bb] = 1; need_j[t / Bb] = 1; }
  }
  uint64_t* tmp = (uint64_t*)malloc(8 * w3);
  uint64_t* Y = (uint64_t*)calloc((size_t)n_ct * Bb * w2, 8);
  uint64_t* Ap = (uint64_t*)calloc((size_t)n_ct * Gg * w2, 8);
  int rc = 0;
  /* baby steps on B', giant steps on A (both noise-boosted) */
  for (int a = 0; a < n_ct && rc == 0; ++a) {
    scale_ct(c, Bp + (size_t)a * w3, (uint64_t)NOISE_BOOST, nl, tmp);
    for (int i = 0; i < Bb && rc == 0; ++i)
      if (need_i[i]) rc = inner_rot(K, tmp, level, lp, i, dmB, Y + ((size_t)a * Bb + i) * w2);
    const uint64_t* aa = A + (size_t)a * w3;
    for (int p = 0; p < 2; ++p)
      memcpy(Ap + (size_t)a * Gg * w2 + (size_t)p * (l2 + 1) * n, aa + (size_t)p * nl * n, 8 * (size_t)(l2 + 1) * n);
    scale_ct(c, aa, (uint64_t)NOISE_BOOST, nl, tmp);
    for (int j = 1; j < Gg && rc == 0; ++j)
      if (need_j[j]) rc = inner_rot(K, tmp, level, lp, lp - j * Bb, dmA, Ap + ((size_t)a * Gg + j) * w2);
  }
  double* v = (double*)malloc(8 * s);
  double* mv = (double*)malloc(8 * s);
  uint64_t* T3 = (uint64_t*)malloc(8 * (size_t)3 * (l2 + 1) * n);
  uint64_t* T = (uint64_t*)malloc(8 * w2);
  uint64_t* U = (uint64_t*)malloc(8 * w1);
  uint64_t* V = (uint64_t*)malloc(8 * w1);
  uint64_t* acc = (uint64_t*)calloc((size_t)n_dense * w1, 8);
  /* giant-step accumulators: [g][j][part], part 0 = H_j (positions >= jB), 1 = Lo_j */
  uint64_t* accj = (uint64_t*)calloc((size_t)n_dense * Gg * 2 * w1, 8);
  uint8_t* used = (uint8_t*)calloc((size_t)n_dense * Gg * 2, 1);
  for (int t = 0; t < lp && rc == 0; ++t) {
    if (!need_t[t]) continue;
    int j = t / Bb, i = t % Bb;
    int g = (t / cc) % n_dense, tau = t % cc, g2 = ((t / cc + 1) % n_out) % n_dense;
    memset(T3, 0, 8 * (size_t)3 * (l2 + 1) * n);
    for (int a = 0; a < n_ct; ++a) tensor_acc(c, T3, Ap + ((size_t)a * Gg + j) * w2, Y + ((size_t)a * Bb + i) * w2, l2 + 1);
    if (orc_relinearize(K, T3, l2, T) != 0) { rc = -1; break; }
    orc_rescale(c, T, l2, 2, U);
    if (tau == 0) memcpy(V, U, 8 * w1);
    else if (orc_rotate(K, U, l1, -(int64_t)tau * blk, V) != 0) { rc = -1; break; }
    for (int side = 0; side < 2; ++side) {          /* side 0: M^{>=tau} into O_g; 1: M^{<tau} into O_{g+1} */
      int go = side == 0 ? g : g2;
      if (side == 1 && tau == 0) continue;
      if (out_mask && !out_mask[go]) continue;
      if (side == 0) mask_blk_ge(s, blk, tau, v); else mask_blk_lt(s, blk, tau, v);
      if (j == 0) { mac_vec(c, acc + (size_t)go * w1, v, dm3, V, l1); continue; }
      for (int part = 0; part < 2; ++part) {
        for (int k = 0; k < s; ++k) {
          int in_hi = (k % lp) >= j * Bb;
          mv[k] = v[k] * ((part == 0) == in_hi ? 1.0 : 0.0);
        }
        size_t slot = ((size_t)go * Gg + j) * 2 + part;
        mac_vec(c, accj + slot * w1, mv, dm3, V, l1);
        used[slot] = 1;
      }
    }
  }
  /* the postponed giant-step rotations: (g, j, H_j) left by jB, (g, j, Lo_j) right by L' - jB */
  for (int g = 0; g < n_dense && rc == 0; ++g)
    for (int j = 1; j < Gg && rc == 0; ++j)
      for (int part = 0; part < 2 && rc == 0; ++part) {
        size_t slot = ((size_t)g * Gg + j) * 2 + part;
        if (!used[slot]) continue;
        int64_t steps = part == 0 ? (int64_t)j * Bb : -(int64_t)(lp - j * Bb);
        if (orc_rotate(K, accj + slot * w1, l1, steps, V) != 0) { rc = -1; break; }
        add_ct(c, acc + (size_t)g * w1, V, l1 + 1, 2);
      }
  if (rc == 0)
    for (int g = 0; g < n_dense; ++g)
      if (!out_mask || out_mask[g]) orc_rescale(c, acc + (size_t)g * w1, l1, 2, O + (size_t)g * 2 * l1 * n);
  free(need_t); free(need_i); free(need_j); free(tmp); free(Y); free(Ap); free(v); free(mv); free(T3); free(T); free(U); free(V);
  free(acc); free(accj); free(used);
  return rc;
}

/* Step 1 with BSGS: with kappa = j b1 + i and B''_a = 2^10 B_a,
 *   sum_kappa Rot_l^kappa(B'') (.) M^1_kappa = sum_j Rot_l^{j b1}( sum_i Rot_l^i(B'') (.) Rot_r^{j b1}(M^1_kappa) )
 *   sum_kappa Rot_r^{L'-kappa}(B'') (.) M^2_kappa = sum_j Rot_r^{L'-j b1}( sum_i Rot_l^i(B'') (.) Rot_l^{L'-j b1}(M^2_kappa) )
 * (M^1_0 = M^0, M^2_0 = 0), the rotation of a product being the product of the rotations.  Both
 * sums share the b1 - 1 baby rotations Rot_l^i(B''); the giant rotations (g1 - 1 left, g1 right)
 * act on the partial sums, before the one rescale.  Pre-rotated masks are exact slot permutations
 * of the plain schedule's masks, encoded at q_level / 2^10.  Output as cc_step1. */
static int cc_step1_bsgs(const orc_keys* K, const uint64_t* A, const uint64_t* B, int n_ct, int level, int H_g, int L, int d,
                         uint64_t* Ad, uint64_t* Bq) {
  const orc_ctx* c = K->c;
  int n = c->n, s = n / 2;
  int32_t geo[4]; orc_cc_geometry(c, H_g, L, d, geo);
  int lp = geo[0];
  int32_t sp[4]; orc_cc_bsgs_split(c, H_g, L, d, sp);
  int b1 = sp[2], g1 = sp[3];
  int nl = level + 1;
  size_t w = (size_t)2 * nl * n, wq = (size_t)2 * level * n;
  double dm1 = (double)c->mod[level] / NOISE_BOOST;
  double* v = (double*)malloc(8 * s);
  double* rv = (double*)malloc(8 * s);
  uint64_t* X = (uint64_t*)malloc(8 * w * (size_t)b1);
  uint64_t* part = (uint64_t*)malloc(8 * w);
  uint64_t* rot = (uint64_t*)malloc(8 * w);
  uint64_t* acc = (uint64_t*)malloc(8 * w);
  int rc = 0;
  for (int a = 0; a < n_ct && rc == 0; ++a) {
    scale_ct(c, B + (size_t)a * w, (uint64_t)NOISE_BOOST, nl, X);
    for (int i = 1; i < b1 && rc == 0; ++i)
      if (orc_rotate(K, X, level, i, X + (size_t)i * w) != 0) rc = -1;
    if (rc) break;
    memset(acc, 0, 8 * w);
    for (int j = 0; j < g1 && rc == 0; ++j) {
      for (int fam = 0; fam < 2 && rc == 0; ++fam) {   /* fam 0: left family M^1, 1: right family M^2 */
        memset(part, 0, 8 * w);
        int terms = 0;
        for (int i = 0; i < b1; ++i) {
          int kap = j * b1 + i;
          if (fam == 1 && kap == 0) continue;
          if (fam == 0) mask_cls(s, lp, H_g, kap, 0, kap == 0 ? lp : lp - kap, v);
          else mask_cls(s, lp, H_g, kap, lp - kap, lp, v);
          if (fam == 0) rot_vec(s, v, -(int64_t)j * b1, rv);          /* Rot_r^{j b1} */
          else rot_vec(s, v, (int64_t)(lp - j * b1), rv);             /* Rot_l^{L' - j b1} */
          mac_vec(c, part, rv, dm1, X + (size_t)i * w, level);
          ++terms;
        }
        if (!terms) continue;
        int64_t steps = fam == 0 ? (int64_t)j * b1 : -(int64_t)(lp - j * b1);
        if (orc_rotate(K, part, level, steps, rot) != 0) { rc = -1; break; }
        add_ct(c, acc, rot, nl, 2);
      }
    }
    if (rc) break;
    orc_rescale(c, acc, level, 2, Bq + (size_t)a * wq);
    const uint64_t* aa = A + (size_t)a * w;
    for (int p = 0; p < 2; ++p) memcpy(Ad + (size_t)a * wq + (size_t)p * level * n, aa + (size_t)p * nl * n, 8 * (size_t)level * n);
  }
  free(v); free(rv); free(X); free(part); free(rot); free(acc);
  return rc;
}

/* One head group of matmul_cc.  b_prerotated != 0: B_a arrive pre-rotated by the client
 * (step 1 applied to the plaintext), inputs at `level` >= 3, output at level-3; else step 1
 * runs homomorphically first, inputs at `level` >= 4, output at level-4. */
static int cc_run(const orc_keys* K, const uint64_t* A, const uint64_t* B, int n_ct, int level, int H_g, int L, int d, int b_prerotated,
                  int schedule, int n_dense, const uint8_t* out_mask, uint64_t* O) {
  if (schedule != 0 && schedule != 1) return -3;
  if (b_prerotated)
    return schedule ? cc_steps23_bsgs(K, A, B, n_ct, level, H_g, L, d, n_dense, out_mask, O)
                    : cc_steps23(K, A, B, n_ct, level, H_g, L, d, n_dense, out_mask, O);
  const orc_ctx* c = K->c;
  if (level < 4) return -2;
  int32_t geo[4]; orc_cc_geometry(c, H_g, L, d, geo);
  if (n_ct != geo[2] || geo[1] < 1 || geo[1] > geo[0]) return -3;
  size_t wq = (size_t)2 * level * c->n * n_ct;
  uint64_t* Ad = (uint64_t*)malloc(8 * wq);
  uint64_t* Bq = (uint64_t*)malloc(8 * wq);
  int rc = schedule ? cc_step1_bsgs(K, A, B, n_ct, level, H_g, L, d, Ad, Bq) : cc_step1(K, A, B, n_ct, level, H_g, L, d, Ad, Bq);
  if (rc == 0)
    rc = schedule ? cc_steps23_bsgs(K, Ad, Bq, n_ct, level - 1, H_g, L, d, n_dense, out_mask, O)
                  : cc_steps23(K, Ad, Bq, n_ct, level - 1, H_g, L, d, n_dense, out_mask, O);
  free(Ad); free(Bq);
  return rc;
}

/* schedule 0: one inner rotation of every B'_a per t (steps 1-3 as written in "Building Blocks");
 * schedule 1: BSGS in steps 1 and 2 with the giant step folded into step 3 (Appendix "BSGS
 * Optimization").  Both decode to the same product; their words differ. */
int orc_matmul_cc_sched(const orc_keys* K, const uint64_t* A, const uint64_t* B, int n_ct, int level, int H_g, int L, int d,
                        int b_prerotated, int schedule, const uint8_t* out_mask, uint64_t* O) {
  int32_t geo[4]; orc_cc_geometry(K->c, H_g, L, d, geo);
  return cc_run(K, A, B, n_ct, level, H_g, L, d, b_prerotated, schedule, geo[3], out_mask, O);
}

int orc_matmul_cc(const orc_keys* K, const uint64_t* A, const uint64_t* B, int n_ct, int level, int H_g, int L, int d, int b_prerotated,
                  const uint8_t* out_mask, uint64_t* O) {
  return orc_matmul_cc_sched(K, A, B, n_ct, level, H_g, L, d, b_prerotated, 0, out_mask, O);
}

/* ------------------------------------------------------------------------------------ */
/* Softmax x V_h with zero padding ("Efficient Fused Computations in Multi-Head          */
/* Attention"; Appendix "Diagonal Ciphertext-Plaintext MatMul", figure diag (b))          */
/* ------------------------------------------------------------------------------------ */
/* The ct-ct protocol needs as many output columns as reduction rows, so V_h (L x d_v) is
 * taken as an L x L' matrix whose columns from d_v on are zero: the operands are A_h = the
 * L x L attention weights (reduction dimension d = L) and B_h = V_h with its d_v columns.
 * With d_v' = 2^ceil(log2 d_v), the diagonals D and D + d_v' (mod L') of the L x L' product are
 * complementary (one of the two is zero in every row), so the L'/d_v' diagonal ciphertexts whose
 * diagonal indices agree mod d_v' are added into one: output g' < d_v'/c holds at slot
 * i + L'(h + H_g kappa) the value Att_h{i, (i + g' c + kappa) mod d_v'} (0 for columns >= d_v),
 * the dense diagonal packing of the L x d_v' matrix.  Requires d_v' <= L' and c <= d_v'. */
void orc_cc_sv_geometry(const orc_ctx* c, int H_g, int L, int d_v, int32_t* out /* [5] */) {
  int32_t geo[4]; orc_cc_geometry(c, H_g, L, L, geo);
  int dvp = 1 << ceil_log2(d_v);
  out[0] = geo[0]; out[1] = geo[1]; out[2] = geo[2];
  out[3] = (dvp <= geo[0] && geo[1] <= dvp) ? dvp / geo[1] : 0;
  out[4] = dvp;
}

int orc_matmul_cc_sv_sched(const orc_keys* K, const uint64_t* A, const uint64_t* B, int n_ct, int level, int H_g, int L, int d_v,
                           int b_prerotated, int schedule, const uint8_t* out_mask, uint64_t* O) {
  int32_t geo[5]; orc_cc_sv_geometry(K->c, H_g, L, d_v, geo);
  if (geo[3] < 1) return -3;
  return cc_run(K, A, B, n_ct, level, H_g, L, L, b_prerotated, schedule, geo[3], out_mask, O);
}

int orc_matmul_cc_sv(const orc_keys* K, const uint64_t* A, const uint64_t* B, int n_ct, int level, int H_g, int L, int d_v,
                     int b_prerotated, const uint8_t* out_mask, uint64_t* O) {
  return orc_matmul_cc_sv_sched(K, A, B, n_ct, level, H_g, L, d_v, b_prerotated, 0, out_mask, O);
}

/* ------------------------------------------------------------------------------------ */
/* Column reordering of W_Q / W_K for the multi-head packing (Multi-Head Optimization, and */
/* "Efficient Fused Computations in Multi-Head Attention": matmul_cp + matmul_cc)         */
/* ------------------------------------------------------------------------------------ */
/* With the columns of W (d_in x n_heads d_head, head h owning columns h d_head .. h d_head +
 * d_head - 1) reordered in plaintext, the spatial-first output of matmul_cp IS the multi-head
 * packing of the ct-ct operands: output ciphertext b holds column b c + u of X W' at block u
 * (c = S / L'), and the operand ciphertext a of a head group (H_g heads from h0, c_g = S / (L' H_g),
 * ceil(d_head / c_g) ciphertexts, groups in order) must hold Y_{h0+h}{:, a c_g + kappa} at block
 * u = h + H_g kappa.  So column b c + u of W' is column (h0 + u mod H_g) d_head + a c_g + u / H_g
 * of W for b = (first ciphertext of the group) + a, and zero where a c_g + u / H_g >= d_head.
 * Writes d_in x n_cols (row-major) to out when it is not NULL; returns n_cols = c * (number of
 * operand ciphertexts), or -1 for a geometry the packing cannot hold. */
int orc_mhp_weight(const orc_ctx* c, const double* W, int d_in, int n_heads, int d_head, int L, double* out) {
  int s = c->n / 2, lp = 1 << ceil_log2(L), cc = s / lp;
  if (lp > s) return -1;
  int n_ct = 0;
  for (int rem = n_heads; rem > 0;) {
    int hg = 1;
    while (hg * 2 <= rem) hg *= 2;
    if (s % (lp * hg)) return -1;
    int cg = s / (lp * hg);
    if (cg > lp) return -1;
    n_ct += (d_head + cg - 1) / cg;
    rem -= hg;
  }
  int n_cols = n_ct * cc;
  if (!out) return n_cols;
  int b = 0, h0 = 0;
  for (int rem = n_heads; rem > 0;) {
    int hg = 1;
    while (hg * 2 <= rem) hg *= 2;
    int cg = s / (lp * hg), nct = (d_head + cg - 1) / cg;
    for (int a = 0; a < nct; ++a, ++b)
      for (int u = 0; u < cc; ++u) {
        int h = h0 + u % hg, col = a * cg + u / hg, j = b * cc + u;
        for (int r = 0; r < d_in; ++r)
          out[(size_t)r * n_cols + j] = col < d_head ? W[(size_t)r * n_heads * d_head + h * d_head + col] : 0.0;
      }
    h0 += hg;
    rem -= hg;
  }
  return n_cols;
}

/* Galois elements of one group's matmul_cc: left t and right L'-t for t < L', right tau H_g L' */
int orc_cc_galois(const orc_ctx* c, int H_g, int L, int d, uint64_t* out) {
  int32_t geo[4]; orc_cc_geometry(c, H_g, L, d, geo);
  int lp = geo[0], cc = geo[1], cnt = 0;
  for (int t = 1; t < lp; ++t) { out[cnt++] = galois_left(c, t); out[cnt++] = galois_left(c, -(int64_t)(lp - t)); }
  for (int tau = 1; tau < cc; ++tau) out[cnt++] = galois_left(c, -(int64_t)tau * H_g * lp);
  return cnt;
}

/* Galois elements of one group's BSGS schedule (steps 1-3), duplicates included:
 * baby left i / right L'-i (i < B), giant on A left L'-jB / right jB and the postponed giant
 * rotations left jB / right L'-jB (0 < j < G), step 3 right tau H_g L', and for step 1 left i
 * (i < b1), left j b1 (0 < j < g1), right L' - j b1 (j < g1).  out holds at least 2B + 4G + c + 2 b1 + 2 g1. */
int orc_cc_galois_bsgs(const orc_ctx* c, int H_g, int L, int d, uint64_t* out) {
  int32_t geo[4]; orc_cc_geometry(c, H_g, L, d, geo);
  int32_t sp[4]; orc_cc_bsgs_split(c, H_g, L, d, sp);
  int lp = geo[0], cc = geo[1], Bb = sp[0], Gg = sp[1], b1 = sp[2], g1 = sp[3], cnt = 0;
  for (int i = 1; i < Bb; ++i) { out[cnt++] = galois_left(c, i); out[cnt++] = galois_left(c, -(int64_t)(lp - i)); }
  for (int j = 1; j < Gg; ++j) {
    out[cnt++] = galois_left(c, lp - j * Bb); out[cnt++] = galois_left(c, -(int64_t)j * Bb);
    out[cnt++] = galois_left(c, j * Bb); out[cnt++] = galois_left(c, -(int64_t)(lp - j * Bb));
  }
  for (int tau = 1; tau < cc; ++tau) out[cnt++] = galois_left(c, -(int64_t)tau * H_g * lp);
  for (int i = 1; i < b1; ++i) out[cnt++] = galois_left(c, i);
  for (int j = 1; j < g1; ++j) out[cnt++] = galois_left(c, j * b1);
  for (int j = 0; j < g1; ++j) out[cnt++] = galois_left(c, -(int64_t)(lp - j * b1));
  return cnt;
}
