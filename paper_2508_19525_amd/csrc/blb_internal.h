// Internal declarations of the gfx950 engine: context / key / plan structures, the
// FP64 modular arithmetic used by every kernel, and the host-side launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <deque>
#include <vector>
#include "../../include/blb.h"

#define BLB_MAXM 16     // max moduli (q's + p's)
#define BLB_MAXQ 12     // max ciphertext primes
#define BLB_MAXSP 4     // max special primes
#define BLB_MAXALPHA 8  // max primes per key-switching digit

// ---------------------------------------------------------------------------------------
// Modular arithmetic on FP64 lanes.
//
// All primes are below 2^50, so every residue, and every sum of a few residues, is an
// integer that a double holds exactly.  A product a*b of integers with |a| <= A, |b| <= B is
// split exactly into p = fl(a*b) and e = fma(a, b, -p) (error-free product, |e| <= A B 2^-53);
// the quotient estimate t = rint(p * fl(1/q)) is within 1/2 + A B 2^-52 / q of a*b/q, so
// r = fma(-t, q, p) is an exact integer and r + e = a*b - t*q exactly, with
// |r + e| <= q/2 + 1.5 A B 2^-52 ("signed-lazy"): below 0.875 q for canonical operands
// (A = B = q), and below 2^53 whenever that bound is.  CDNA4 issues FP64 FMA at full rate,
// which makes this cheaper than 32-bit limb integer products.
// ---------------------------------------------------------------------------------------
#define BLB_TWO52 4503599627370496.0

__device__ __forceinline__ double u2d(uint64_t x) {  // x < 2^52
  return __longlong_as_double((long long)(x | 0x4330000000000000ull)) - BLB_TWO52;
}
__device__ __forceinline__ uint64_t d2u(double d) {  // integer 0 <= d < 2^52
  return (uint64_t)__double_as_longlong(d + BLB_TWO52) & 0x000FFFFFFFFFFFFFull;
}
// a*b - t*q, |result| <= q/2 + 1.5 |a| |b| 2^-52 (see above)
__device__ __forceinline__ double mulmod_s(double a, double b, double q, double qinv) {
  const double p = a * b;
  const double e = __builtin_fma(a, b, -p);
  const double t = __builtin_rint(p * qinv);
  const double r = __builtin_fma(-t, q, p);
  return r + e;
}
// x - round(x/q) q, |result| <= q/2 + tiny, for |x| < 2^52
__device__ __forceinline__ double reduce_s(double x, double q, double qinv) {
  const double t = __builtin_rint(x * qinv);
  return __builtin_fma(-t, q, x);
}
// signed-lazy (|x| < q) -> canonical [0, q)
__device__ __forceinline__ double canon(double x, double q) { return x < 0.0 ? x + q : x; }
// any |x| < 2^52 -> canonical
__device__ __forceinline__ double canon_full(double x, double q, double qinv) { return canon(reduce_s(x, q, qinv), q); }

// ---------------------------------------------------------------------------------------
// Shared structures (host and device)
// ---------------------------------------------------------------------------------------
struct ModEntry {
  double q;
  double qinv;  // fl(1/q)
  double ninv;  // N^-1 mod q
};
struct ModTable {
  ModEntry m[BLB_MAXM];
};
struct ModMap {
  int len;               // period of the modulus pattern over consecutive polys
  int idx[BLB_MAXM];     // modulus index of poly p = idx[p % len]
};

// Per-level key-switching constants.  Extended basis index e: 0..nl-1 = q_0..q_{nl-1},
// nl..nl+K-1 = p_0..p_{K-1}.
struct KsLevelConst {
  int nl, n_ext, n_digits, n_key_mod;
  int dlo[BLB_MAXQ], dhi[BLB_MAXQ];               // digit j covers extended indices [dlo, dhi)
  ModEntry ext[BLB_MAXM];
  double qhat_inv[BLB_MAXQ][BLB_MAXALPHA];        // [(Q_D/q_i)^-1]_{q_i}
  double qhat_mod[BLB_MAXQ][BLB_MAXALPHA][BLB_MAXM];  // [Q_D/q_i]_{m_e}
  double phat_inv[BLB_MAXSP];                     // [(P/p_t)^-1]_{p_t}
  double phat_mod[BLB_MAXSP][BLB_MAXQ];           // [P/p_t]_{q_i}
  double p_inv[BLB_MAXQ];                         // [P^-1]_{q_i}
};

// One key-switch output of a batch: source index (into the ModUp buffer), the source's c1
// (evaluation form, for the digit's own limbs), the switching key and the Galois element
// (0 = none).
struct KsOut {
  const uint64_t* c1;
  const uint64_t* key;
  uint32_t gal;
  int32_t src;
};

// Key-grouped inner product: ord lists output indices so that each group's outputs (first,
// count <= kKsGroupMax) share one switching key and Galois element.
constexpr int kKsGroupMax = 16;
constexpr int kKsMaxDigits = 4;
struct KsGroup {
  int first, count;
};

// matmul_cc launch records
struct CcPair {
  const uint64_t* x;
  const uint64_t* mx;
  const uint64_t* y;
  const uint64_t* my;
  uint64_t* out;
};
struct CcTerm {
  const uint64_t* ct;
  const uint64_t* mask;
};

// batched matmul_cp MAC
// Plaintexts of a ct-pt plan are held as 64-bit words (8N bytes per limb-poly) or, in the 50-bit
// format (every prime of the chain is below 2^50), as the words' low 32 bits (N x u32), the next
// 16 (N x u16) and the top 2 (N/16 x u32; word k at bits 2 (k mod 16) of u32 k / 16): 25N/4
// bytes.  The MAC streams either; 50-bit words are rebuilt into doubles in registers.
__host__ __device__ constexpr size_t pt50_bytes(int n) { return (size_t)n * 25 / 4; }
__host__ __device__ constexpr size_t pt_poly_bytes(int n, int p50) { return p50 ? pt50_bytes(n) : (size_t)n * 8; }

struct MacGroup {
  const uint64_t* pt;           // plan plaintexts [(b, j)][(a, i)][limb] limb-polys (pt_poly_bytes each)
  const uint64_t* const* rx;    // [instance][n_ai] rotated inputs ([2][nl][N] each)
  uint64_t* const* inner;       // [instance] -> [n_bj][2][nl][N]
  int n_ai, n_bj, nl, n_inst;
};
struct MacItem {
  int group, inst0, tile, kb, limb, n_limb;  // limbs limb .. limb + n_limb - 1 (limb grouping)
};

struct CpGeom {
  int d_in, d_out, L;
  int Lp, c, c_eff, c_out, n_in, n_out, B, G;
  // complex-slot output packing: output ciphertext b carries column blocks 2b (real parts) and
  // 2b + 1 (imaginary parts); n_out then counts output ciphertexts, ceil(blocks / 2)
  int cplx;
};

// Diagonal-packed input of the ct-pt product (the dense outputs of Softmax x V_h, head groups
// concatenated): input ciphertext a is the o-th output of a group of 2^logH heads starting at
// head h0 with c_g columns per ciphertext; its block u holds head h0 + (u mod 2^logH) and
// diagonal o c_g + floor(u / 2^logH) of that head.
struct CpDiagIn {
  int h0, logH, cg, o;
};
struct CpDiag {
  const CpDiagIn* tab;  // device, one entry per input ciphertext; null: spatial-first input
  int d_v, dvp, L;      // columns per head, 2^ceil(log2 d_v), rows
};

// ---------------------------------------------------------------------------------------
// Host-side structures
// ---------------------------------------------------------------------------------------
// Descriptor upload ring: pinned host staging + device mirror; a host region is reused only
// after the copy that last read it has completed.
// Pinned staging ring for descriptor tables, one per stream: host bytes are copied to the
// same offsets of a device ring on that stream, so a region's readers (kernels enqueued on the
// stream after its copy) always run before the copy that later overwrites it; the host only
// waits for the earlier copy of a region before rewriting its staging bytes.
struct UploadRegion {
  size_t lo, hi;
  hipEvent_t copied;
};
struct Uploader {
  hipStream_t stream = nullptr;
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0, head = 0;
  std::deque<UploadRegion> inflight;
  std::vector<hipEvent_t> free_events;
};

// Kernel timing spans recorded with HIP events on the context stream (when enabled).
struct TimedSpan {
  int kind;
  hipEvent_t a, b;
  double units;
};

// Recording state of a graph executor: while set on a context, temporaries come from the
// executor's arena, descriptor tables go to its blob, timing spans are off, and the mask
// seed is read from its parameter block.
// A fixed device region that temporaries are carved from, stack-like, instead of the stream
// stacks (the allocation-free entry points)
struct FixedArena {
  char* base;
  size_t cap, off;
  bool overflow;
};

struct ExecRec {
  char* arena = nullptr;
  size_t arena_cap = 0, arena_off = 0;
  char* blob_dev = nullptr;
  size_t blob_cap = 0;
  std::vector<char> blob_host;
  uint64_t* param = nullptr;  // device: [0] = mask seed
  bool overflow = false;
};

// Per-stream stack of temporaries.  Temporaries are scoped (released in reverse order of
// creation), so each stream's are carved from one device buffer like a stack; bytes released
// by a call are reused by the next call on the same stream in stream order, and eager calls
// never reach the allocator in steady state.  A temporary that does not fit comes from the
// stream-ordered pool; `need` records the deepest stack seen (counting those), and the buffer
// grows to it the next time the stack is empty.
struct Workspace {
  hipStream_t stream = nullptr;
  char* base = nullptr;
  size_t cap = 0;
  size_t off = 0;   // top of the stack
  size_t virt = 0;  // top counting the temporaries that did not fit
  size_t need = 0;  // deepest virt seen
  bool frozen = false;  // growing failed: stay at the current size
};

struct blb_ctx {
  int log_n, n, n_q, n_sp, dnum, alpha;
  ExecRec* rec = nullptr;
  FixedArena* fixed = nullptr;     // set only inside an allocation-free entry point
  std::vector<Workspace*> stacks;  // stacks of temporaries by stream
  bool timing = false;
  std::vector<TimedSpan> spans;
  std::vector<hipEvent_t> ev_pool;
  int device;
  hipStream_t stream;
  uint64_t budget;
  uint64_t dev_bytes = 0;
  uint64_t mod[BLB_MAXM];
  ModTable mt;
  uint64_t* d_mods = nullptr;
  double* d_tw_fwd = nullptr;
  double* d_tw_inv = nullptr;
  double* d_enc_tw = nullptr;     // [N/4][4] eta^k (dd complex), eta = exp(2 pi i / (N/2))
  double* d_enc_twist = nullptr;  // [N/2][4] zeta^-k (dd complex)
  int32_t* d_slot_inv = nullptr;  // DFT position u -> slot j with (5^j mod 2N - 1) / 4 = u
  KsLevelConst* d_kc[BLB_MAXQ] = {};
  KsLevelConst h_kc[BLB_MAXQ];
  char* scratch = nullptr;
  size_t scratch_cap = 0;
  std::vector<Uploader*> ups;      // upload rings by stream
  int* d_flag = nullptr;          // device error flag (encoder overflow)
  int mac_variant = 0;            // k_cp_mac tile shape (autotuned; never changes results)
  int batch_variant = 0;          // k_cp_mac_batch shape (autotuned)
  int batch_grid = 2048;          // persistent grid size of k_cp_mac_batch (autotuned)
  int batch_limbs = 1;            // limbs per work item of k_cp_mac_batch, 0 = all (autotuned)
  int plan_p50 = 0;               // new ct-pt plans in the 50-bit format (else 64-bit words)
  int ntt_variant = 1;            // 0: one workgroup per poly, 1: persistent pipelined (autotuned)
  int ntt_radix = 16;             // values per work-item: 16 (4-stage passes) or 32 (5-stage passes) (autotuned)
  int ks_variant = 1;             // key inner product: 0 per output, 1 grouped by key where the launch
                                  // stays wide, 2 always grouped (autotuned)
  int n_cu = 256;                 // compute units of the device
  int64_t counters[8] = {};       // operation counters (see blb_ctx_counters)
};

// Switching key in evaluation form: [digit][2 (b, a)][modulus (all q's then p's)][N] residues
struct SwKey {
  uint64_t id;  // 0 = relinearisation, else Galois element
  uint64_t* data;
};

struct blb_keys {
  blb_ctx* ctx;
  uint64_t seed;
  uint64_t* s_ntt;  // secret in evaluation form for all moduli [modulus][N]
  uint64_t* pk = nullptr;  // public key (-a s + e, a), evaluation form [2][n_q][N]
  std::vector<SwKey> keys;
  size_t bytes;
};

// matmul_cc geometry of one head group
struct CcGroup {
  int H;      // heads in the group
  int c;      // columns (of d) per ciphertext
  int n_ct;   // ciphertexts per operand
  int n_out;  // output ciphertexts: L'/c diagonal-packed, or d_v'/c dense (Softmax x V_h)
  int n_diag; // diagonal ciphertexts the schedule accumulates (L'/c); n_out divides it
  int ct0;    // first operand ciphertext of the group
  int out0;   // first output ciphertext of the group
  uint64_t* m_ge;  // [c][nl3][N] masks M^{>=tau} at level-2, scale q_{level-2}
  uint64_t* m_lt;  // [c][nl3][N] masks M^{<tau}
  uint64_t* m_s1;  // step 1 on the server: [2c][level+1][N] masks M^0, M^1_kappa (index kappa),
                   // M^2_kappa (index c + kappa) at the input level, scale q_level / 2^10;
                   // BSGS schedule: [2 (family)][g1][b1][level+1][N], pre-rotated per giant step
  uint64_t* m_bs;  // BSGS schedule: [G-1 (j >= 1)][4 (side, half)][c (tau)][nl3][N] step-3 product masks
                   // M^{>=tau} H_j, M^{>=tau} Lo_j, M^{<tau} H_j, M^{<tau} Lo_j at level-2, scale q_{level-2} / 2^10
  int b1, g1;      // BSGS split of step 1 (b1 g1 = c)
};

struct blb_plan {
  blb_ctx* ctx;
  int kind;  // 1 = matmul_cp, 2 = matmul_cc
  int level;  // input level
  int hom1 = 0;  // matmul_cc: step 1 (row pre-rotation of B) runs on the server
  CpGeom g;
  bool owns_pt = true;  // false: pt lives in caller memory (the serving plan arena)
  int p50 = 0;           // matmul_cp: plaintexts in the 50-bit format
  uint64_t* pt;  // matmul_cp: [(b, j)][(a, i)][limb][N] evaluation-form plaintexts
                 // matmul_cc: [2][T][limb][N] step-2 masks M^lo_t, M^hi_t (level, scale q_level 2^10),
                 // T = L' (plain schedule) or B (BSGS: baby steps only)
  size_t bytes;
  // matmul_cc
  int heads, L, d, Lp, n_ct, n_out;
  int sched = 0;        // 0: an inner rotation of every B'_a per t; 1: BSGS (giant steps postponed into step 3)
  int bs_B = 0, bs_G = 0;  // BSGS split of step 2 (B G = L')
  uint64_t* pt_a = nullptr;  // BSGS: [2][G][limb][N] masks of the giant inner rotations of A (t = L' - jB),
                             // level, scale q_level / 2^10 (j = 0 unused)
  std::vector<CcGroup> groups;
  std::vector<void*> extra;
  std::vector<size_t> extra_bytes;
};

// ---------------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------------
struct PolyDesc;
void launch_sample_uniform(blb_ctx* c, uint64_t* out, int n_limbs, ModMap map, uint64_t seed, uint32_t obj, uint32_t tag);
void launch_sample_int(blb_ctx* c, uint64_t* out, int n_limbs, ModMap map, uint64_t seed, uint32_t obj, uint32_t tag, bool gaussian);
int cp_check_keys(const blb_ctx* c, const blb_keys* K, int L, int d_in, int d_out);
void uploader_forget_stream(blb_ctx* c, hipStream_t s);
void stack_forget_stream(blb_ctx* c, hipStream_t s);
size_t cp_plan_bytes(const blb_ctx* c, int L, int d_in, int d_out, int level, int cplx = 0, int p50 = 0);
// p50: plaintext format (0: 64-bit words, 1: 50-bit, -1: the context's BLB_KNOB_PLAN_FORMAT)
int cp_plan_create(blb_ctx* c, const double* W, int d_in, int d_out, int L, int level, uint64_t* mem, blb_plan** out, int* flag_host,
                   const double* W_dev, int diag_heads = 0, int diag_dv = 0, int cplx = 0, int p50 = -1);
void launch_sample_flood(blb_ctx* c, uint64_t* out, int n_limbs, ModMap map, uint64_t seed, uint32_t obj, uint32_t tag, int bits);
void upload_cdt(const uint64_t* table20);

enum EwOp { EW_ADD = 0, EW_SUB = 1, EW_MUL = 2, EW_NEG = 3, EW_COPY = 4, EW_MULADD = 5 };
void launch_ew(blb_ctx* c, int op, uint64_t* out, const uint64_t* a, const uint64_t* b, const uint64_t* cc, int count, ModMap map);
struct LimbVals {
  int use;
  double v[BLB_MAXM];  // per-limb multiplier of the `extra` term
};
void launch_rlwe_combine(blb_ctx* c, uint64_t* out0, const uint64_t* a, const uint64_t* s, const uint64_t* e, const uint64_t* extra,
                         LimbVals extra_mul, int n_limbs, ModMap map);
void launch_automorph(blb_ctx* c, uint64_t* out, const uint64_t* in, int count, uint32_t g);
void launch_modup(blb_ctx* c, const uint64_t* dcoef, uint64_t* X, const KsLevelConst* kc_dev, int n_src, int nl, int n_ext, int n_digits);
void launch_ks_inner(blb_ctx* c, const KsOut* outs_dev, int n_out, const uint64_t* X, const KsLevelConst* kc_dev, uint64_t* U, int nl,
                     int n_ext, int n_digits);
void launch_ks_inner_grouped(blb_ctx* c, const KsOut* outs_dev, const int* ord_dev, const KsGroup* groups_dev, int n_groups,
                             const uint64_t* X, const KsLevelConst* kc_dev, uint64_t* U, int nl, int n_ext, int n_digits);
void launch_moddown_conv(blb_ctx* c, const uint64_t* U, uint64_t* Corr, const KsLevelConst* kc_dev, int n_out, int nl, int n_ext);
void launch_cp_mac(blb_ctx* c, const uint64_t* pt, const uint64_t* const* rx_tab, uint64_t* inner, int nl, int n_ai, int n_bj, int variant,
                   int p50);
void launch_sum_cts(blb_ctx* c, const uint64_t* const* srcs, uint64_t* const* dsts, int n_out, int n_terms, int nl);
void launch_mask_pair(blb_ctx* c, const CcPair* pairs_dev, int n_pairs, int nl);
int batch_mac_shape(int variant, int* tb, int* ib, int* cpt);
void launch_cp_mac_batch(blb_ctx* c, const MacGroup* groups, const MacItem* items, int n_items, int variant, int grid, int p50);
// forward NTT of count limb-polys stored back to back at base ([item][nl][N]); the results go
// to out in the 50-bit plan format (base is left as it was)
void launch_ntt_pack50(blb_ctx* c, const uint64_t* base, uint8_t* out, int count, int nl);
void launch_sum_var(blb_ctx* c, const uint64_t* const* srcs, const int* off, uint64_t* const* dsts, int n_out, int nl);
// out[t] ([2][nl][N]) = k * (the first nl limbs of each poly of in[t], stored with nl_in >= nl limbs)
void launch_scale_cts(blb_ctx* c, const uint64_t* const* in, uint64_t* out, int count, int nl, double k, int nl_in = 0);

// Noise boost: operands of key-switched rotations inside the matmuls are multiplied by this
// integer first (key-switch noise is absolute, so it shrinks relative to the message); the
// plaintext factors that follow are encoded at scales divided by it.
#define BLB_NOISE_BOOST 1024.0
// a_per_t: A_tab holds one operand per (t, a) ([n_t][n_ct]) instead of one per a
void launch_tensor_sum(blb_ctx* c, const uint64_t* const* A_tab, const uint64_t* const* R_tab, uint64_t* T3, int n_t, int n_ct, int nlA,
                       int nl2, bool a_per_t = false);
void launch_masked_acc(blb_ctx* c, const CcTerm* terms, const int* off, uint64_t* const* outs, int n_out, int nl, bool accumulate);
void launch_mask_sample(blb_ctx* c, uint64_t* r_out, uint64_t* share, int n_ct, int tl, uint64_t seed, const uint64_t* seed_dev, uint32_t tag);
void launch_set_u64(blb_ctx* c, uint64_t* dst, uint64_t value);
void launch_zero(blb_ctx* c, uint64_t* dst, size_t words);
// paired: the buffers hold (count + 1) / 2 complex vectors, each packing two real inputs
int run_encode_dense(blb_ctx* c, const double* vals, int n_vals, int count, double* bufA, double* bufB, double scale, int nl, uint64_t* out,
                     int* d_overflow);
int run_encode_cp(blb_ctx* c, const double* W, CpGeom g, int p0, int count, double* bufA, double* bufB, double scale, int nl, uint64_t* out,
                  int* d_overflow, CpDiag dg = CpDiag{nullptr, 0, 0, 0});
