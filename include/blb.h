/*
 * blb.h -- C ABI of the MI355X (gfx950) engine for the server-side RNS-CKKS path of
 * "Breaking the Layer Barrier" (BLB, arXiv 2508.19525): ciphertext-plaintext matmul
 * (matmul_cp), multi-head ciphertext-ciphertext matmul (matmul_cc), rescale, and the
 * CKKS-to-MPC mask-and-share step.
 *
 * Conventions for every call:
 *   - Return value: BLB_OK (0) or a negative BLB_E* code.  On error no output buffer has been
 *     written (arguments are validated before any work is enqueued).  blb_status_str() names
 *     a code.  No C++ exception crosses this boundary.
 *   - Ordering: work is enqueued on the context's HIP stream in call order.  Calls whose
 *     outputs are host buffers (blb_export, blb_decode, blb_ctx_moduli...) synchronise that
 *     stream before returning.
 *   - Ownership: blb_ctx, blb_keys and blb_plan are library-owned and released with their
 *     *_destroy call.  Ciphertext and plaintext buffers (blb_ct.data, pt_dev, share_dev) are
 *     caller-owned DEVICE memory, borrowed for the duration of the enqueued work.
 *   - Ring: Z[X]/(X^N + 1), N = 2^log_n; RNS chain q_0..q_{n_q-1} (50-bit primes, q = 1 mod 2N,
 *     the largest such primes below 2^50 taken in decreasing order) followed by n_special
 *     special primes p_0..p_{K-1} used only inside key switching.
 *   - A ciphertext at level l has l+1 active limbs q_0..q_l.  Its device layout is
 *     [degree+1][l+1][N] uint64 residues in [0, q_i), in the library's evaluation (NTT) form;
 *     blb_export / blb_import convert from / to the canonical coefficient form.
 *   - Plaintexts at the boundary (pt_dev) are coefficient-form residues [l+1][N] uint64.
 */
#ifndef BLB_H
#define BLB_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BLB_OK = 0,
  BLB_EINVAL = -1,  /* malformed argument (null pointer, size, shape) */
  BLB_ELEVEL = -2,  /* not enough limbs left for the operation, or level mismatch */
  BLB_ESCALE = -3,  /* operand scales disagree beyond 2^-30 relative */
  BLB_ENOKEY = -4,  /* a needed Galois / relinearisation key was not generated */
  BLB_ENOMEM = -5,  /* device allocation failed or HBM budget exceeded */
  BLB_EDEVICE = -6, /* HIP runtime error */
  BLB_EBUSY = -7,   /* serving queue full */
  BLB_ETOOBIG = -8  /* operand needs more than the fixed scratch of an allocation-free entry point */
};

typedef struct blb_ctx blb_ctx;
typedef struct blb_keys blb_keys;
typedef struct blb_plan blb_plan;

/* A ciphertext (Preliminaries, "CKKS Plaintext and Ciphertext": a pair of ring elements).
 * data: caller-owned device buffer of (degree+1)*(level+1)*N uint64 words. */
typedef struct {
  uint64_t* data;
  int32_t level;  /* active limbs = level + 1 */
  int32_t degree; /* 1: (c0, c1); 2: (d0, d1, d2) after a tensor product */
  double scale;   /* Delta of the encoded message */
} blb_ct;

typedef struct {
  int32_t log_n;             /* 12..14 (N = 4096 .. 16384; EINVAL otherwise) */
  int32_t n_q;               /* ciphertext primes, 1..12 */
  int32_t n_special;         /* key-switching primes K, 1..4 */
  int32_t dnum;              /* number of key-switching digits, 1..n_q */
  int32_t device;            /* HIP device ordinal */
  void* stream;              /* hipStream_t, NULL = the null stream */
  uint64_t hbm_budget_bytes; /* cap on library-owned device memory (keys, plans, scratch); 0 = none */
} blb_params;

/* ---- context ------------------------------------------------------------------------- */
int blb_ctx_create(const blb_params* params, blb_ctx** out);
void blb_ctx_destroy(blb_ctx* ctx);
/* out: n_q + n_special moduli (q's then p's); synchronises nothing. */
int blb_ctx_moduli(const blb_ctx* ctx, uint64_t* out);
/* Library-owned device bytes currently allocated (keys, plans, scratch). */
uint64_t blb_ctx_device_bytes(const blb_ctx* ctx);
/* Synchronises the stream and returns cached temporary memory of the eager path to the device. */
int blb_ctx_trim(blb_ctx* ctx);
const char* blb_status_str(int code);

/* ---- kernel timing (HIP events on the context stream) ----------------------------------
 * When enabled, every launch of the listed kernel families is bracketed by HIP events.
 * blb_ctx_read_timing synchronises the stream and returns, for one family, the summed
 * elapsed milliseconds, the number of launches and the summed work units (polynomials for
 * the NTT family, output ciphertext-limbs x coefficients for the others). */
enum { BLB_T_CP_MAC = 0, BLB_T_NTT = 1, BLB_T_KS_INNER = 2, BLB_T_MODUP = 3, BLB_T_MODDOWN = 4, BLB_T_MASK = 5,
       BLB_T_EW = 6, BLB_T_CC_TENSOR = 7, BLB_T_KINDS = 8 };
int blb_ctx_set_timing(blb_ctx* ctx, int enable);
int blb_ctx_read_timing(blb_ctx* ctx, int kind, double* total_ms, int64_t* launches, double* units);
int blb_ctx_reset_timing(blb_ctx* ctx);

/* ---- operation counters (counted when work is enqueued) ---------------------------------
 * out[8]: key switches, NTT / inverse-NTT limb-polys, ct-pt products (one plaintext times one
 * ciphertext), ct-ct tensor products, relinearisations, rescaled ciphertexts, ModUp sources,
 * plaintext bytes streamed by the matmul_cp MAC.  reset != 0 zeroes them after reading. */
int blb_ctx_counters(blb_ctx* ctx, int64_t* out, int reset);

/* ---- launch-shape knobs (never change a result bit; chosen by the autotuner) ------------ */
enum { BLB_KNOB_MAC_VARIANT = 0, BLB_KNOB_BATCH_VARIANT = 1, BLB_KNOB_BATCH_GRID = 2, BLB_KNOB_NTT_VARIANT = 3, BLB_KNOB_KS_VARIANT = 4,
       BLB_KNOB_NTT_RADIX = 5, BLB_KNOB_BATCH_LIMBS = 6, BLB_KNOB_PLAN_FORMAT = 7, BLB_KNOB_KINDS = 8 };
/* value ranges: MAC variant 0..BLB_MAC_VARIANTS-1 (outputs per block x coefficients per thread x
 * input-loop unroll x full-tile split), batch variant 0..BLB_BATCH_VARIANTS-1 (outputs x instances x
 * coefficients per thread), batch grid 1..2^20 workgroups, NTT variant 0..1 (one workgroup per
 * limb-poly, or a persistent grid prefetching the next one), NTT radix 16 or 32 (values per
 * work-item: passes of 4 or 5 radix-2 stages, N/16 or N/32 work-items per limb-poly), batched-MAC
 * limb grouping 0..12 (RNS limbs per work item of the instance-batched MAC; 0 = all limbs), key
 * inner-product variant 0..2 (0: one key-switch output per thread; 1: the outputs of a batch that
 * share a key and Galois element, up to 16 per thread, which reads each key word once for all of
 * them, where the launch keeps about 8192 workgroups busy that way (else one output per thread);
 * 2: always grouped), plan format 0..1 (how matmul_cp plans made afterwards hold their
 * plaintexts, the same values either way: 0, the default, as 64-bit words, 8N bytes per
 * limb-poly; 1, every prime being below 2^50, as 50-bit words in three planes, the low 32 bits,
 * the next 16 and the top 2, 25N/4 bytes per limb-poly: 22% less plan memory and MAC traffic for
 * some decoding work in the MAC.  A server takes the value the context has when it is created;
 * one blb_batch_matmul_cp call takes plans of one format, EINVAL otherwise) */
enum { BLB_MAC_VARIANTS = 18, BLB_BATCH_VARIANTS = 9 };
int blb_ctx_set_knob(blb_ctx* ctx, int knob, int value);
int blb_ctx_get_knob(const blb_ctx* ctx, int knob);

/* ---- keys (Preliminaries, "Rotation"; hybrid key switching as the reading of the library
 * the paper builds on) ------------------------------------------------------------------- */
/* Ternary secret from `seed`; relinearisation key (target s^2); one Galois key per entry of
 * rot_steps (left rotation by that many slots; negative = right).  Keys live on the device. */
int blb_keygen(blb_ctx* ctx, uint64_t seed, const int32_t* rot_steps, int n_rot, blb_keys** out);
void blb_keys_destroy(blb_keys* keys);
/* Galois element 5^steps mod 2N of a left rotation by `steps` slots. */
uint64_t blb_galois_elt(const blb_ctx* ctx, int32_t steps);

/* ---- encode / encrypt / decrypt / decode (eq. ckks_encode; real slots, complex on decode) - */
/* v: host array of n <= N/2 reals (missing slots are 0); writes round-half-away(Delta *
 * pi^-1(v)) reduced into limbs 0..level of pt_dev (coefficient form, [level+1][N]). */
int blb_encode(blb_ctx* ctx, const double* v, int64_t n, double scale, int level, uint64_t* pt_dev);
/* Secret-key encryption (-a s + e + pt, a); a and e drawn from Philox4x32-10 keyed by seed,
 * object id ct_id.  out->data must hold 2*(level+1)*N words. */
int blb_encrypt(blb_ctx* ctx, const blb_keys* keys, const uint64_t* pt_dev, int level, double scale,
                uint64_t seed, uint32_t ct_id, blb_ct* out);
/* pt_dev <- c0 + c1 s (+ c2 s^2), coefficient form [level+1][N]. */
int blb_decrypt(blb_ctx* ctx, const blb_keys* keys, const blb_ct* ct, uint64_t* pt_dev);
/* v (host, n values) <- Delta^-1 * pi(centred CRT lift of pt_dev).  Synchronises. */
int blb_decode(blb_ctx* ctx, const uint64_t* pt_dev, int level, double scale, double* v, int64_t n);
/* Complex slots: v_re, v_im (host, n values each) <- real and imaginary parts of
 * Delta^-1 * pi(centred CRT lift of pt_dev).  EINVAL as blb_decode or when v_im is null. */
int blb_decode_cplx(blb_ctx* ctx, const uint64_t* pt_dev, int level, double scale, double* v_re, double* v_im, int64_t n);
/* Canonical coefficient-form words of a ciphertext to / from host memory ([degree+1][level+1][N]). */
int blb_export(blb_ctx* ctx, const blb_ct* ct, uint64_t* host_words);
int blb_import(blb_ctx* ctx, const uint64_t* host_words, blb_ct* ct);

/* ---- homomorphic operations ------------------------------------------------------------ */
/* Left rotation by `steps` slots (Preliminaries, "Rotation"): sigma_{5^steps} and a hybrid
 * key switch with the automorphism applied after ModUp. in/out may not alias. */
int blb_rotate(blb_ctx* ctx, const blb_keys* keys, const blb_ct* in, int32_t steps, blb_ct* out);
/* blb_rotate for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same result, word for word, with
 * every temporary of the key switch carved from one fixed 8 MiB array per device that the
 * library holds until the process ends (its device address is looked up once per device when
 * a context is created).  Allocates nothing: no hipMalloc / hipFree, no pool, no events.
 * Needs 8 N (nl + n_digits n_ext + 2 n_ext + 2 nl) + 1024 bytes at the input's level (nl = level + 1
 * limbs, n_ext = nl + special primes); larger inputs return BLB_ETOOBIG with the output
 * untouched (e.g. N = 16384 with 4 primes + 2 special fits at every level; 10 primes + 2 special
 * at dnum 5 does not at the top level).  Every call on one GPU shares that GPU's array, so calls
 * that overlap on one GPU (other streams, other contexts, other threads) race; not callable
 * while a graph executor is being recorded on the context (BLB_EINVAL). */
int blb_rotate_noalloc(blb_ctx* ctx, const blb_keys* keys, const blb_ct* in, int32_t steps, blb_ct* out);
/* Rescale (Preliminaries, "Rescaling"): divide by the last prime q_l with rounding.
 * out->data must hold (degree+1)*level*N words; out gets level-1 and scale/q_l. */
int blb_rescale(blb_ctx* ctx, const blb_ct* in, blb_ct* out);
/* Batched negacyclic NTT over R_q = Z_q[X]/(X^N + 1) (Preliminaries, the ring of CKKS
 * polynomials), in place on caller-owned device words laid out [n_polys][n_limbs][N]; limb i
 * of every poly is reduced modulo prime i of the chain (the n_q ciphertext primes, then the
 * special primes), 1 <= n_limbs <= n_q + n_special.  Inputs must be canonical residues in
 * [0, q_i); outputs are canonical.  Forward (inverse = 0): word j of the output is
 * sum_k a_k psi^((2 brv(j) + 1) k) mod q_i, brv = bit reversal over log2 N bits, psi =
 * x^((q_i - 1) / 2N) for the smallest integer x >= 2 whose result has psi^N = -1 (the order
 * every ciphertext of this library is held in).  Inverse (inverse = 1) undoes it exactly.
 * Stream-ordered; EINVAL on bad sizes or a null pointer with n_polys > 0. */
int blb_ntt(blb_ctx* ctx, uint64_t* data, int64_t n_polys, int32_t n_limbs, int32_t inverse);

/* ---- matmul_cp (Section "Efficient Protocol for Fused MatMuls"; Appendix "BSGS
 * Optimization"; spatial-first packing of "Consistent Packing for Single Operator") ----- */
/* Builds the BSGS diagonal plaintexts of W (host, d_in x d_out row-major) for inputs of L rows
 * at ciphertext level `level`: encoded on the device at scale q_level / 2^10 and kept resident
 * (the inputs are multiplied by the integer 2^10 before their key-switched rotations, which
 * shrinks the key-switch noise relative to the message; the product scale is Delta_X q_level).
 * info (optional, 8 ints): L', c, c_eff, c_out, n_in, n_out, B, G. */
int blb_plan_matmul_cp(blb_ctx* ctx, const double* W, int d_in, int d_out, int L, int level, blb_plan** out);
void blb_plan_destroy(blb_plan* plan);
int blb_plan_info(const blb_plan* plan, int32_t* info8);
/* Y_b = Rescale( sum_j Rot^{jBL'}( sum_a sum_i pt_{a,b,j,i} (.) Rot^{iL'}(X_a) ) ), b < n_out.
 * X: n_in ciphertexts at the plan's level; Y: n_out buffers of 2*level*N words. */
int blb_matmul_cp(blb_ctx* ctx, const blb_keys* keys, const blb_plan* plan, const blb_ct* X, int n_in,
                  blb_ct* Y, int n_out);
/* Complex-slot output packing (the encoding's slots are complex; "CKKS Approximate HE and
 * Message Encoding" keeps only their real parts).  The same schedule with the plaintexts of
 * output blocks 2b and 2b + 1 joined into one, d_{a,2b,t} + i d_{a,2b+1,t}: output ciphertext b
 * decodes to Y_{2b} + i Y_{2b+1} (real parts block 2b, imaginary parts block 2b + 1; an odd block
 * count leaves the last imaginary part 0).  Plaintexts, their MAC bytes, giant-step rotations,
 * rescales and output ciphertexts halve; the baby steps stay.  blb_plan_info's n_out is the
 * number of output ciphertexts, ceil(blocks / 2); run the plan with blb_matmul_cp (or its
 * executors and the instance-batched call).  Decode with blb_decode_cplx.  Arguments and errors
 * as blb_plan_matmul_cp. */
int blb_plan_matmul_cp_cplx(blb_ctx* ctx, const double* W, int d_in, int d_out, int L, int level, blb_plan** out);

/* ---- matmul_cc (Section "Efficient Protocol for Fused MatMuls": observations 1-2, the three
 * steps and the Multi-Head Optimization; output in diagonal packing) ---------------------
 * Heads are split into power-of-two groups, largest first (12 = 8 + 4).  For a group of H heads
 * with L' = 2^ceil(log2 L) and c = (N/2) / (L' H) columns per ciphertext, operand ciphertext a
 * of the group holds at slot i + L'(h + H kappa):
 *     A:  A_h{i, a c + kappa}                      (Q_h, spatial-first per head)
 *     B': B_h{a c + kappa, (i + kappa) mod L'}      (K_h^T rows, reduce-first, step 1 applied by
 *                                                   the client before encryption), or
 *     B:  B_h{a c + kappa, i}                       (no pre-rotation: step 1 runs on the server)
 * and output ciphertext g (g < L'/c) of the group holds C_h{i, (i + g c + kappa) mod L'}.
 * Operands are at the plan's level; outputs come out 3 levels lower (level >= 3) with B', or
 * 4 levels lower (level >= 4) with B.
 * Rotations per group: step 1 (server side only) 2 (c-1) per B ciphertext (hoisted); step 2
 * 2 (L'-1) per B' ciphertext (hoisted); step 3 L' - L'/c.  Step 1 needs no keys beyond step 2's. */
/* Rotation steps the keys must cover (left t, right L'-t, right tau H L'); returns the count
 * written to steps (or needed, when steps is NULL). */
int blb_cc_rotations(const blb_ctx* ctx, int n_heads, int L, int32_t* steps, int cap);
/* Masks encoded on the device.  b_prerotated = 1: step-2 masks at scale q_level 2^10, step-3
 * masks at q_{level-2} / 2^10.  b_prerotated = 0: step-1 masks at q_level / 2^10 (M^0: blocks of
 * class kappa = 0; M^1_kappa: class kappa, i < L' - kappa; M^2_kappa: class kappa, i >= L' - kappa),
 * then steps 2-3 as above one level lower.  Before each batch of key-switched rotations the
 * rotated ciphertext is multiplied by the integer 2^10, so the key-switch noise shrinks
 * relative to the message; the mask scales undo the factor. */
int blb_plan_matmul_cc(blb_ctx* ctx, int n_heads, int L, int d_head, int level, int32_t b_prerotated, blb_plan** out);
/* info: L', n_ct, n_out, then per group (H, c, n_ct, n_out, first ct); returns group count. */
int blb_plan_cc_info(const blb_plan* plan, int32_t* info, int cap);
/* C_g for every group; n_ct operands each (groups concatenated), n_out outputs, each of
 * 2 (level - 2) N words (B pre-rotated) or 2 (level - 3) N words (step 1 on the server). */
int blb_matmul_cc(blb_ctx* ctx, const blb_keys* keys, const blb_plan* plan, const blb_ct* A, const blb_ct* Bp, int n_ct,
                  blb_ct* C_diag, int n_out);

/* ---- matmul_cc with BSGS (Appendix "BSGS Optimization", figure bsgs) ------------------
 * The same operands, outputs, levels and output scale as blb_plan_matmul_cc / _sv, computed by
 * a second schedule (schedule = 1; schedule = 0 is the plain one above, and the two give
 * different words that decode to the same product).  With L' = B G (B = 2^ceil(log2(L')/2))
 * and t = j B + i, step 2 inner-rotates each B' ciphertext only by the baby steps i < B and each
 * A ciphertext by the giant steps (right by jB, masks at q_level / 2^10 after a 2^10 boost), and
 * the tensor of A'_{a,j} with Y_{a,i} is diagonal t rotated right by jB within its block.  Step 3
 * undoes that rotation once per output instead of once per ciphertext: each rotated U_t of giant
 * step j >= 1 is split with the product of its step-3 block mask and the half-block masks
 * (in-block position >= jB or < jB), the halves accumulate per (output, j) and are rotated left
 * by jB or right by L' - jB before joining the output.  Depth is unchanged.  Step 1 on the
 * server (b_prerotated = 0) uses c = b1 g1 (b1 = 2^ceil(log2(c)/2)): b1 - 1 hoisted baby
 * rotations shared by the left and right families, whose pre-rotated masks are summed per giant
 * step and rotated left by j b1 (g1 - 1) or right by L' - j b1 (g1).  Rotations per group:
 * 2 n_ct (B - 1) + 2 n_ct (G - 1) + (L' - L'/c) + 2 (number of (output, j >= 1) pairs that
 * receive a term) [+ n_ct (b1 + 2 g1 - 2) for step 1]; relinearisations L'. */
int blb_plan_matmul_cc_sched(blb_ctx* ctx, int n_heads, int L, int d_head, int level, int32_t b_prerotated, int32_t schedule,
                             blb_plan** out);
int blb_plan_matmul_cc_sv_sched(blb_ctx* ctx, int n_heads, int L, int d_v, int level, int32_t b_prerotated, int32_t schedule,
                                blb_plan** out);
/* Rotation steps of a schedule (as blb_cc_rotations, which is schedule 0); b_prerotated = 0 adds
 * the server-side step 1's steps. */
int blb_cc_rotations_sched(const blb_ctx* ctx, int n_heads, int L, int32_t b_prerotated, int32_t schedule, int32_t* steps, int cap);

/* ---- matmul_cp feeding matmul_cc (Multi-Head Optimization; Section "Efficient Fused
 * Computations in Multi-Head Attention": the columns of W_Q / W_K reordered in plaintext) --------
 * A matmul_cp plan for W (host, d_in x (n_heads d_head) row-major, head h owning columns
 * h d_head .. (h+1) d_head - 1) whose spatial-first outputs ARE the ct-ct operands in the multi-head
 * packing above (head groups concatenated): output b = operand ciphertext b holds, for its group
 * of H heads from h0 with c_g = (N/2) / (L' H), column a c_g + kappa of (X W)_{h0+h} at block
 * h + H kappa (a = b minus the group's first ciphertext; 0 past d_head).  Run it with blb_matmul_cp:
 * X W_Q' gives the A operand, X W_K' the B operand before step 1 (b_prerotated = 0).  The plan
 * has n_out = the ct-ct plan's n_ct and the cost of a plain matmul_cp with that many outputs.
 * EINVAL for a geometry the ct-ct packing cannot hold (c_g > L'). */
int blb_plan_matmul_cp_mhp(blb_ctx* ctx, const double* W, int d_in, int n_heads, int d_head, int L, int level, blb_plan** out);

/* ---- Softmax x V_h with zero padding (Section "Efficient Fused Computations in Multi-Head
 * Attention"; Appendix "Diagonal Ciphertext-Plaintext MatMul", figure diag (b)) -----------
 * The same protocol (run with blb_matmul_cc) with A_h = the L x L attention weights
 * (reduction dimension L: the packing above with d = L) and B_h = V_h, L x d_v, whose columns
 * from d_v to L' are zero (operand B': slot i + L'(h + H kappa) holds V_h{a c + kappa,
 * (i + kappa) mod L'}, 0 for columns >= d_v).  With d_v' = 2^ceil(log2 d_v), diagonals D and
 * D + d_v' of the padded product are complementary, so each group's L'/c diagonal ciphertexts
 * are accumulated mod d_v'/c before their final rescale: output o (o < d_v'/c) of a group holds
 * at slot i + L'(h + H kappa) the value Att_h{i, (i + o c + kappa) mod d_v'} (0 for columns >= d_v),
 * the dense diagonal packing that blb_plan_matmul_cp_diag takes.  Outputs per group: d_v'/c.
 * Requires d_v' <= L' and c <= d_v' for every group (EINVAL otherwise); keys as blb_cc_rotations.
 * blb_plan_cc_info reports n_out = d_v'/c per group. */
int blb_plan_matmul_cc_sv(blb_ctx* ctx, int n_heads, int L, int d_v, int level, int32_t b_prerotated, blb_plan** out);

/* ---- matmul_cp with diagonal-packed input (Appendix "Diagonal Ciphertext-Plaintext MatMul",
 * figure diag (c)) --------------------------------------------------------------------------
 * E = Concat_h(Att_h) W for W (host, (n_heads d_v) x d_out row-major) and inputs in the dense
 * diagonal packing of blb_plan_matmul_cc_sv (its outputs, head groups concatenated).  Output
 * spatial-first, as blb_matmul_cp: run the plan with blb_matmul_cp (or its executors).  The
 * BSGS schedule and geometry are those of a spatial-first input with n_heads d_v' columns
 * (blb_plan_info; c_eff = c = (N/2) / L'), with the diagonals
 *     d_{a,b,t}[u L' + r] = W{h d_v + (r + tau) mod d_v', b c + (u mod c_out)},
 * (h, tau) = head and diagonal held by block (u + t) mod c of input a, and 0 for r >= L or
 * (r + tau) mod d_v' >= d_v; encoded at q_level / 2^10 like blb_plan_matmul_cp.  EINVAL when the
 * head groups do not tile the input (the limits of blb_plan_matmul_cc_sv). */
int blb_plan_matmul_cp_diag(blb_ctx* ctx, const double* W, int n_heads, int d_v, int d_out, int L, int level, blb_plan** out);
/* The diagonal-input plan in the complex-slot output packing (see blb_plan_matmul_cp_cplx). */
int blb_plan_matmul_cp_diag_cplx(blb_ctx* ctx, const double* W, int n_heads, int d_v, int d_out, int L, int level,
                                 blb_plan** out);

/* ---- re-randomisation before mask-to-share (opt-in) -----------------------------------
 * Algorithm ckks2mpc hands the masked ciphertext to the client as evaluated; its c1 depends on
 * the server's weights, which the paper does not address.  This call adds a public-key
 * encryption of zero with a flooding term, in place, at each ciphertext's level:
 *     (c0 + v p0 + e0, c1 + v p1 + e1),  pk = (p0, p1) = (-a s + e, a) made by blb_keygen
 * (a uniform: tag 7, e Gaussian: tag 8, object 0, key seed), v ternary (tag 9), e1 Gaussian
 * (tag 11), e0 uniform in [-2^F, 2^F] (tag 10: the 128-bit Philox block mod 2^(F+1) + 1,
 * minus 2^F), object id = index t in cts, key `seed`.  F = flood_bits in [32, 48]; the decoded
 * value moves by about 2^F / scale.  EINVAL on bad arguments (nothing written). */
int blb_rerandomize(blb_ctx* ctx, const blb_keys* keys, blb_ct* cts, int n_ct, uint64_t seed, int flood_bits);

/* ---- CKKS-to-MPC mask-and-share (Algorithm ckks2mpc, step 1; functionality F_C2M) ------- */
/* For each ciphertext t < n_ct: reduce to target_level (dropping top limbs) if lower, sample
 * r uniform in R_{Q_target} (Philox, object id t), set c0 <- c0 + r in place and write the
 * server share -r mod q_i in coefficient form to share_dev[t][limb][N]. */
int blb_mask_to_share(blb_ctx* ctx, blb_ct* cts, int n_ct, uint64_t seed, int target_level, uint64_t* share_dev);

/* ---- MPC-to-CKKS, the server's step (Algorithm mpc2ckks: P_1 adds its share to the client's
 * encryption of the other share) ---------------------------------------------------------------
 * cts[t] = (c0 + share_t, c1) mod q_i in place, share_dev: device words [t][limb][N], the server's
 * ring share of the encoded message in coefficient form, one residue per limb in [0, q_i)
 * (canonical residues are the caller's contract: other words give unspecified, in-bounds results),
 * at the ciphertexts' common level (ELEVEL if the levels differ).  Applied to the output of
 * blb_mask_to_share with its share it restores the ciphertext word for word.  Stream-ordered. */
int blb_add_share(blb_ctx* ctx, blb_ct* cts, int n_ct, const uint64_t* share_dev);

/* ---- Rotate-and-sum summation and broadcast (Section "Consistent Packing for Single Operator":
 * the Expansion and Reduction operators) -------------------------------------------------------
 * Per ciphertext: m^0 = m, m^i = m^{i-1} + Rot^{2^{i-1} block}(m^{i-1}), i = 1 .. log2 n_blocks,
 * with left rotations (direction 0, summation) or right rotations (direction 1, broadcast);
 * n_blocks a power of two, block * n_blocks <= N/2.  Summation with mask = 1 then keeps the first
 * `block` slots (mask [1 x block, 0, ...] encoded at q_level, product rescaled: out at level - 1 with
 * the input scale); otherwise out = m^{log2 n_blocks} at the input level.  For a spatial-first
 * matrix (block = L', n_blocks columns per ciphertext) summation gives the row sums in the first
 * block; broadcast of a first-block vector replicates it over n_blocks blocks.  Keys: rotations
 * by +-2^i block (ENOKEY otherwise); inputs at one level and scale; out[t] buffers of the input
 * size, distinct from the inputs. */
int blb_rotate_sum(blb_ctx* ctx, const blb_keys* keys, const blb_ct* in, int n_ct, int block, int n_blocks, int direction, int mask,
                   blb_ct* out);

/* ---- Identity and Expansion operators (Table "opertors": ewadd / ewmul of ct-ct and ct-pt,
 * sadd / smul; Section "Consistent Packing for Single Operator": scalar operators by broadcast,
 * and a summation followed by a scalar operator with neither mask nor broadcast) ----------------
 * All take n_ct ciphertexts at one level (ELEVEL otherwise), degree 1, and write out[t] (buffers
 * of the input size; out may be the first operand) at the same level; nothing is rescaled:
 * products leave the product of the scales and the caller rescales with blb_rescale.
 *   blb_ew_add:       a + b (ESCALE unless the scales agree within 1e-9 relative)
 *   blb_ew_add_plain: (c0 + pt, c1), pt_dev [t][level+1][N] coefficient-form residues encoded at a's scale
 *   blb_ew_mul_plain: (c0 pt, c1 pt), pt_dev as above, encoded at pt_scale; out scale = a.scale pt_scale
 *   blb_ew_mul_relin: the tensor of a and b relinearised with the s^2 key (ENOKEY without it);
 *                     out scale = a.scale b.scale
 *   blb_scalar_op:    a (op 0: +, 1: x with relinearisation) the vector V made from s:
 *                     from_sum = 0: s holds the scalar column in its first `block` slots (zero
 *                     elsewhere) and V is its broadcast over n_blocks blocks (blb_rotate_sum,
 *                     direction 1: log2 n_blocks rotations);
 *                     from_sum = 1: s is the input of a summation over its n_blocks blocks, which
 *                     fill the ciphertext (block n_blocks = N/2, EINVAL otherwise), and V is the
 *                     unmasked left rotate-and-sum, which already holds the sum in every block
 *                     (log2 n_blocks rotations, no mask product, no level).
 *                     Keys as blb_rotate_sum (plus relinearisation for op 1). */
int blb_ew_add(blb_ctx* ctx, const blb_ct* a, const blb_ct* b, int n_ct, blb_ct* out);
int blb_ew_add_plain(blb_ctx* ctx, const blb_ct* a, int n_ct, const uint64_t* pt_dev, blb_ct* out);
int blb_ew_mul_plain(blb_ctx* ctx, const blb_ct* a, int n_ct, const uint64_t* pt_dev, double pt_scale, blb_ct* out);
int blb_ew_mul_relin(blb_ctx* ctx, const blb_keys* keys, const blb_ct* a, const blb_ct* b, int n_ct, blb_ct* out);
int blb_scalar_op(blb_ctx* ctx, const blb_keys* keys, const blb_ct* a, const blb_ct* s, int n_ct, int block, int n_blocks, int op,
                  int from_sum, blb_ct* out);

/* ---- batched matmul_cp over independent instances ------------------------------------
 * Each instance has its own keys (its client), plan (plans may be shared between instances
 * with the same weights and L'), inputs and outputs; all plans must be at one level.  Every
 * stage (baby-step key switches, plaintext MACs, giant-step key switches, sums, rescale) runs
 * once for the whole batch; the MACs of all instances are one persistent launch that applies
 * each plaintext word to several instances sharing its plan.  Results are bit-identical to
 * per-instance blb_matmul_cp calls. */
typedef struct {
  const blb_keys* keys;
  const blb_plan* plan;
  const blb_ct* X;
  int n_in;
  blb_ct* Y;
  int n_out;
} blb_cp_instance;
int blb_batch_matmul_cp(blb_ctx* ctx, const blb_cp_instance* inst, int n_inst);

/* ---- graph executors -------------------------------------------------------------------
 * One fused operator invocation over fixed ciphertext buffers (matmul_cp or matmul_cc,
 * optionally followed by mask-and-share of its outputs to mask_target_level; -1 = no mask)
 * recorded into a HIP graph.  Scratch and descriptor tables are owned by the executor, so a
 * replay issues a single graph launch on the context stream.  The mask seed is a replay
 * parameter (fresh masks per run).  The output blb_ct structs are updated (level, scale) at
 * creation.  Buffers and keys passed at creation must stay alive while the executor is used. */
typedef struct blb_exec blb_exec;
int blb_exec_create_cp(blb_ctx* ctx, const blb_keys* keys, const blb_plan* plan, const blb_ct* X, int n_in, blb_ct* Y, int n_out,
                       int mask_target_level, uint64_t* share_dev, blb_exec** out);
int blb_exec_create_cc(blb_ctx* ctx, const blb_keys* keys, const blb_plan* plan, const blb_ct* A, const blb_ct* Bp, int n_ct,
                       blb_ct* C_diag, int n_out, int mask_target_level, uint64_t* share_dev, blb_exec** out);
/* The whole batch in one graph launch; with a mask, all outputs (instance order) are masked as
 * one list, share_dev receiving [output][limb][N] for them in that order. */
int blb_exec_create_batch_cp(blb_ctx* ctx, const blb_cp_instance* inst, int n_inst, int mask_target_level, uint64_t* share_dev,
                             blb_exec** out);
int blb_exec_run(blb_exec* exec, uint64_t mask_seed);
/* The same replay on `stream` (a hipStream_t; null = the context stream).  Executors own their
 * scratch, so replays of different executors (with different output buffers) may run at once
 * on different streams and overlap on the device; replays of one executor must stay ordered
 * (one stream, or synchronised by the caller), since they share its scratch. */
int blb_exec_run_stream(blb_exec* exec, uint64_t mask_seed, void* stream);
uint64_t blb_exec_device_bytes(const blb_exec* exec);
void blb_exec_destroy(blb_exec* exec);

/* ---- serving: a request loop with HBM-budget admission and continuous batching ---------
 * A worker thread owns the context while the server exists (create keys and buffers before
 * creating it; afterwards use the context only through the server calls).  Weights are
 * registered once (host copy kept); the diagonal plaintexts of (weight, L') are generated on
 * the device when a request needs them and kept in a plan cache: one device allocation of
 * plan_cache_bytes made at creation (ENOMEM if it cannot be made), carved into plans first-fit,
 * evicting least-recently-used plans no running request uses until a contiguous range is free.  A request is admitted when its
 * plan is resident or fits; admitted requests join the next batch (one blb_batch_matmul_cp
 * plus per-request mask-and-share) launched on one of n_streams streams, so requests that
 * arrive while earlier batches run are admitted and overlap with them.  Latency is measured
 * from submission to completion (host clock).  A request whose plan can never fit is rejected
 * with BLB_ENOMEM; a full queue returns BLB_EBUSY at submission. */
typedef struct blb_server blb_server;
typedef struct {
  uint64_t plan_cache_bytes;
  int max_batch;  /* requests per batch */
  int max_queue;  /* queued (not yet admitted) requests */
  int n_streams;  /* batches in flight, 1..8 */
  int policy;     /* 0: admit in arrival order; 1: requests whose plan is resident first, then the
                   * oldest (its plan generated, then every queued request on the same plan); a
                   * request older than max_wait_ms goes first in any case */
  double max_wait_ms;
} blb_server_config;
int blb_server_create(blb_ctx* ctx, const blb_server_config* cfg, blb_server** out);
/* W: host d_in x d_out row-major (copied); inputs of requests on this weight are at `level`.
 * A weight id can be registered once (EINVAL on a second registration). */
int blb_server_add_weights(blb_server* server, int weight_id, const double* W, int d_in, int d_out, int level);
/* The same, with the complex-slot output packing of blb_plan_matmul_cp_cplx: a request on this
 * weight has ceil(blocks / 2) output ciphertexts, blocks = ceil(d_out / c), and its plans take
 * half the cache. */
int blb_server_add_weights_cplx(blb_server* server, int weight_id, const double* W, int d_in, int d_out, int level);
/* X (n_in cts) and Y (n_out buffers of 2*level*N words) must stay alive until completion; the
 * blb_ct array Y is updated (level, scale) by the worker.  mask_target_level < 0: no mask.
 * Refused at submission: EINVAL (shapes), ELEVEL (input level), ENOKEY (keys lack a rotation
 * of this request's schedule), EBUSY (queue full). */
int blb_server_submit(blb_server* server, const blb_keys* keys, int weight_id, int L, const blb_ct* X, int n_in, blb_ct* Y, int n_out,
                      uint64_t mask_seed, int mask_target_level, uint64_t* share_dev, int64_t* req_id);
/* state: 0 queued, 1 running, 2 done, < 0 the error code; latency_ms (done only, else -1). */
int blb_server_poll(blb_server* server, int64_t req_id, int* state, double* latency_ms);
/* waits until nothing is queued or running (BLB_EBUSY on timeout) */
int blb_server_drain(blb_server* server, double timeout_s);
/* out[cap >= 10]: completed, rejected, p50 ms, p99 ms, mean ms, plan hits (requests whose plan
 * was ready when first considered), plan misses (plans generated), batches, plan generation
 * seconds (enqueue to completion), resident plan bytes; out[10] (cap > 10): requests whose
 * batch failed at launch (their poll state holds the error code); out[11..15] (cap > 15):
 * plan generations deferred for lack of a free range in the plan cache, deferred for lack of
 * device memory for their temporaries, plan bytes generated, batch launches retried after
 * ENOMEM, seconds with queued requests and nothing on the GPU for them. */
int blb_server_stats(blb_server* server, double* out, int cap);
void blb_server_destroy(blb_server* server);

#ifdef __cplusplus
}
#endif
#endif /* BLB_H */
