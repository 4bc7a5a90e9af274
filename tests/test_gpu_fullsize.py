"""Full-size configurations on the GPU, through the same entry points the benchmark times.

- BERT-base fused linear op (N = 8192, three primes, X 128 x 768, W 768 x 768): the library's
  encryption of X equals the oracle's; on the oracle's input ciphertexts, sampled outputs of
  matmul_cp equal the oracle's word for word; all outputs decode to X W within 2^-20; the
  operation counters equal the schedule's closed forms (BSGS with B = 8, G = 4).
- 12-head attention Q_h K_h^T (N = 16384, four primes + two special): one sampled
  diagonal-packed output of each head group (8 + 4) equals the oracle's; every head decodes to
  Q_h K_h^T within 2^-20; tensor products = m^2 d / s (m = 128 tokens, d = 768, s = 8192
  slots), one relinearisation per inner rotation t.

The oracle computes only the sampled outputs (tens of seconds on the host)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def B():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_19525_amd as B
    B.lib()
    return B


def _ct(B, keep, n, level, degree=1):
    c, t = B.new_ct(n, level, degree)
    keep.append(t)
    return c


def _import(B, ctx, keep, words, n, level, scale):
    c = _ct(B, keep, n, level)
    B.blb_import(ctx, words, c)
    c.scale = scale
    return c


@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("cplx", [False, True])
def test_bert_base_matmul_cp_full_size(B, orc, cplx, fmt):
    """The headline operator at full size, real-slot or complex-slot output packing, plaintexts as
    64-bit words (fmt 0) or in the 50-bit format (fmt 1): inputs encrypted by the library equal the
    oracle's, counters equal the schedule's closed forms, sampled outputs equal the oracle's word
    for word, every output decodes to X W within 2^-20."""
    from paper_2508_19525_amd import workloads as wl
    cfg = wl.C2
    p = cfg["params"]
    L, d = cfg["L"], cfg["d_in"]
    n, level = p.n, p.n_q - 1
    X = wl.activations(2, L, d, cfg["x_dist"])
    W = wl.weights(2, d, cfg["d_out"], cfg["w_std"])
    o = orc.Context(p.log_n, p.n_q, p.n_special, p.dnum)
    keys_o = orc.Keys(o, 77, o.cp_galois(L, d, d))
    xw = np.stack([keys_o.encrypt(o.encode_rns(o.pack_spatial(X, a), p.scale, level), level, 78, a)
                   for a in range(o.cp_geometry(L, d, d)["n_in"])])
    ctx = B.blb_ctx_create(p.log_n, p.n_q, p.n_special, p.dnum, 0, torch.cuda.current_stream().cuda_stream)
    keep = []
    try:
        B.blb_ctx_set_knob(ctx, B.BLB_KNOB_PLAN_FORMAT, fmt)
        plan = (B.blb_plan_matmul_cp_cplx if cplx else B.blb_plan_matmul_cp)(ctx, W, L, level)
        g = B.blb_plan_info(plan)
        n_y = 12 if cplx else 24  # output ciphertexts
        assert (g["B"], g["G"], g["n_in"], g["n_out"]) == (8, 4, 24, n_y)
        steps = [k * g["Lp"] for k in range(1, g["B"])] + [j * g["B"] * g["Lp"] for j in range(1, g["G"])]
        keys = B.blb_keygen(ctx, 77, steps)
        # the library's own encode + encrypt of X equals the oracle's words
        pt = torch.empty((level + 1) * n, dtype=torch.int64, device="cuda")
        for a in (0, 11, 23):
            B.blb_encode(ctx, wl.pack_spatial(X, n // 2, a), p.scale, level, pt)
            ct = _ct(B, keep, n, level)
            B.blb_encrypt(ctx, keys, pt, level, p.scale, 78, a, ct)
            torch.cuda.synchronize()
            assert np.array_equal(B.blb_export(ctx, ct, n), xw[a]), f"input ciphertext {a}"
        xs = [_import(B, ctx, keep, xw[a], n, level, p.scale) for a in range(g["n_in"])]
        ys = [_ct(B, keep, n, level - 1) for _ in range(g["n_out"])]
        B.blb_ctx_counters(ctx, reset=True)
        B.blb_matmul_cp(ctx, keys, plan, xs, ys)
        cnt = B.blb_ctx_counters(ctx, reset=True)
        torch.cuda.synchronize()
        assert cnt["key_switches"] == 24 * 7 + n_y * 3  # 240 real, 204 complex
        assert cnt["ct_pt_products"] == 24 * n_y * 32  # 18432 real, 9216 complex
        assert cnt["modup_sources"] == 24 + n_y * 3
        assert cnt["rescaled_cts"] == n_y
        assert cnt["plaintext_bytes"] == 24 * n_y * 32 * 3 * (n * 25 // 4 if fmt else n * 8)
        samples = [0, 7] if cplx else [0, 17]
        want = keys_o.matmul_cp(xw, level, W, L, outputs=samples, cplx=cplx)
        for b in samples:
            assert np.array_equal(B.blb_export(ctx, ys[b], n), want[b]), f"output {b}"
        vecs = []
        dec = torch.empty(level * n, dtype=torch.int64, device="cuda")
        for b in range(g["n_out"]):
            B.blb_decrypt(ctx, keys, ys[b], dec)
            if cplx:
                vecs += list(B.blb_decode_cplx(ctx, dec, level - 1, ys[b].scale, n // 2))
            else:
                vecs.append(B.blb_decode(ctx, dec, level - 1, ys[b].scale, n // 2))
        got = wl.unpack_spatial(vecs, L, d, n // 2)
        assert np.abs(got - X @ W).max() < 2.0 ** -20
        B.blb_plan_destroy(plan)
        B.blb_keys_destroy(keys)
    finally:
        torch.cuda.synchronize()
        B.blb_ctx_destroy(ctx)


def _bsgs_counts(lp, groups):
    """Key switches and ct-pt (mask) products of the BSGS schedule with B' pre-rotated, counted
    from its definition: groups = [(c, n_ct, n_out)], B = 2^ceil(log2(L')/2), G = L'/B; baby inner
    rotations (i < B) of B', giant ones (0 < j < G) of A, a step-3 rotation per t with t mod c != 0,
    one postponed rotation per (output, j > 0, half) receiving a term, one relinearisation per t."""
    lb = (lp - 1).bit_length()
    Bb = 1 << ((lb + 1) // 2)
    G = lp // Bb
    ks, ptm = 0, 0
    for cc, m, n_out in groups:
        n_diag = lp // cc
        ks += 2 * m * (Bb - 1) + 2 * m * (G - 1) + sum(1 for t in range(lp) if t % cc) + lp
        ptm += m * (1 + 2 * (Bb - 1)) + 2 * m * (G - 1)
        for j in range(G):
            outs = set()
            for t in range(j * Bb, j * Bb + Bb):
                n_mask = 1 + (1 if t % cc else 0)
                ptm += n_mask * (1 if j == 0 else 2)
                outs.add((t // cc) % n_out)
                if t % cc:
                    outs.add(((t // cc + 1) % n_diag) % n_out)
            if j:
                ks += 2 * len(outs)
    return ks, ptm


@pytest.mark.parametrize("schedule", [0, 1])
def test_attention_matmul_cc_full_size(B, orc, schedule):
    """BERT-base Q_h K_h^T (12 heads of 128 tokens, d_head 64, N = 16384, four primes + two special)
    through the plain and the BSGS schedule: operation counters equal each schedule's closed form
    (BSGS: 1086 key switches instead of 3536), one sampled output per head group equals the
    oracle's word for word, and every head decodes to Q_h K_h^T within 2^-20."""
    from paper_2508_19525_amd import workloads as wl
    cfg = wl.C3
    p = cfg["params"]
    heads, L, d = cfg["heads"], cfg["L"], cfg["d_head"]
    n, level = p.n, p.n_q - 1
    rng = np.random.default_rng(wl.seed_for(3, wl.ROLE_X))
    Q = [rng.normal(0, 1, (L, d)) for _ in range(heads)]
    Kt = [rng.normal(0, 1, (L, d)).T.copy() for _ in range(heads)]
    o = orc.Context(p.log_n, p.n_q, p.n_special, p.dnum)
    ctx = B.blb_ctx_create(p.log_n, p.n_q, p.n_special, p.dnum, 0, torch.cuda.current_stream().cuda_stream)
    keep = []
    try:
        steps = B.blb_cc_rotations(ctx, heads, L, schedule)
        keys_o = orc.Keys(o, 79, sorted({o.galois_elt(s) for s in steps}))
        keys = B.blb_keygen(ctx, 79, steps)
        plan = B.blb_plan_matmul_cc(ctx, heads, L, d, level, schedule=schedule)
        info = B.blb_plan_cc_info(plan)
        assert [(g["H"], g["c"], g["n_ct"], g["n_out"]) for g in info["groups"]] == [(8, 8, 8, 16), (4, 16, 4, 8)]
        A, Bp, words, h0 = [], [], [], 0
        for gi, grp in enumerate(info["groups"]):
            H = grp["H"]
            aw = np.stack([keys_o.encrypt(o.encode_rns(o.pack_mhp(Q[h0:h0 + H], H, L, d, a, "A"), p.scale, level), level, 80 + gi, a)
                           for a in range(grp["n_ct"])])
            bw = np.stack([keys_o.encrypt(o.encode_rns(o.pack_mhp(Kt[h0:h0 + H], H, L, d, a, "Bp"), p.scale, level), level, 90 + gi, a)
                           for a in range(grp["n_ct"])])
            A += [_import(B, ctx, keep, w, n, level, p.scale) for w in aw]
            Bp += [_import(B, ctx, keep, w, n, level, p.scale) for w in bw]
            words.append((aw, bw))
            h0 += H
        Cd = [_ct(B, keep, n, level - 3) for _ in range(info["n_out"])]
        B.blb_ctx_counters(ctx, reset=True)
        B.blb_matmul_cc(ctx, keys, plan, A, Bp, Cd)
        cnt = B.blb_ctx_counters(ctx, reset=True)
        torch.cuda.synchronize()
        # step 2: two key-switched inner rotations per (t > 0, a); one relinearisation per t;
        # step 3: one right rotation per t with t mod c != 0
        assert cnt["tensor_products"] == 128 * 128 * 768 // 8192 == 1536
        assert cnt["relinearisations"] == 2 * 128
        if schedule == 0:
            assert cnt["key_switches"] == 12 * 2 * 127 + 2 * 128 + (128 - 16) + (128 - 8)
            assert cnt["ct_pt_products"] == 12 * (1 + 2 * 127) + (16 + 2 * 112) + (8 + 2 * 120)
        else:
            assert (cnt["key_switches"], cnt["ct_pt_products"]) == _bsgs_counts(128, [(8, 8, 16), (16, 4, 8)]) == (1086, 1455)
        # one sampled output per head group, word for word
        base, sample = 0, 5
        for (aw, bw), grp in zip(words, info["groups"]):
            want = keys_o.matmul_cc(aw, bw, level, grp["H"], L, d, outputs=[sample], schedule=schedule)
            assert np.array_equal(B.blb_export(ctx, Cd[base + sample], n), want[sample]), f"group H={grp['H']}"
            base += grp["n_out"]
        # every head decodes to Q_h K_h^T
        dec = torch.empty(n, dtype=torch.int64, device="cuda")
        h0, base, err = 0, 0, 0.0
        for grp in info["groups"]:
            vecs = []
            for k in range(grp["n_out"]):
                ct = Cd[base + k]
                B.blb_decrypt(ctx, keys, ct, dec)
                vecs.append(B.blb_decode(ctx, dec, 0, ct.scale, n // 2))
            Cs = wl.unpack_diag(vecs, grp["H"], L, n // 2)
            for h in range(grp["H"]):
                err = max(err, float(np.abs(Cs[h] - Q[h0 + h] @ Kt[h0 + h]).max()))
            h0 += grp["H"]
            base += grp["n_out"]
        assert err < 2.0 ** -20
        B.blb_plan_destroy(plan)
        B.blb_keys_destroy(keys)
    finally:
        torch.cuda.synchronize()
        B.blb_ctx_destroy(ctx)


@pytest.mark.parametrize("schedule", [0, 1])
def test_attention_output_full_size(B, orc, schedule):
    """BERT-base attention output (N = 16384, five primes + two special): Softmax x V_h for 12
    heads of 128 tokens with d_v = 64 (V_h zero-padded to 128 columns, folded to the dense
    diagonal packing), then Concat(Att_h) W_O (768 x 768) on that packing.  Tensor products =
    m^3 H / s = 3072; key switches as each schedule's closed form (BSGS: 1614 instead of 6584);
    every head decodes to S_h V_h within 2^-20 and E to (S_h V_h)_h W_O within 2^-14.  On the
    oracle's encryptions of a dense diagonal-packed input, one sampled output of the diagonal-input
    product equals the oracle's word for word."""
    from paper_2508_19525_amd import workloads as wl
    cfg = wl.C6
    p = cfg["params"]
    heads, L, d_v, d_out = cfg["heads"], cfg["L"], cfg["d_v"], cfg["d_out"]
    n, level, slots = p.n, p.n_q - 1, p.n // 2
    S = wl.attention_weights(6, heads, L)
    V = wl.head_values(6, heads, L, d_v)
    W = wl.weights(6, heads * d_v, d_out, cfg["w_std"])
    o = orc.Context(p.log_n, p.n_q, p.n_special, p.dnum)
    ctx = B.blb_ctx_create(p.log_n, p.n_q, p.n_special, p.dnum, 0, torch.cuda.current_stream().cuda_stream)
    keep = []
    try:
        g = o.cp_geometry(L, heads * d_v, d_out)
        assert (g["Lp"], g["c"], g["c_eff"], g["n_in"], g["n_out"], g["B"], g["G"]) == (128, 64, 64, 12, 12, 8, 8)
        cp_steps = [i * g["Lp"] for i in range(1, g["B"])] + [j * g["B"] * g["Lp"] for j in range(1, g["G"])]
        steps = list(B.blb_cc_rotations(ctx, heads, L, schedule)) + cp_steps
        gal = sorted({o.galois_elt(s) for s in steps})
        keys_o = orc.Keys(o, 83, gal)
        keys = B.blb_keygen(ctx, 83, steps)
        plan = B.blb_plan_matmul_cc_sv(ctx, heads, L, d_v, level, schedule=schedule)
        info = B.blb_plan_cc_info(plan)
        assert [(x["H"], x["c"], x["n_ct"], x["n_out"]) for x in info["groups"]] == [(8, 8, 16, 8), (4, 16, 8, 4)]
        A, Bv, h0 = [], [], 0
        for gi, grp in enumerate(info["groups"]):
            H = grp["H"]
            for a in range(grp["n_ct"]):
                aw = keys_o.encrypt(o.encode_rns(o.pack_mhp(S[h0:h0 + H], H, L, L, a, "A"), p.scale, level), level, 84 + gi, a)
                bw = keys_o.encrypt(o.encode_rns(o.pack_mhp(V[h0:h0 + H], H, L, L, a, "Bp"), p.scale, level), level, 86 + gi, a)
                A.append(_import(B, ctx, keep, aw, n, level, p.scale))
                Bv.append(_import(B, ctx, keep, bw, n, level, p.scale))
            h0 += H
        Att = [_ct(B, keep, n, level - 3) for _ in range(info["n_out"])]
        B.blb_ctx_counters(ctx, reset=True)
        B.blb_matmul_cc(ctx, keys, plan, A, Bv, Att)
        cnt = B.blb_ctx_counters(ctx, reset=True)
        torch.cuda.synchronize()
        assert cnt["tensor_products"] == 128 ** 3 * 12 // 8192 == 3072
        assert cnt["relinearisations"] == 2 * 128
        if schedule == 0:
            assert cnt["key_switches"] == 24 * 2 * 127 + 2 * 128 + (128 - 16) + (128 - 8)
        else:
            assert cnt["key_switches"] == _bsgs_counts(128, [(8, 16, 8), (16, 8, 4)])[0] == 1614
        dec = torch.empty((level + 1) * n, dtype=torch.int64, device="cuda")  # room for any level

        def decode(ct):
            B.blb_decrypt(ctx, keys, ct, dec)
            return B.blb_decode(ctx, dec, ct.level, ct.scale, slots)

        got = np.stack([decode(ct) for ct in Att])
        ct_i, sl, hs, rs, cs = wl.dense_diag_layout(heads, L, d_v, slots)
        want = np.zeros_like(got)
        want[ct_i, sl] = np.stack([S[h] @ V[h] for h in range(heads)])[hs, rs, cs]
        assert np.abs(got - want).max() < 2.0 ** -20
        # Concat(Att_h) W_O on the dense diagonal packing, spatial-first output
        lvl = level - 3
        cplan = B.blb_plan_matmul_cp_diag(ctx, W, heads, d_v, L, lvl)
        assert B.blb_plan_info(cplan) == g
        E = [_ct(B, keep, n, lvl - 1) for _ in range(g["n_out"])]
        B.blb_matmul_cp(ctx, keys, cplan, Att, E)
        vecs = [decode(e) for e in E]
        ref = np.concatenate([S[h] @ V[h] for h in range(heads)], axis=1) @ W
        assert np.abs(wl.unpack_spatial(vecs, L, d_out, slots) - ref).max() < 2.0 ** -14
        if schedule == 0:  # the diagonal-input product does not depend on the ct-ct schedule
            B.blb_plan_destroy(cplan)
            B.blb_plan_destroy(plan)
            B.blb_keys_destroy(keys)
            return
        # word-for-word sample of the diagonal-input product on oracle-encrypted inputs
        rng = np.random.default_rng(wl.seed_for(6, wl.ROLE_ENC))
        X = np.zeros((g["n_in"], slots))
        X[ct_i, sl] = rng.uniform(-1, 1, ct_i.size)
        xw = [keys_o.encrypt(o.encode_rns(X[a], p.scale, lvl), lvl, 88, a) for a in range(g["n_in"])]
        Xc = [_import(B, ctx, keep, w, n, lvl, p.scale) for w in xw]
        E2 = [_ct(B, keep, n, lvl - 1) for _ in range(g["n_out"])]
        B.blb_matmul_cp(ctx, keys, cplan, Xc, E2)
        sample = 5
        want_b = keys_o.matmul_cp_diag(np.stack(xw), lvl, W, L, heads, d_v, outputs=[sample])
        assert np.array_equal(B.blb_export(ctx, E2[sample], n), want_b[sample])
        B.blb_plan_destroy(cplan)
        B.blb_plan_destroy(plan)
        B.blb_keys_destroy(keys)
    finally:
        torch.cuda.synchronize()
        B.blb_ctx_destroy(ctx)
