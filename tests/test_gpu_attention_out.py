"""GPU parity of the attention-output operators against the CPU oracle, word for word, through the
C ABI:

- Softmax x V_h (the ct-ct protocol with V_h zero-padded to L' columns and the diagonal
  ciphertexts folded into the dense diagonal packing), head groups 8 + 4, with the B operand
  pre-rotated by the client or rotated on the server (step 1);
- the ct-pt product with diagonal-packed input (Concat(Att_h) W_O, spatial-first output);
- the two composed on the GPU, eagerly and as recorded graphs.

Inputs are the oracle's encryptions of seeded synthetic matrices (attention weights = softmax
rows, V_h ~ N(0, 1)).  Decoded outputs are checked against FP64 products as well."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def blb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_19525_amd as B
    B.lib()
    return B


class Ctx:
    """GPU context + oracle context with the same parameters"""

    def __init__(self, B, orc, log_n, n_q, n_sp, dnum):
        self.B, self.orc = B, orc
        self.n = 1 << log_n
        self.n_q = n_q
        self.h = B.blb_ctx_create(log_n, n_q, n_sp, dnum, 0, torch.cuda.current_stream().cuda_stream)
        self.o = orc.Context(log_n, n_q, n_sp, dnum)
        self.keep = []

    def close(self):
        torch.cuda.synchronize()
        self.B.blb_ctx_destroy(self.h)

    def ct(self, level, degree=1):
        c, t = self.B.new_ct(self.n, level, degree)
        self.keep.append(t)
        return c

    def import_ct(self, words, level, scale):
        c = self.ct(level)
        self.B.blb_import(self.h, words, c)
        c.scale = scale
        return c

    def export(self, c):
        torch.cuda.synchronize()
        return self.B.blb_export(self.h, c, self.n)

    def decode(self, keys, ct):
        pt = torch.empty((ct.level + 1) * self.n, dtype=torch.int64, device="cuda")
        self.B.blb_decrypt(self.h, keys, ct, pt)
        return self.B.blb_decode(self.h, pt, ct.level, ct.scale, self.n // 2)


@pytest.fixture(scope="module")
def c16(blb, orc):
    """N = 16384, four primes + two special (digits of two primes)"""
    x = Ctx(blb, orc, 14, 4, 2, 2)
    yield x
    x.close()


@pytest.fixture(scope="module")
def c16p5(blb, orc):
    """N = 16384, five primes + two special: Softmax x V_h and one more level (step 1 on the
    server, or the ct-pt product after it)"""
    x = Ctx(blb, orc, 14, 5, 2, 3)
    yield x
    x.close()


@pytest.fixture(scope="module")
def c8(blb, orc):
    x = Ctx(blb, orc, 13, 3, 1, 3)
    yield x
    x.close()


def _softmax_rows(rng, L):
    z = rng.normal(0, 1, (L, L))
    e = np.exp(z - z.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def _unrotated_b(mats, H, L, a, slots):
    """slot i + L'(h + H kappa) <- B_h{a c + kappa, i} (B_h = mats[h], L rows): the operand before
    step 1"""
    lp = 1 << int(np.ceil(np.log2(L)))
    c = slots // (lp * H)
    v = np.zeros(slots)
    for h in range(H):
        for kap in range(c):
            k = a * c + kap
            if k < mats[h].shape[0]:
                w = mats[h].shape[1]
                v[lp * (h + H * kap): lp * (h + H * kap) + w] = mats[h][k, :]
    return v


def _dense_expected(wl, mats, heads, L, d_v, n_ct, slots):
    """slot vectors of the dense diagonal packing of the L x d_v matrices mats (0 elsewhere)"""
    ct, sl, hs, rs, cs = wl.dense_diag_layout(heads, L, d_v, slots)
    v = np.zeros((n_ct, slots))
    v[ct, sl] = np.stack(mats)[hs, rs, cs]
    return v


def _sv_case(c, heads, L, d_v, seed, outputs=None, prerot=True, extra_steps=(), with_oracle=True, schedule=0):
    from paper_2508_19525_amd import workloads as wl
    B, orc = c.B, c.orc
    rng = np.random.default_rng(seed)
    S = [_softmax_rows(rng, L) for _ in range(heads)]
    V = [rng.normal(0, 1, (L, d_v)) for _ in range(heads)]
    level, scale = c.n_q - 1, 2.0 ** 40
    steps = list(B.blb_cc_rotations(c.h, heads, L, schedule, b_prerotated=prerot)) + [s for s in extra_steps]
    gal = sorted({c.o.galois_elt(s) for s in steps})
    keys_o = orc.Keys(c.o, 41, gal)
    keys_g = B.blb_keygen(c.h, 41, steps)
    plan = B.blb_plan_matmul_cc_sv(c.h, heads, L, d_v, level, b_prerotated=prerot, schedule=schedule)
    info = B.blb_plan_cc_info(plan)
    A_g, B_g, want, h0 = [], [], [], 0
    slots = c.n // 2
    for gi, grp in enumerate(info["groups"]):
        H = grp["H"]
        assert H == wl.head_groups(heads)[gi]
        og = c.o.cc_sv_geometry(H, L, d_v)
        assert (og["c"], og["n_ct"], og["n_out"]) == (grp["c"], grp["n_ct"], grp["n_out"])
        Aw = np.stack([keys_o.encrypt(c.o.encode_rns(c.o.pack_mhp(S[h0:h0 + H], H, L, L, a, "A"), scale, level), level, 60 + gi, a)
                       for a in range(og["n_ct"])])
        if prerot:
            bvec = [c.o.pack_mhp(V[h0:h0 + H], H, L, L, a, "Bp") for a in range(og["n_ct"])]
            assert np.array_equal(wl.pack_mhp(V[h0:h0 + H], H, L, L, 0, "Bp", slots), bvec[0])
        else:
            bvec = [_unrotated_b(V[h0:h0 + H], H, L, a, slots) for a in range(og["n_ct"])]
        Bw = np.stack([keys_o.encrypt(c.o.encode_rns(v, scale, level), level, 70 + gi, a) for a, v in enumerate(bvec)])
        A_g += [c.import_ct(w, level, scale) for w in Aw]
        B_g += [c.import_ct(w, level, scale) for w in Bw]
        outs = None if outputs is None else [o for o in outputs if o < og["n_out"]]
        if with_oracle:
            want.append((keys_o.matmul_cc_sv(Aw, Bw, level, H, L, d_v, outputs=outs, b_prerotated=prerot, schedule=schedule), outs,
                         grp))
        h0 += H
    Cd = [c.ct(level - (3 if prerot else 4)) for _ in range(info["n_out"])]
    B.blb_matmul_cc(c.h, keys_g, plan, A_g, B_g, Cd)
    return dict(S=S, V=V, keys_o=keys_o, keys_g=keys_g, plan=plan, info=info, A=A_g, B=B_g, C=Cd, want=want, level=level)


@pytest.mark.parametrize("heads,L,d_v,outputs,prerot,schedule", [
    (12, 64, 32, [0], True, 0), (4, 50, 20, None, True, 0), (4, 64, 32, None, False, 0),
    (12, 64, 32, [0], True, 1), (4, 50, 20, None, True, 1), (4, 64, 32, None, False, 1)])
def test_softmax_v_matches_oracle(request, heads, L, d_v, outputs, prerot, schedule):
    """Dense diagonal-packed Softmax x V_h word for word against the oracle (groups 8 + 4 with
    two and one dense outputs, a ragged L with d_v = 20 padded to 32, and step 1 on the server),
    and, where every output is computed, decoded against S_h V_h in FP64 (zero in the padded
    columns and rows); for the plain and the BSGS schedule."""
    from paper_2508_19525_amd import workloads as wl
    c = request.getfixturevalue("c16" if prerot else "c16p5")
    r = _sv_case(c, heads, L, d_v, heads + L + d_v, outputs, prerot, schedule=schedule)
    base = 0
    for O_want, outs, grp in r["want"]:
        for o in (range(grp["n_out"]) if outs is None else outs):
            assert np.array_equal(c.export(r["C"][base + o]), O_want[o]), f"group H={grp['H']} output {o}"
        base += grp["n_out"]
    if outputs is None:
        got = np.stack([c.decode(r["keys_g"], ct) for ct in r["C"]])
        want = _dense_expected(wl, [r["S"][h] @ r["V"][h] for h in range(heads)], heads, L, d_v, len(r["C"]), c.n // 2)
        assert np.abs(got - want).max() < 2.0 ** -20
    c.B.blb_plan_destroy(r["plan"])
    c.B.blb_keys_destroy(r["keys_g"])


def _diag_case(c, heads, L, d_v, d_out, level, seed, outputs=None):
    from paper_2508_19525_amd import workloads as wl
    B, orc = c.B, c.orc
    rng = np.random.default_rng(seed)
    att = [rng.uniform(-1, 1, (L, d_v)) for _ in range(heads)]
    W = rng.normal(0, 0.05, (heads * d_v, d_out))
    dvp = 1 << int(np.ceil(np.log2(d_v)))
    g = c.o.cp_geometry(L, heads * dvp, d_out)
    plan = B.blb_plan_matmul_cp_diag(c.h, W, heads, d_v, L, level)
    assert B.blb_plan_info(plan) == g
    steps = [i * g["Lp"] for i in range(1, g["B"])] + [j * g["B"] * g["Lp"] for j in range(1, g["G"])]
    keys_o = orc.Keys(c.o, 43, c.o.cp_galois(L, heads * dvp, d_out))
    keys_g = B.blb_keygen(c.h, 43, steps)
    scale = 2.0 ** 30
    vecs = _dense_expected(wl, att, heads, L, d_v, g["n_in"], c.n // 2)
    Xw = np.stack([keys_o.encrypt(c.o.encode_rns(vecs[a], scale, level), level, 110, a) for a in range(g["n_in"])])
    X = [c.import_ct(w, level, scale) for w in Xw]
    Y = [c.ct(level - 1) for _ in range(g["n_out"])]
    B.blb_matmul_cp(c.h, keys_g, plan, X, Y)
    want = keys_o.matmul_cp_diag(Xw, level, W, L, heads, d_v, outputs=outputs)
    return dict(att=att, W=W, g=g, plan=plan, keys_g=keys_g, X=X, Y=Y, want=want)


@pytest.mark.parametrize("case", ["n8192_12heads", "n16384_ragged"])
def test_matmul_cp_diag_matches_oracle(request, case):
    """Diagonal-input ct-pt product word for word against the oracle (12 heads = 8 + 4 at
    N = 8192: six inputs from two head groups; a ragged L and d_v = 24 at N = 16384), decoded
    against Concat(Att_h) W in FP64."""
    from paper_2508_19525_amd import workloads as wl
    if case == "n8192_12heads":
        c, args = request.getfixturevalue("c8"), (12, 64, 32, 96, 2)
    else:
        c, args = request.getfixturevalue("c16"), (6, 100, 24, 72, 1)
    heads, L, d_v, d_out, level = args
    r = _diag_case(c, heads, L, d_v, d_out, level, sum(args))
    g = r["g"]
    for b in range(g["n_out"]):
        assert np.array_equal(c.export(r["Y"][b]), r["want"][b]), f"output {b}"
    vecs = [c.decode(r["keys_g"], y) for y in r["Y"]]
    got = wl.unpack_spatial(vecs, L, d_out, c.n // 2)
    assert np.abs(got - np.concatenate(r["att"], axis=1) @ r["W"]).max() < 2.0 ** -10
    c.B.blb_plan_destroy(r["plan"])
    c.B.blb_keys_destroy(r["keys_g"])


def test_plan_limits_rejected(c16):
    """Geometries the dense fold cannot express are refused before any work: d_v' > L', or a
    head group with more columns per ciphertext than d_v'."""
    B = c16.B
    for args in [(8, 32, 64), (1, 64, 64)]:
        with pytest.raises(B.BlbError):
            B.blb_plan_matmul_cc_sv(c16.h, args[0], args[1], args[2], 3)
        with pytest.raises(B.BlbError):
            B.blb_plan_matmul_cp_diag(c16.h, np.zeros((args[0] * args[2], 8)), args[0], args[2], args[1], 1)


def test_attention_output_pipeline_eager_and_graph(c16p5):
    """Softmax x V_h then Concat(Att_h) W_O on the GPU with no repacking in between: decodes to
    (S_h V_h)_h W_O; recorded graphs of the two operators replay to the eager words."""
    from paper_2508_19525_amd import workloads as wl
    c = c16p5
    B = c.B
    heads, L, d_v, d_out = 12, 64, 32, 64
    g = c.o.cp_geometry(L, heads * d_v, d_out)
    cp_steps = [i * g["Lp"] for i in range(1, g["B"])] + [j * g["B"] * g["Lp"] for j in range(1, g["G"])]
    r = _sv_case(c, heads, L, d_v, 5, extra_steps=cp_steps, with_oracle=False)
    rng = np.random.default_rng(6)
    W = rng.normal(0, 0.05, (heads * d_v, d_out))
    lvl = r["level"] - 3
    plan = B.blb_plan_matmul_cp_diag(c.h, W, heads, d_v, L, lvl)
    E = [c.ct(lvl - 1) for _ in range(g["n_out"])]
    B.blb_matmul_cp(c.h, r["keys_g"], plan, r["C"], E)
    vecs = [c.decode(r["keys_g"], e) for e in E]
    ref = np.concatenate([r["S"][h] @ r["V"][h] for h in range(heads)], axis=1) @ W
    assert np.abs(wl.unpack_spatial(vecs, L, d_out, c.n // 2) - ref).max() < 2.0 ** -16
    eager_c = [c.export(x) for x in r["C"]]
    eager_e = [c.export(x) for x in E]
    Cg = [c.ct(lvl) for _ in range(len(r["C"]))]
    Eg = [c.ct(lvl - 1) for _ in range(g["n_out"])]
    ex1 = B.blb_exec_create_cc(c.h, r["keys_g"], r["plan"], r["A"], r["B"], Cg)
    ex2 = B.blb_exec_create_cp(c.h, r["keys_g"], plan, Cg, Eg)
    for rep in range(2):
        B.blb_exec_run(ex1)
        B.blb_exec_run(ex2)
        torch.cuda.synchronize()
        for k, x in enumerate(Cg):
            assert np.array_equal(c.export(x), eager_c[k]), f"replay {rep} Att ct {k}"
        for k, x in enumerate(Eg):
            assert np.array_equal(c.export(x), eager_e[k]), f"replay {rep} E ct {k}"
        # eager work between replays
        B.blb_matmul_cp(c.h, r["keys_g"], plan, r["C"], E)
        torch.cuda.synchronize()
    B.blb_exec_destroy(ex1)
    B.blb_exec_destroy(ex2)
    B.blb_plan_destroy(plan)
    B.blb_plan_destroy(r["plan"])
    B.blb_keys_destroy(r["keys_g"])


# --------------------------------------------------------------------------------------
# matmul_cp with W_Q / W_K columns reordered for the multi-head packing, and Q_h K_h^T from X
# --------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c16p6(blb, orc):
    """N = 16384, six primes + two special (dnum 3): matmul_cp, then the ct-ct product with step 1
    on the server"""
    x = Ctx(blb, orc, 14, 6, 2, 3)
    yield x
    x.close()


def _cp_keys(c, L, d_in, d_out):
    g = c.o.cp_geometry(L, d_in, d_out)
    return g, [i * g["Lp"] for i in range(1, g["B"])] + [j * g["B"] * g["Lp"] for j in range(1, g["G"])]


def test_cp_mhp_matches_oracle(c8):
    """The reordered-column plan word for word against the oracle's matmul_cp on the oracle's own
    reordering of W (12 heads = 8 + 4, ragged operand ciphertexts), decoded against the multi-head
    packing of X W."""
    from paper_2508_19525_amd import workloads as wl
    c, B = c8, c8.B
    heads, L, d_in, d_head, level = 12, 64, 96, 16, 2
    rng = np.random.default_rng(12)
    X = rng.uniform(-1, 1, (L, d_in))
    W = rng.normal(0, 0.05, (d_in, heads * d_head))
    Wp = c.o.mhp_weight(W, heads, d_head, L)
    g, steps = _cp_keys(c, L, d_in, Wp.shape[1])
    plan = B.blb_plan_matmul_cp_mhp(c.h, W, heads, d_head, L, level)
    assert B.blb_plan_info(plan) == g
    keys_o = c.orc.Keys(c.o, 45, c.o.cp_galois(L, d_in, Wp.shape[1]))
    keys_g = B.blb_keygen(c.h, 45, steps)
    scale = 2.0 ** 30
    xw = np.stack([keys_o.encrypt(c.o.encode_rns(c.o.pack_spatial(X, a), scale, level), level, 120, a) for a in range(g["n_in"])])
    Xc = [c.import_ct(w, level, scale) for w in xw]
    Y = [c.ct(level - 1) for _ in range(g["n_out"])]
    B.blb_matmul_cp(c.h, keys_g, plan, Xc, Y)
    want = keys_o.matmul_cp(xw, level, Wp, L)
    for b in range(g["n_out"]):
        assert np.array_equal(c.export(Y[b]), want[b]), f"output {b}"
    Ym, h0, b = X @ W, 0, 0
    for H in wl.head_groups(heads):
        mats = [Ym[:, (h0 + h) * d_head:(h0 + h + 1) * d_head] for h in range(H)]
        cg = c.n // 2 // (g["Lp"] * H)
        for a in range(-(-d_head // cg)):
            v = c.decode(keys_g, Y[b])
            assert np.abs(v - wl.pack_mhp(mats, H, L, d_head, a, "A", c.n // 2)).max() < 2.0 ** -10
            b += 1
        h0 += H
    B.blb_plan_destroy(plan)
    B.blb_keys_destroy(keys_g)


def test_fused_qk_from_x_matches_oracle(c16p6):
    """X -> Q = X W_Q', K = X W_K' -> ct-ct product with step 1 on the server (N = 16384, six
    primes, 12 heads): the two reordered-column products and one sampled diagonal output of each
    head group equal the oracle's composition word for word; every head decodes to Q_h K_h^T."""
    from paper_2508_19525_amd import workloads as wl
    c, B = c16p6, c16p6.B
    heads, L, d_in, d_head, level = 12, 64, 64, 32, 5
    rng = np.random.default_rng(13)
    X = rng.normal(0, 1, (L, d_in))
    WQ = rng.normal(0, 0.15, (d_in, heads * d_head))
    WK = rng.normal(0, 0.15, (d_in, heads * d_head))
    WQp, WKp = c.o.mhp_weight(WQ, heads, d_head, L), c.o.mhp_weight(WK, heads, d_head, L)
    g, cp_steps = _cp_keys(c, L, d_in, WQp.shape[1])
    steps = list(B.blb_cc_rotations(c.h, heads, L)) + cp_steps
    keys_o = c.orc.Keys(c.o, 47, sorted({c.o.galois_elt(s) for s in steps}))
    keys_g = B.blb_keygen(c.h, 47, steps)
    scale = 2.0 ** 40
    xw = np.stack([keys_o.encrypt(c.o.encode_rns(c.o.pack_spatial(X, a), scale, level), level, 130, a) for a in range(g["n_in"])])
    Xc = [c.import_ct(w, level, scale) for w in xw]
    pq = B.blb_plan_matmul_cp_mhp(c.h, WQ, heads, d_head, L, level)
    pk = B.blb_plan_matmul_cp_mhp(c.h, WK, heads, d_head, L, level)
    pcc = B.blb_plan_matmul_cc(c.h, heads, L, d_head, level - 1, b_prerotated=False)
    info = B.blb_plan_cc_info(pcc)
    assert info["n_ct"] == g["n_out"]
    Qc = [c.ct(level - 1) for _ in range(g["n_out"])]
    Kc = [c.ct(level - 1) for _ in range(g["n_out"])]
    B.blb_matmul_cp(c.h, keys_g, pq, Xc, Qc)
    B.blb_matmul_cp(c.h, keys_g, pk, Xc, Kc)
    Cd = [c.ct(level - 5) for _ in range(info["n_out"])]
    B.blb_matmul_cc(c.h, keys_g, pcc, Qc, Kc, Cd)
    Qw, Kw = keys_o.matmul_cp(xw, level, WQp, L), keys_o.matmul_cp(xw, level, WKp, L)
    for b in range(g["n_out"]):
        assert np.array_equal(c.export(Qc[b]), Qw[b]), f"Q ct {b}"
        assert np.array_equal(c.export(Kc[b]), Kw[b]), f"K ct {b}"
    base, sample = 0, 1
    for grp in info["groups"]:
        sl = slice(grp["ct0"], grp["ct0"] + grp["n_ct"])
        want = keys_o.matmul_cc(Qw[sl], Kw[sl], level - 1, grp["H"], L, d_head, outputs=[sample], b_prerotated=False)
        assert np.array_equal(c.export(Cd[base + sample]), want[sample]), f"group H={grp['H']}"
        base += grp["n_out"]
    Qm, Km = X @ WQ, X @ WK
    h0, base, err = 0, 0, 0.0
    for grp in info["groups"]:
        vecs = [c.decode(keys_g, Cd[base + o]) for o in range(grp["n_out"])]
        Cs = wl.unpack_diag(vecs, grp["H"], L, c.n // 2)
        for h in range(grp["H"]):
            hh = h0 + h
            ref = Qm[:, hh * d_head:(hh + 1) * d_head] @ Km[:, hh * d_head:(hh + 1) * d_head].T
            err = max(err, float(np.abs(Cs[h] - ref).max()))
        h0 += grp["H"]
        base += grp["n_out"]
    assert err < 2.0 ** -18
    for p in (pq, pk, pcc):
        B.blb_plan_destroy(p)
    B.blb_keys_destroy(keys_g)
