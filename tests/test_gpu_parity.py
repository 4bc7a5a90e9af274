"""GPU parity: the HIP library (through its C ABI) against the CPU oracle, word for word.

Ciphertexts are compared in canonical coefficient form (blb_export) against the oracle's
coefficient-form words.  Encryption randomness comes from the same seeds on both sides
(each side implements Philox4x32-10 itself).
"""
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
        self.n_q, self.n_sp = n_q, n_sp
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

    def pt_dev(self, level):
        t = torch.empty((level + 1) * self.n, dtype=torch.int64, device="cuda")
        self.keep.append(t)
        return t

    def upload_words(self, words):
        a = np.ascontiguousarray(words, dtype=np.uint64)
        t = torch.from_numpy(a.view(np.int64).reshape(-1).copy()).cuda()
        self.keep.append(t)
        return t

    def import_ct(self, words, level, degree=1):
        c = self.ct(level, degree)
        self.B.blb_import(self.h, words, c)
        return c

    def export(self, c):
        torch.cuda.synchronize()
        return self.B.blb_export(self.h, c, self.n)


@pytest.fixture(scope="module")
def c1(blb, orc):
    x = Ctx(blb, orc, 12, 2, 1, 2)
    yield x
    x.close()


@pytest.fixture(scope="module")
def c2s(blb, orc):
    x = Ctx(blb, orc, 13, 3, 1, 3)
    yield x
    x.close()


@pytest.fixture(scope="module")
def c3s(blb, orc):
    x = Ctx(blb, orc, 14, 4, 2, 2)
    yield x
    x.close()


def _ctxs(request, names):
    return [request.getfixturevalue(n) for n in names]


def test_moduli_match_oracle(c1, c2s, c3s):
    for c in (c1, c2s, c3s):
        m = c.B.blb_ctx_moduli(c.h, len(c.o.moduli))
        assert np.array_equal(m, c.o.moduli)


@pytest.mark.parametrize("name", ["c1", "c2s", "c3s"])
def test_encode_matches_oracle(request, name):
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(1)
    top = c.n_q - 1
    for scale, dist in [(2.0 ** 40, "normal"), (2.0 ** 30, "uniform"), (float(c.o.q[top]), "weights")]:
        if dist == "normal":
            v = rng.normal(0, 1, c.n // 2)
        elif dist == "uniform":
            v = rng.uniform(-1, 1, c.n // 2 - 5)  # ragged: trailing slots zero
        else:
            v = rng.normal(0, 0.02, c.n // 2)
        pt = c.pt_dev(top)
        c.B.blb_encode(c.h, v, scale, top, pt)
        torch.cuda.synchronize()
        got = pt.cpu().numpy().view(np.uint64).reshape(top + 1, c.n)
        want = c.o.encode_rns(v, scale, top)
        mism = int((got != want).sum())
        assert mism == 0, f"{mism} encode mismatches at scale {scale}"


@pytest.mark.parametrize("name", ["c1", "c2s", "c3s"])
def test_encrypt_decrypt_match_oracle(request, name):
    c = request.getfixturevalue(name)
    keys_o = c.orc.Keys(c.o, 11)
    keys_g = c.B.blb_keygen(c.h, 11, [])
    rng = np.random.default_rng(2)
    for level in (c.n_q - 1, 0):
        want_pt = c.o.encode_rns(rng.normal(0, 1, c.n // 2), 2.0 ** 30, level)
        ct = c.ct(level)
        c.B.blb_encrypt(c.h, keys_g, c.upload_words(want_pt), level, 2.0 ** 30, 77, 5, ct)
        got = c.export(ct)
        want = keys_o.encrypt(want_pt, level, 77, 5)
        assert np.array_equal(got, want)
        dec = c.pt_dev(level)
        c.B.blb_decrypt(c.h, keys_g, ct, dec)
        torch.cuda.synchronize()
        assert np.array_equal(dec.cpu().numpy().view(np.uint64).reshape(level + 1, c.n), keys_o.decrypt(want, level))
    c.B.blb_keys_destroy(keys_g)


@pytest.mark.parametrize("name,steps", [("c1", [1, 5, -3]), ("c2s", [128, 1024, -1]), ("c3s", [128, 3, -128])])
def test_rotate_matches_oracle(request, name, steps):
    c = request.getfixturevalue(name)
    keys_o = c.orc.Keys(c.o, 21, [c.o.galois_elt(s) for s in steps])
    keys_g = c.B.blb_keygen(c.h, 21, steps)
    rng = np.random.default_rng(3)
    for level in sorted({c.n_q - 1, 1, 0}):
        if level >= c.n_q:
            continue
        m = rng.normal(0, 1, c.n // 2)
        want_ct = keys_o.encrypt(c.o.encode_rns(m, 2.0 ** 30, level), level, 9, 0)
        ct = c.import_ct(want_ct, level)
        for s in steps:
            out = c.ct(level)
            c.B.blb_rotate(c.h, keys_g, ct, s, out)
            got = c.export(out)
            want = keys_o.rotate(want_ct, level, s)
            assert np.array_equal(got, want), f"rotation {s} at level {level}"
    c.B.blb_keys_destroy(keys_g)


@pytest.mark.parametrize("name", ["c1", "c2s", "c3s"])
def test_rescale_matches_oracle(request, name):
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(4)
    for level in range(c.n_q - 1, 0, -1):
        words = np.stack([np.stack([rng.integers(0, int(q), c.n, dtype=np.uint64) for q in c.o.q[: level + 1]]) for _ in range(2)])
        ct = c.import_ct(words, level)
        out = c.ct(level - 1)
        c.B.blb_rescale(c.h, ct, out)
        assert out.level == level - 1
        assert np.array_equal(c.export(out), c.o.rescale(words, level))


def _cp_case(c, L, d_in, d_out, level, seed, x_std=None):
    B, orc = c.B, c.orc
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (L, d_in)) if x_std is None else rng.normal(0, x_std, (L, d_in))
    W = rng.normal(0, 0.02, (d_in, d_out))
    g = c.o.cp_geometry(L, d_in, d_out)
    gal = c.o.cp_galois(L, d_in, d_out)
    steps = [i * g["Lp"] for i in range(1, g["B"])] + [j * g["B"] * g["Lp"] for j in range(1, g["G"])]
    keys_o = orc.Keys(c.o, 31, gal)
    keys_g = B.blb_keygen(c.h, 31, steps)
    scale = 2.0 ** 30
    X_words = np.stack([keys_o.encrypt(c.o.encode_rns(c.o.pack_spatial(X, a), scale, level), level, 100, a) for a in range(g["n_in"])])
    Xc = []
    for a in range(g["n_in"]):
        ct = c.import_ct(X_words[a], level)
        ct.scale = scale
        Xc.append(ct)
    plan = B.blb_plan_matmul_cp(c.h, W, L, level)
    info = B.blb_plan_info(plan)
    assert info == g
    Yc = [c.ct(level - 1) for _ in range(g["n_out"])]
    B.blb_matmul_cp(c.h, keys_g, plan, Xc, Yc)
    return dict(X=X, W=W, g=g, keys_o=keys_o, keys_g=keys_g, X_words=X_words, Yc=Yc, plan=plan, scale=scale)


@pytest.mark.parametrize("shape", [(32, 32, 32), (20, 40, 24), (5, 96, 70)])
def test_matmul_cp_matches_oracle_c1(c1, shape):
    L, d_in, d_out = shape
    r = _cp_case(c1, L, d_in, d_out, 1, sum(shape))
    want = r["keys_o"].matmul_cp(r["X_words"], 1, r["W"], L)
    for b in range(r["g"]["n_out"]):
        assert np.array_equal(c1.export(r["Yc"][b]), want[b]), f"output {b}"
    c1.B.blb_plan_destroy(r["plan"])
    c1.B.blb_keys_destroy(r["keys_g"])


def test_matmul_cp_matches_oracle_n8192_ragged(c2s):
    """N = 8192, three primes, ragged L and widths spanning several output ciphertexts"""
    L, d_in, d_out = 100, 96, 80
    r = _cp_case(c2s, L, d_in, d_out, 2, 7, x_std=1.0)
    want = r["keys_o"].matmul_cp(r["X_words"], 2, r["W"], L)
    for b in range(r["g"]["n_out"]):
        assert np.array_equal(c2s.export(r["Yc"][b]), want[b]), f"output {b}"
    # decoded accuracy against FP64
    vecs = []
    for b in range(r["g"]["n_out"]):
        pt = c2s.pt_dev(1)
        c2s.B.blb_decrypt(c2s.h, r["keys_g"], r["Yc"][b], pt)
        vecs.append(c2s.B.blb_decode(c2s.h, pt, 1, r["scale"], c2s.n // 2))
    from paper_2508_19525_amd.workloads import unpack_spatial
    got = unpack_spatial(vecs, L, d_out, c2s.n // 2)
    assert np.abs(got - r["X"] @ r["W"]).max() < 2.0 ** -10
    c2s.B.blb_plan_destroy(r["plan"])
    c2s.B.blb_keys_destroy(r["keys_g"])


@pytest.mark.parametrize("name", ["c1", "c2s"])
def test_mask_to_share_matches_oracle(request, name):
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(5)
    keys_o = c.orc.Keys(c.o, 41)
    level = c.n_q - 1
    words = [keys_o.encrypt(c.o.encode_rns(rng.normal(0, 1, c.n // 2), 2.0 ** 30, level), level, 3, t) for t in range(3)]
    for target in (level, 0):
        cts = [c.import_ct(w, level) for w in words]
        share = torch.zeros(3 * (target + 1) * c.n, dtype=torch.int64, device="cuda")
        c.B.blb_mask_to_share(c.h, cts, 1234, target, share)
        torch.cuda.synchronize()
        sh = share.cpu().numpy().view(np.uint64).reshape(3, target + 1, c.n)
        for t in range(3):
            masked, want_share = c.o.mask_to_share(words[t], level, target, 1234, t)
            assert cts[t].level == target
            assert np.array_equal(c.export(cts[t]), masked)
            assert np.array_equal(sh[t], want_share)


@pytest.mark.parametrize("name", ["c1", "c2s", "c3s"])
def test_add_share_matches_oracle(request, name):
    """The server's step of the MPC-to-CKKS conversion word for word (shares uniform per limb),
    and mask-to-share followed by it restores the ciphertexts exactly."""
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(8)
    keys_o = c.orc.Keys(c.o, 44)
    level = c.n_q - 1
    words = [keys_o.encrypt(c.o.encode_rns(rng.normal(0, 1, c.n // 2), 2.0 ** 30, level), level, 9, t) for t in range(3)]
    sh = np.stack([np.stack([c.orc.sample_uniform(77, i, t, 6, int(c.o.q[i]), c.n) for i in range(level + 1)]) for t in range(3)])
    cts = [c.import_ct(w, level) for w in words]
    c.B.blb_add_share(c.h, cts, c.upload_words(sh))
    for t in range(3):
        assert np.array_equal(c.export(cts[t]), c.o.add_share(words[t], level, sh[t])), f"ct {t}"
    cts = [c.import_ct(w, level) for w in words]
    share = torch.zeros(3 * (level + 1) * c.n, dtype=torch.int64, device="cuda")
    c.B.blb_mask_to_share(c.h, cts, 4321, level, share)
    c.B.blb_add_share(c.h, cts, share)
    for t in range(3):
        assert np.array_equal(c.export(cts[t]), words[t]), f"round trip ct {t}"


@pytest.mark.parametrize("name,block,n_blocks", [("c1", 32, 16), ("c2s", 64, 32), ("c2s", 128, 32)])
def test_rotate_sum_matches_oracle(request, name, block, n_blocks):
    """Rotate-and-sum word for word against the oracle on three ciphertexts: summation with the
    first-block mask, without it, and broadcast (block x n_blocks below and equal to N/2)."""
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(block + n_blocks)
    steps, st = [], block
    while st < block * n_blocks:
        steps += [st, -st]
        st *= 2
    keys_o = c.orc.Keys(c.o, 46, sorted({c.o.galois_elt(x) for x in steps}))
    keys_g = c.B.blb_keygen(c.h, 46, steps)
    level = c.n_q - 1
    words = [keys_o.encrypt(c.o.encode_rns(rng.uniform(-1, 1, c.n // 2), 2.0 ** 30, level), level, 12, t) for t in range(3)]
    for direction, mask in ((0, True), (0, False), (1, False)):
        cts = [c.import_ct(w, level) for w in words]
        for x in cts:
            x.scale = 2.0 ** 30
        lv = level - 1 if mask else level
        outs = [c.ct(lv) for _ in range(3)]
        c.B.blb_rotate_sum(c.h, keys_g, cts, outs, block, n_blocks, direction, mask)
        for t in range(3):
            assert outs[t].level == lv
            want = keys_o.rotate_sum(words[t], level, block, n_blocks, direction, mask)
            assert np.array_equal(c.export(outs[t]), want), f"direction {direction} mask {mask} ct {t}"
    c.B.blb_keys_destroy(keys_g)


@pytest.mark.parametrize("name", ["c1", "c2s"])
def test_rerandomize_matches_oracle(request, name):
    """Public-key re-randomisation with flooding (object id = position in the list), word for
    word, at two levels and two flooding widths; then mask-to-share on the result."""
    c = request.getfixturevalue(name)
    rng = np.random.default_rng(6)
    keys_o = c.orc.Keys(c.o, 43)
    keys_g = c.B.blb_keygen(c.h, 43, [])
    level = c.n_q - 1
    for lvl, bits in ((level, 40), (0, 32)):
        words = [keys_o.encrypt(c.o.encode_rns(rng.normal(0, 1, c.n // 2), 2.0 ** 30, lvl), lvl, 7, t) for t in range(3)]
        cts = [c.import_ct(w, lvl) for w in words]
        c.B.blb_rerandomize(c.h, keys_g, cts, 555, bits)
        for t in range(3):
            assert np.array_equal(c.export(cts[t]), keys_o.rerandomize(words[t], lvl, 555, t, bits)), f"level {lvl} ct {t}"
    with pytest.raises(c.B.BlbError):
        c.B.blb_rerandomize(c.h, keys_g, cts, 1, 49)
    c.B.blb_keys_destroy(keys_g)


# --------------------------------------------------------------------------------------
# matmul_cc
# --------------------------------------------------------------------------------------
def _unrotated_b(mats, H, L, d, a, slots):
    """B operand without the client-side row rotation: slot i + L'(h + H kappa) <- B_h{a c + kappa, i}"""
    lp = 1 << int(np.ceil(np.log2(L)))
    cc = slots // (lp * H)
    v = np.zeros(slots)
    for h in range(H):
        for kap in range(cc):
            k = a * cc + kap
            if k < d:
                v[lp * (h + H * kap): lp * (h + H * kap) + L] = mats[h][k, :]
    return v


def _cc_case(c, heads, L, d, seed, outputs=None, prerot=True, schedule=0):
    from paper_2508_19525_amd import workloads as wl
    B, orc = c.B, c.orc
    rng = np.random.default_rng(seed)
    Q = [rng.normal(0, 1, (L, d)) for _ in range(heads)]
    Kt = [rng.normal(0, 1, (L, d)).T.copy() for _ in range(heads)]
    level, scale = c.n_q - 1, 2.0 ** 40
    steps = B.blb_cc_rotations(c.h, heads, L, schedule, b_prerotated=prerot)
    gal = sorted({c.o.galois_elt(s) for s in steps})
    keys_o = orc.Keys(c.o, 51, gal)
    keys_g = B.blb_keygen(c.h, 51, steps)
    plan = B.blb_plan_matmul_cc(c.h, heads, L, d, level, b_prerotated=prerot, schedule=schedule)
    info = B.blb_plan_cc_info(plan)
    A_g, B_g, want, h0 = [], [], [], 0
    for gi, grp in enumerate(info["groups"]):
        H = grp["H"]
        assert H == wl.head_groups(heads)[gi]
        og = c.o.cc_geometry(H, L, d)
        assert (og["c"], og["n_ct"], og["n_out"]) == (grp["c"], grp["n_ct"], grp["n_out"])
        Aw = np.stack([keys_o.encrypt(c.o.encode_rns(c.o.pack_mhp(Q[h0:h0 + H], H, L, d, a, "A"), scale, level), level, 60 + gi, a)
                       for a in range(og["n_ct"])])
        bvec = [c.o.pack_mhp(Kt[h0:h0 + H], H, L, d, a, "Bp") if prerot else _unrotated_b(Kt[h0:h0 + H], H, L, d, a, c.n // 2)
                for a in range(og["n_ct"])]
        Bw = np.stack([keys_o.encrypt(c.o.encode_rns(v, scale, level), level, 70 + gi, a) for a, v in enumerate(bvec)])
        # the client-side packing of the library's helper module agrees with the oracle's
        assert np.array_equal(wl.pack_mhp(Q[h0:h0 + H], H, L, d, 0, "A", c.n // 2), c.o.pack_mhp(Q[h0:h0 + H], H, L, d, 0, "A"))
        assert np.array_equal(wl.pack_mhp(Kt[h0:h0 + H], H, L, d, 0, "Bp", c.n // 2), c.o.pack_mhp(Kt[h0:h0 + H], H, L, d, 0, "Bp"))
        for a in range(og["n_ct"]):
            x = c.import_ct(Aw[a], level)
            x.scale = scale
            A_g.append(x)
            y = c.import_ct(Bw[a], level)
            y.scale = scale
            B_g.append(y)
        outs = None if outputs is None else [o for o in outputs if o < og["n_out"]]
        want.append((keys_o.matmul_cc(Aw, Bw, level, H, L, d, outputs=outs, b_prerotated=prerot, schedule=schedule), outs, grp))
        h0 += H
    Cd = [c.ct(level - (3 if prerot else 4)) for _ in range(info["n_out"])]
    B.blb_matmul_cc(c.h, keys_g, plan, A_g, B_g, Cd)
    return dict(Q=Q, Kt=Kt, keys_o=keys_o, keys_g=keys_g, plan=plan, info=info, A=A_g, B=B_g, C=Cd, want=want, level=level)


@pytest.fixture(scope="module")
def c5p(blb, orc):
    """five ciphertext primes at N = 16384 (two special, digits of two primes): room for step 1
    on the server"""
    x = Ctx(blb, orc, 14, 5, 2, 3)
    yield x
    x.close()


@pytest.mark.parametrize("heads,L,d,outputs,prerot,schedule", [
    (8, 32, 32, None, True, 0), (12, 64, 32, [0, 1], True, 0), (8, 32, 32, None, False, 0), (12, 40, 32, [0, 3], False, 0),
    (8, 32, 32, None, True, 1), (12, 64, 32, None, True, 1), (12, 100, 24, [1, 2], True, 1), (8, 32, 32, None, False, 1),
    (12, 40, 32, [0, 3], False, 1)])
def test_matmul_cc_matches_oracle(request, heads, L, d, outputs, prerot, schedule):
    """Multi-head ct-ct matmul word for word against the oracle, including the 8 + 4 head-group
    split; decoded outputs equal Q_h K_h^T.  prerot: B pre-rotated by the client (steps 2-3,
    four primes); otherwise step 1 runs on the server first (five primes).  schedule 1 is the
    BSGS schedule (baby / giant inner rotations, giant rotations postponed into step 3; step 1
    split into baby and giant rotations), with a ragged L and d among its cases."""
    from paper_2508_19525_amd import workloads as wl
    c3s = request.getfixturevalue("c3s" if prerot else "c5p")
    r = _cc_case(c3s, heads, L, d, heads + L, outputs, prerot, schedule)
    h0 = 0
    for O_want, outs, grp in r["want"]:
        sel = range(grp["n_out"]) if outs is None else outs
        for o in sel:
            got = c3s.export(r["C"][_out_index(r["info"], grp, o)])
            assert np.array_equal(got, O_want[o]), f"group H={grp['H']} output {o}"
        if outs is None:
            vecs = []
            for o in range(grp["n_out"]):
                ct = r["C"][_out_index(r["info"], grp, o)]
                pt = c3s.pt_dev(0)
                c3s.B.blb_decrypt(c3s.h, r["keys_g"], ct, pt)
                vecs.append(c3s.B.blb_decode(c3s.h, pt, 0, ct.scale, c3s.n // 2))
            Cs = wl.unpack_diag(vecs, grp["H"], L, c3s.n // 2)
            for h in range(grp["H"]):
                ref = r["Q"][h0 + h] @ r["Kt"][h0 + h]
                assert np.abs(Cs[h] - ref).max() < 2.0 ** -20
        h0 += grp["H"]
    c3s.B.blb_plan_destroy(r["plan"])
    c3s.B.blb_keys_destroy(r["keys_g"])


def _out_index(info, grp, o):
    base = 0
    for g in info["groups"]:
        if g is grp or g == grp:
            return base + o
        base += g["n_out"]
    raise AssertionError


# --------------------------------------------------------------------------------------
# graph executors: every replay equals the eager result
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("fmt", [0, 1])
def test_exec_cp_replays_match_eager(c2s, fmt):
    """Graph replays of a matmul_cp + mask-to-share executor equal eager calls with the same mask
    seeds, with the plan's plaintexts as 64-bit words (fmt 0) or in the 50-bit format (fmt 1); the
    50-bit plan's words also equal those of a 64-bit plan of the same weight."""
    B = c2s.B
    L, d_in, d_out, level = 64, 96, 64, 2
    B.blb_ctx_set_knob(c2s.h, B.BLB_KNOB_PLAN_FORMAT, fmt)
    try:
        r = _cp_case(c2s, L, d_in, d_out, level, 77, x_std=1.0)
    finally:
        B.blb_ctx_set_knob(c2s.h, B.BLB_KNOB_PLAN_FORMAT, 0)
    n_out = r["g"]["n_out"]
    if fmt:
        plan64 = B.blb_plan_matmul_cp(c2s.h, r["W"], L, level)
        Y64 = [c2s.ct(level - 1) for _ in range(n_out)]
        B.blb_matmul_cp(c2s.h, r["keys_g"], plan64, _xcts(c2s, r, level), Y64)
        for b in range(n_out):
            assert np.array_equal(c2s.export(r["Yc"][b]), c2s.export(Y64[b])), f"50-bit plan against 64-bit plan, output {b}"
        B.blb_plan_destroy(plan64)
    Ye = [c2s.ct(level - 1) for _ in range(n_out)]
    Yg = [c2s.ct(level - 1) for _ in range(n_out)]
    share_e = torch.zeros(n_out * level * c2s.n, dtype=torch.int64, device="cuda")
    share_g = torch.zeros_like(share_e)
    ex = B.blb_exec_create_cp(c2s.h, r["keys_g"], r["plan"], _xcts(c2s, r, level), Yg, level - 1, share_g)
    for rep, seed in enumerate([5, 6, 5]):
        B.blb_exec_run(ex, seed)
        torch.cuda.synchronize()
        got = [c2s.export(y) for y in Yg]
        got_share = share_g.cpu().numpy().copy()
        # eager work between replays
        B.blb_matmul_cp(c2s.h, r["keys_g"], r["plan"], _xcts(c2s, r, level), Ye)
        B.blb_mask_to_share(c2s.h, Ye, seed, level - 1, share_e)
        torch.cuda.synchronize()
        for b in range(n_out):
            assert np.array_equal(got[b], c2s.export(Ye[b])), f"replay {rep} output {b}"
        assert np.array_equal(got_share, share_e.cpu().numpy()), f"replay {rep} share"
    B.blb_exec_destroy(ex)
    B.blb_plan_destroy(r["plan"])
    B.blb_keys_destroy(r["keys_g"])


def test_exec_two_executors_on_two_streams(c2s):
    """Two executors of one plan (own scratch, own outputs) replayed alternately on two streams
    overlap on the device; every output equals an eager run with the same mask seed."""
    B = c2s.B
    L, d_in, d_out, level = 64, 96, 64, 2
    r = _cp_case(c2s, L, d_in, d_out, level, 78, x_std=1.0)
    n_out = r["g"]["n_out"]
    Ys = [[c2s.ct(level - 1) for _ in range(n_out)] for _ in range(2)]
    shares = [torch.zeros(n_out * level * c2s.n, dtype=torch.int64, device="cuda") for _ in range(2)]
    exs = [B.blb_exec_create_cp(c2s.h, r["keys_g"], r["plan"], _xcts(c2s, r, level), Ys[e], level - 1, shares[e]) for e in range(2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    last = {}
    for k in range(7):
        last[k % 2] = 900 + k
        B.blb_exec_run_stream(exs[k % 2], last[k % 2], streams[k % 2].cuda_stream)
    torch.cuda.synchronize()
    for e in range(2):
        Ye = [c2s.ct(level - 1) for _ in range(n_out)]
        she = torch.zeros_like(shares[e])
        B.blb_matmul_cp(c2s.h, r["keys_g"], r["plan"], _xcts(c2s, r, level), Ye)
        B.blb_mask_to_share(c2s.h, Ye, last[e], level - 1, she)
        torch.cuda.synchronize()
        for b in range(n_out):
            assert np.array_equal(c2s.export(Ys[e][b]), c2s.export(Ye[b])), f"executor {e} output {b}"
        assert np.array_equal(shares[e].cpu().numpy(), she.cpu().numpy()), f"executor {e} share"
    for ex in exs:
        B.blb_exec_destroy(ex)


def _xcts(c, r, level):
    if "_xc" not in r:
        xs = []
        for a in range(r["g"]["n_in"]):
            ct = c.import_ct(r["X_words"][a], level)
            ct.scale = r["scale"]
            xs.append(ct)
        r["_xc"] = xs
    return r["_xc"]


@pytest.mark.parametrize("schedule", [0, 1])
def test_exec_cc_replays_match_eager(c3s, schedule):
    B = c3s.B
    r = _cc_case(c3s, 8, 32, 32, 3, schedule=schedule)
    n_out = r["info"]["n_out"]
    Cg = [c3s.ct(r["level"] - 3) for _ in range(n_out)]
    ex = B.blb_exec_create_cc(c3s.h, r["keys_g"], r["plan"], r["A"], r["B"], Cg)
    for rep in range(3):
        B.blb_exec_run(ex, 0)
        torch.cuda.synchronize()
        got = [c3s.export(x) for x in Cg]
        B.blb_matmul_cc(c3s.h, r["keys_g"], r["plan"], r["A"], r["B"], r["C"])
        torch.cuda.synchronize()
        for o in range(n_out):
            assert np.array_equal(got[o], c3s.export(r["C"][o])), f"replay {rep} output {o}"
    B.blb_exec_destroy(ex)


# --------------------------------------------------------------------------------------
# launch-shape knobs never change a bit
# --------------------------------------------------------------------------------------
def test_ntt_variants_bit_identical(c3s):
    """Every NTT launch shape -- one workgroup per poly or the persistent pipelined grid (knob
    NTT_VARIANT), 16 or 32 values per work-item (knob NTT_RADIX) -- gives identical words through a
    full matmul_cc (rotations, rescales and ModDowns at three levels), equal to the oracle's."""
    B = c3s.B
    r = _cc_case(c3s, 8, 32, 32, 11)
    base = [c3s.export(x) for x in r["C"]]
    default = (B.blb_ctx_get_knob(c3s.h, B.BLB_KNOB_NTT_VARIANT), B.blb_ctx_get_knob(c3s.h, B.BLB_KNOB_NTT_RADIX))
    try:
        for variant in (0, 1):
            for radix in (16, 32):
                B.blb_ctx_set_knob(c3s.h, B.BLB_KNOB_NTT_VARIANT, variant)
                B.blb_ctx_set_knob(c3s.h, B.BLB_KNOB_NTT_RADIX, radix)
                C2 = [c3s.ct(r["level"] - 3) for _ in range(len(r["C"]))]
                B.blb_matmul_cc(c3s.h, r["keys_g"], r["plan"], r["A"], r["B"], C2)
                for o in range(len(C2)):
                    assert np.array_equal(c3s.export(C2[o]), base[o]), f"variant {variant} radix {radix} output {o}"
        for o in range(len(r["want"][0][0])):
            assert np.array_equal(base[o], r["want"][0][0][o])
    finally:
        B.blb_ctx_set_knob(c3s.h, B.BLB_KNOB_NTT_VARIANT, default[0])
        B.blb_ctx_set_knob(c3s.h, B.BLB_KNOB_NTT_RADIX, default[1])
    B.blb_plan_destroy(r["plan"])
    B.blb_keys_destroy(r["keys_g"])


@pytest.mark.parametrize("ks_variant", [0, 2])
def test_ks_variants_bit_identical(c3s, c2s, ks_variant):
    """The per-output key inner product (knob 0) and the key-grouped one forced on every batch
    (knob 2: outputs sharing a key and Galois element in one thread, groups of up to 16, here with
    many outputs per group -- the BSGS ct-ct product's baby steps over several operand ciphertexts and
    its relinearisations, the cp baby steps across inputs) give the oracle's words through a full
    matmul_cc and through matmul_cp."""
    B = c3s.B
    for c, run in ((c3s, "cc"), (c2s, "cp")):
        default = B.blb_ctx_get_knob(c.h, B.BLB_KNOB_KS_VARIANT)
        B.blb_ctx_set_knob(c.h, B.BLB_KNOB_KS_VARIANT, ks_variant)
        try:
            if run == "cc":
                r = _cc_case(c, 12, 64, 32, 21, outputs=[0, 1], schedule=1)
                base = 0
                for O_want, outs, grp in r["want"]:
                    for o in outs:
                        assert np.array_equal(c.export(r["C"][base + o]), O_want[o]), f"cc group H={grp['H']} output {o}"
                    base += grp["n_out"]
                B.blb_plan_destroy(r["plan"])
            else:
                r = _cp_case(c, 100, 96, 80, 2, 7, x_std=1.0)
                want = r["keys_o"].matmul_cp(r["X_words"], 2, r["W"], 100)
                for b in range(r["g"]["n_out"]):
                    assert np.array_equal(c.export(r["Yc"][b]), want[b]), f"cp output {b}"
                B.blb_plan_destroy(r["plan"])
            B.blb_keys_destroy(r["keys_g"])
        finally:
            B.blb_ctx_set_knob(c.h, B.BLB_KNOB_KS_VARIANT, default)


@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("shape", [(64, 96, 64), (20, 1, 24)])
def test_mac_variants_bit_identical(c2s, shape, fmt):
    """Every MAC launch shape gives the oracle's words, with the plan's plaintexts held as 64-bit
    words (fmt 0) or in the 50-bit format (fmt 1); the second shape has a single rotated input, so
    the unrolled variants run their remainder loop, and a partial last output tile.  The plan takes
    8N or 25N/4 bytes per limb-poly, and the MAC counts that many plaintext bytes."""
    B = c2s.B
    B.blb_ctx_set_knob(c2s.h, B.BLB_KNOB_PLAN_FORMAT, fmt)
    try:
        assert B.blb_ctx_get_knob(c2s.h, B.BLB_KNOB_PLAN_FORMAT) == fmt
        B.blb_ctx_counters(c2s.h, reset=True)
        r = _cp_case(c2s, *shape, 2, 5, x_std=1.0)
        plaintext_bytes = B.blb_ctx_counters(c2s.h)["plaintext_bytes"]
    finally:
        B.blb_ctx_set_knob(c2s.h, B.BLB_KNOB_PLAN_FORMAT, 0)
    g = r["g"]
    n_pt = g["n_out"] * g["G"] * g["n_in"] * g["B"]
    poly_bytes = c2s.n * 25 // 4 if fmt else c2s.n * 8
    assert plaintext_bytes == n_pt * 3 * poly_bytes
    base = [c2s.export(y) for y in r["Yc"]]
    want = r["keys_o"].matmul_cp(r["X_words"], 2, r["W"], shape[0])
    assert all(np.array_equal(base[b], want[b]) for b in range(len(base)))
    Xc = _xcts(c2s, r, 2)
    for var in range(B.BLB_MAC_VARIANTS):
        B.blb_ctx_set_knob(c2s.h, B.BLB_KNOB_MAC_VARIANT, var)
        Y = [c2s.ct(1) for _ in range(len(base))]
        B.blb_matmul_cp(c2s.h, r["keys_g"], r["plan"], Xc, Y)
        for b in range(len(Y)):
            assert np.array_equal(c2s.export(Y[b]), base[b]), f"variant {var}"
    B.blb_ctx_set_knob(c2s.h, B.BLB_KNOB_MAC_VARIANT, 0)
    torch.cuda.synchronize()
    held = B.blb_ctx_device_bytes(c2s.h)
    B.blb_plan_destroy(r["plan"])
    assert held - B.blb_ctx_device_bytes(c2s.h) == n_pt * 3 * poly_bytes  # the plan's own allocation
    B.blb_keys_destroy(r["keys_g"])


# --------------------------------------------------------------------------------------
# the batched transform on its own
# --------------------------------------------------------------------------------------
def _brv(log_n):
    j = np.arange(1 << log_n)
    r = np.zeros_like(j)
    for b in range(log_n):
        r |= ((j >> b) & 1) << (log_n - 1 - b)
    return r


@pytest.mark.parametrize("name,n_polys", [("c1", 3), ("c2s", 5), ("c3s", 37)])
@pytest.mark.parametrize("variant,radix", [(0, 16), (1, 16), (0, 32), (1, 32)])
def test_ntt_matches_oracle(request, name, n_polys, variant, radix):
    """blb_ntt: word j of the forward transform is the evaluation at psi^(2 brv(j) + 1), which is
    entry brv(j) of the oracle's natural-order textbook transform; every prime of the chain
    (special primes included); the inverse returns the input exactly; a ragged poly count."""
    c = request.getfixturevalue(name)
    B = c.B
    mods = B.blb_ctx_moduli(c.h, c.n_q + c.n_sp)
    nl = len(mods)
    log_n = int(np.log2(c.n))
    rng = np.random.default_rng(1000 + n_polys)
    words = np.stack([np.stack([rng.integers(0, int(q), c.n, dtype=np.uint64) for q in mods]) for _ in range(n_polys)])
    dev = c.upload_words(words)
    default = (B.blb_ctx_get_knob(c.h, B.BLB_KNOB_NTT_VARIANT), B.blb_ctx_get_knob(c.h, B.BLB_KNOB_NTT_RADIX))
    B.blb_ctx_set_knob(c.h, B.BLB_KNOB_NTT_VARIANT, variant)
    B.blb_ctx_set_knob(c.h, B.BLB_KNOB_NTT_RADIX, radix)
    try:
        B.blb_ntt(c.h, dev, n_polys, nl, inverse=False)
        torch.cuda.synchronize()
        got = dev.cpu().numpy().view(np.uint64).reshape(n_polys, nl, c.n)
        perm = _brv(log_n)
        for p in sorted({0, n_polys - 1}):
            for m in range(nl):
                want = c.o.ntt_forward(m, words[p, m])
                assert np.array_equal(got[p, m], want[perm]), f"poly {p} limb {m}"
        B.blb_ntt(c.h, dev, n_polys, nl, inverse=True)
        torch.cuda.synchronize()
        back = dev.cpu().numpy().view(np.uint64).reshape(n_polys, nl, c.n)
        assert np.array_equal(back, words)
    finally:
        B.blb_ctx_set_knob(c.h, B.BLB_KNOB_NTT_VARIANT, default[0])
        B.blb_ctx_set_knob(c.h, B.BLB_KNOB_NTT_RADIX, default[1])
    with pytest.raises(B.BlbError):
        B.blb_ntt(c.h, dev, 1, nl + 1)
    B.blb_ntt(c.h, dev, 0, 1)
