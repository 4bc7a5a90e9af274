"""Serving runtime: a request's result is the same alone and inside a mix of concurrent
requests of other lengths and operators (word for word), requests are admitted by the
plan-cache budget (eviction, rejection of a plan that can never fit), and latency statistics
are reported."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_19525_amd as B
    from paper_2508_19525_amd import workloads as wl
    ctx = B.blb_ctx_create(13, 3, 1, 3, 0, torch.cuda.current_stream().cuda_stream)
    yield B, wl, ctx
    torch.cuda.synchronize()
    B.blb_ctx_destroy(ctx)


SHAPES = {0: (64, 64), 1: (64, 128), 2: (128, 64)}


def _make_requests(B, wl, ctx, specs, keys, level=2, n=8192, scale=2.0 ** 40, cplx=False):
    """specs: [(weight_id, L, client, input seed)] -> list of dicts with ABI arrays (cplx: output
    arrays sized for the complex-slot output packing)"""
    keep, reqs = [], []
    pt = torch.empty((level + 1) * n, dtype=torch.int64, device="cuda")
    keep.append(pt)
    for wid, L, client, xs in specs:
        d_in, d_out = SHAPES[wid]
        lp = wl.lp_of(L)
        cc = (n // 2) // lp
        n_in, n_out = -(-d_in // cc), -(-d_out // cc)
        if cplx:
            n_out = (n_out + 1) // 2
        X = np.random.default_rng(xs).normal(0, 1, (L, d_in))
        xcts, ycts = [], []
        for a in range(n_in):
            B.blb_encode(ctx, wl.pack_spatial(X, n // 2, a), scale, level, pt)
            ct, t = B.new_ct(n, level)
            keep.append(t)
            B.blb_encrypt(ctx, keys[client], pt, level, scale, 7000 + xs, a, ct)
            xcts.append(ct)
        for b in range(n_out):
            ct, t = B.new_ct(n, level - 1)
            keep.append(t)
            ycts.append(ct)
        share = torch.zeros(n_out * level * n, dtype=torch.int64, device="cuda")
        keep.append(share)
        reqs.append(dict(wid=wid, L=L, client=client, X=(B.blb_ct * n_in)(*xcts), Y=(B.blb_ct * n_out)(*ycts), share=share, Xm=X))
    torch.cuda.synchronize()
    return reqs, keep


def _keys_for_all(B, wl, ctx, n_clients):
    steps = set()
    for wid, (d_in, d_out) in SHAPES.items():
        for lp in (8, 16, 32, 64, 128, 256, 512):
            cc = 4096 // lp
            dp = 1 << int(np.ceil(np.log2(d_in)))
            ce = min(cc, dp)
            Bb = 1 << ((int(np.ceil(np.log2(ce))) + 1) // 2)
            G = ce // Bb
            steps |= {k * lp for k in range(1, Bb)} | {j * Bb * lp for j in range(1, G)}
    return [B.blb_keygen(ctx, 6100 + c, sorted(steps)) for c in range(n_clients)]


@pytest.mark.parametrize("policy,fmt", [(1, 0), (0, 0), (1, 1)])
def test_alone_equals_in_mix(env, policy, fmt):
    """A request served alone and inside a mix gives the same words and share, under either
    admission policy and with the cached plans as 64-bit words (fmt 0) or in the 50-bit format"""
    B, wl, ctx = env
    keys = _keys_for_all(B, wl, ctx, 3)
    specs = [(0, 40, 0, 1)] + [(i % 3, [16, 100, 33, 200, 64, 7, 300][i % 7], i % 3, 10 + i) for i in range(12)]
    reqs, keep = _make_requests(B, wl, ctx, specs, keys)
    Ws = {wid: wl.serving_weights(wid, SHAPES[wid]) for wid in SHAPES}
    # plan budget fits a handful of plans: forces eviction between batches
    B.blb_ctx_set_knob(ctx, B.BLB_KNOB_PLAN_FORMAT, fmt)  # taken by the server at creation
    srv = None
    try:
        srv = B.blb_server_create(ctx, plan_cache_bytes=600 << 20, max_batch=6, n_streams=2, policy=policy, max_wait_ms=50.0)
        for wid, W in Ws.items():
            B.blb_server_add_weights(srv, wid, W, 2)
        r0 = reqs[0]
        rid = B.blb_server_submit(srv, keys[r0["client"]], r0["wid"], r0["L"], r0["X"], r0["Y"], 55, 1, r0["share"])
        B.blb_server_drain(srv, 120)
        st, lat = B.blb_server_poll(srv, rid)
        assert st == 2 and lat > 0
        alone = [B.blb_export(ctx, r0["Y"][b], 8192) for b in range(len(r0["Y"]))]
        alone_share = r0["share"].cpu().numpy().copy()
        ids = []
        for k, r in enumerate(reqs):  # request 0 again, inside the mix
            seed = 55 if k == 0 else 1000 + k
            ids.append(B.blb_server_submit(srv, keys[r["client"]], r["wid"], r["L"], r["X"], r["Y"], seed, 1, r["share"]))
        B.blb_server_drain(srv, 300)
        states = [B.blb_server_poll(srv, rid)[0] for rid in ids]
        assert states == [2] * len(ids), f"request states {states}"
        mix = [B.blb_export(ctx, r0["Y"][b], 8192) for b in range(len(r0["Y"]))]
        for b in range(len(mix)):
            assert np.array_equal(alone[b], mix[b]), f"output {b} differs alone vs in the mix"
        assert np.array_equal(alone_share, r0["share"].cpu().numpy())
        st = B.blb_server_stats(srv)
        assert st["completed"] == len(reqs) + 1 and st["rejected"] == 0
        assert st["plan_misses"] >= 3 and st["batches"] >= 2
        assert st["p99_ms"] >= st["p50_ms"] > 0
        assert st["plan_bytes"] <= 600 << 20
        # every request decodes (after unmasking with its share) to X @ W
        dec = torch.empty(2 * 8192, dtype=torch.int64, device="cuda")
        for r in reqs[1:4]:
            vecs = []
            for b in range(len(r["Y"])):
                B.blb_decrypt(ctx, keys[r["client"]], r["Y"][b], dec)
                d = dec.cpu().numpy().view(np.uint64).reshape(2, 8192).copy()
                sh = r["share"].cpu().numpy().view(np.uint64).reshape(len(r["Y"]), 2, 8192)[b]
                mods = B.blb_ctx_moduli(ctx, 4)
                for i in range(2):
                    q = int(mods[i])
                    d[i] = ((d[i].astype(object) + sh[i].astype(object)) % q).astype(np.uint64)
                t = torch.from_numpy(d.view(np.int64).reshape(-1).copy()).cuda()
                vecs.append(B.blb_decode(ctx, t, 1, r["Y"][b].scale, 4096))
            got = wl.unpack_spatial(vecs, r["L"], SHAPES[r["wid"]][1], 4096)
            assert np.abs(got - r["Xm"] @ Ws[r["wid"]]).max() < 2.0 ** -20
    finally:
        if srv is not None:
            B.blb_server_destroy(srv)
        B.blb_ctx_set_knob(ctx, B.BLB_KNOB_PLAN_FORMAT, 0)
        for k in keys:
            B.blb_keys_destroy(k)


def test_admission_rejects_plan_over_budget(env):
    B, wl, ctx = env
    keys = _keys_for_all(B, wl, ctx, 1)
    reqs, keep = _make_requests(B, wl, ctx, [(1, 500, 0, 3)], keys)
    srv = B.blb_server_create(ctx, plan_cache_bytes=1 << 20, max_batch=4, n_streams=1)
    try:
        B.blb_server_add_weights(srv, 1, wl.serving_weights(1, SHAPES[1]), 2)
        r = reqs[0]
        rid = B.blb_server_submit(srv, keys[0], 1, r["L"], r["X"], r["Y"])
        B.blb_server_drain(srv, 60)
        st, lat = B.blb_server_poll(srv, rid)
        assert st == B.BLB_ENOMEM
        assert B.blb_server_stats(srv)["rejected"] == 1
    finally:
        B.blb_server_destroy(srv)
        for k in keys:
            B.blb_keys_destroy(k)


def test_submit_refuses_request_without_its_keys(env):
    """A request whose keys lack a rotation of its schedule is refused at submission (ENOKEY)
    instead of failing the batch it would have joined; the server keeps serving."""
    B, wl, ctx = env
    keys = _keys_for_all(B, wl, ctx, 1)
    bare = B.blb_keygen(ctx, 98, [])
    reqs, keep = _make_requests(B, wl, ctx, [(0, 40, 0, 4)], keys)
    srv = B.blb_server_create(ctx, plan_cache_bytes=256 << 20, max_batch=4, n_streams=1)
    try:
        B.blb_server_add_weights(srv, 0, wl.serving_weights(0, SHAPES[0]), 2)
        with pytest.raises(B.BlbError):  # registered weights are immutable
            B.blb_server_add_weights(srv, 0, wl.serving_weights(0, SHAPES[0]), 2)
        r = reqs[0]
        with pytest.raises(B.BlbError) as ei:
            B.blb_server_submit(srv, bare, 0, r["L"], r["X"], r["Y"])
        assert ei.value.code == B.BLB_ENOKEY
        rid = B.blb_server_submit(srv, keys[0], 0, r["L"], r["X"], r["Y"])
        B.blb_server_drain(srv, 60)
        assert B.blb_server_poll(srv, rid)[0] == 2
        st = B.blb_server_stats(srv)
        assert st["completed"] == 1 and st["failed"] == 0
    finally:
        B.blb_server_destroy(srv)
        B.blb_keys_destroy(bare)
        for k in keys:
            B.blb_keys_destroy(k)


def test_served_c5_geometry_against_oracle(orc):
    """The serving configuration's own geometry: N = 16384, four primes + two special (dnum 2),
    BERT-large 1024 x 4096 and 4096 x 1024 operators at L = 200 (L' = 256) and a GPT-2-base
    768 x 768 operator at L = 100, submitted together.  Sampled outputs equal the oracle's words
    (SHA-256 of the oracle's outputs written by tests/golden/make_cp_sampled_hashes.py), every
    output decodes to X W in FP64 within 2^-20, and each request run alone afterwards gives the
    words it gave in the mix."""
    import os
    import sys
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_cp_sampled_hashes as gold
    import paper_2508_19525_amd as B
    from paper_2508_19525_amd import workloads as wl
    names = ["c5_1024x4096_L200", "c5_4096x1024_L200", "c5_768x768_L100"]
    table = gold.load()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # the plan cache below is one 150 GiB device allocation
    n, level, scale = 16384, 3, 2.0 ** 40
    ctx = B.blb_ctx_create(14, 4, 2, 2, 0, torch.cuda.current_stream().cuda_stream)
    keep, reqs, keys = [], [], []
    srv = None
    try:
        pt = torch.empty((level + 1) * n, dtype=torch.int64, device="cuda")
        for name in names:
            prm, lvl, L, src, xseed, kseed, eseed, outs = gold.CASES[name]
            assert prm == (14, 4, 2, 2) and lvl == level
            W, X = gold.inputs(name)
            lp = wl.lp_of(L)
            cc = (n // 2) // lp
            d_in, d_out = W.shape
            ce = min(cc, 1 << int(np.ceil(np.log2(d_in))))
            Bb = 1 << ((int(np.ceil(np.log2(ce))) + 1) // 2)
            steps = [k * lp for k in range(1, Bb)] + [j * Bb * lp for j in range(1, ce // Bb)]
            k = B.blb_keygen(ctx, kseed, steps)
            keys.append(k)
            n_in, n_out = -(-d_in // cc), -(-d_out // cc)
            xs = []
            for a in range(n_in):
                B.blb_encode(ctx, wl.pack_spatial(X, n // 2, a), scale, level, pt)
                ct, t = B.new_ct(n, level)
                keep.append(t)
                B.blb_encrypt(ctx, k, pt, level, scale, eseed, a, ct)
                xs.append(ct)
            ys = []
            for b in range(n_out):
                ct, t = B.new_ct(n, level - 1)
                keep.append(t)
                ys.append(ct)
            reqs.append(dict(name=name, wid=src[1], W=W, X=X, L=L, keys=k, Xa=(B.blb_ct * n_in)(*xs), Y=(B.blb_ct * n_out)(*ys),
                             outs=outs))
        torch.cuda.synchronize()
        srv = B.blb_server_create(ctx, plan_cache_bytes=150 << 30, max_batch=4, n_streams=2)
        for r in reqs:
            B.blb_server_add_weights(srv, r["wid"], r["W"], level)
        ids = [B.blb_server_submit(srv, r["keys"], r["wid"], r["L"], r["Xa"], r["Y"]) for r in reqs]
        B.blb_server_drain(srv, 300)
        assert [B.blb_server_poll(srv, i)[0] for i in ids] == [2] * len(ids)
        mix = [[B.blb_export(ctx, y, n) for y in r["Y"]] for r in reqs]
        o = orc.Context(14, 4, 2, 2)
        dec = torch.empty(level * n, dtype=torch.int64, device="cuda")
        for r, words in zip(reqs, mix):
            prm, lvl, L, src, xseed, kseed, eseed, outs = gold.CASES[r["name"]]
            keys_o = orc.Keys(o, kseed, [])
            want0 = keys_o.encrypt(o.encode_rns(o.pack_spatial(r["X"], 0), scale, level), level, eseed, 0)
            assert np.array_equal(B.blb_export(ctx, r["Xa"][0], n), want0), r["name"]
            for b in outs:
                assert gold.words_hash(words[b]) == table[(r["name"], b)], f"{r['name']} output {b}"
            vecs = []
            for y in r["Y"]:
                B.blb_decrypt(ctx, r["keys"], y, dec)
                vecs.append(B.blb_decode(ctx, dec, level - 1, y.scale, n // 2))
            got = wl.unpack_spatial(vecs, r["L"], r["W"].shape[1], n // 2)
            assert np.abs(got - r["X"] @ r["W"]).max() < 2.0 ** -20, r["name"]
        # each request alone (its plan now resident) gives the words it gave in the mix
        for r, words in zip(reqs, mix):
            ys = []
            for b in range(len(r["Y"])):
                ct, t = B.new_ct(n, level - 1)
                keep.append(t)
                ys.append(ct)
            Y2 = (B.blb_ct * len(ys))(*ys)
            rid = B.blb_server_submit(srv, r["keys"], r["wid"], r["L"], r["Xa"], Y2)
            B.blb_server_drain(srv, 300)
            assert B.blb_server_poll(srv, rid)[0] == 2
            for b in range(len(ys)):
                assert np.array_equal(B.blb_export(ctx, Y2[b], n), words[b]), f"{r['name']} output {b} alone vs mix"
    finally:
        if srv is not None:
            B.blb_server_destroy(srv)
        for k in keys:
            B.blb_keys_destroy(k)
        torch.cuda.synchronize()
        B.blb_ctx_destroy(ctx)


@pytest.mark.parametrize("policy", [1, 0])
def test_weights_at_different_levels(env, policy):
    """Two weights registered at different levels: batches hold requests of one level, so a mix of
    both completes, and every request gives the words it gives alone."""
    B, wl, ctx = env
    keys = _keys_for_all(B, wl, ctx, 2)
    hi, keep_hi = _make_requests(B, wl, ctx, [(0, 40, 0, 21), (0, 100, 1, 22), (0, 16, 0, 23)], keys, level=2)
    lo, keep_lo = _make_requests(B, wl, ctx, [(1, 40, 1, 24), (1, 64, 0, 25)], keys, level=1)
    srv = B.blb_server_create(ctx, plan_cache_bytes=1 << 30, max_batch=8, n_streams=2, policy=policy, max_wait_ms=50.0)
    try:
        B.blb_server_add_weights(srv, 0, wl.serving_weights(0, SHAPES[0]), 2)
        B.blb_server_add_weights(srv, 1, wl.serving_weights(1, SHAPES[1]), 1)
        mixed = [hi[0], lo[0], hi[1], lo[1], hi[2]]
        ids = [B.blb_server_submit(srv, keys[r["client"]], r["wid"], r["L"], r["X"], r["Y"]) for r in mixed]
        B.blb_server_drain(srv, 120)
        assert [B.blb_server_poll(srv, i)[0] for i in ids] == [2] * len(ids)
        assert B.blb_server_stats(srv)["failed"] == 0
        words = [[B.blb_export(ctx, y, 8192) for y in r["Y"]] for r in mixed]
        for r, w in zip(mixed, words):
            rid = B.blb_server_submit(srv, keys[r["client"]], r["wid"], r["L"], r["X"], r["Y"])
            B.blb_server_drain(srv, 120)
            assert B.blb_server_poll(srv, rid)[0] == 2
            for b, y in enumerate(r["Y"]):
                assert np.array_equal(B.blb_export(ctx, y, 8192), w[b]), f"weight {r['wid']} L {r['L']} output {b}"
    finally:
        B.blb_server_destroy(srv)
        for k in keys:
            B.blb_keys_destroy(k)


def test_submit_checks_mask_target_and_share(env):
    """A mask target above the outputs' level is refused at submission (ELEVEL), so it cannot fail
    the batch it would join; an undersized share tensor is refused by the binding."""
    B, wl, ctx = env
    keys = _keys_for_all(B, wl, ctx, 1)
    reqs, keep = _make_requests(B, wl, ctx, [(0, 40, 0, 31)], keys)
    srv = B.blb_server_create(ctx, plan_cache_bytes=256 << 20, max_batch=4, n_streams=1)
    try:
        B.blb_server_add_weights(srv, 0, wl.serving_weights(0, SHAPES[0]), 2)
        r = reqs[0]
        big = torch.zeros(len(r["Y"]) * 3 * 8192, dtype=torch.int64, device="cuda")  # room for a level-2 target
        with pytest.raises(B.BlbError) as ei:
            B.blb_server_submit(srv, keys[0], 0, r["L"], r["X"], r["Y"], 5, 2, big)
        assert ei.value.code == B.BLB_ELEVEL
        small = torch.zeros(8, dtype=torch.int64, device="cuda")
        with pytest.raises(B.BlbError) as ei:
            B.blb_server_submit(srv, keys[0], 0, r["L"], r["X"], r["Y"], 5, 1, small)
        assert ei.value.code == B.BLB_EINVAL
        rid = B.blb_server_submit(srv, keys[0], 0, r["L"], r["X"], r["Y"], 5, 1, r["share"])
        B.blb_server_drain(srv, 60)
        assert B.blb_server_poll(srv, rid)[0] == 2
        assert B.blb_server_stats(srv)["rejected"] == 0
    finally:
        B.blb_server_destroy(srv)
        for k in keys:
            B.blb_keys_destroy(k)


def test_complex_packed_weights(env):
    """Weights registered with the complex-slot output packing, the server's plans in the 50-bit
    format: every served request equals the eager matmul_cp on a complex plan of 64-bit words of
    the same weight and length, word for word, and its decoded real / imaginary parts give X W;
    the real-packing output count is refused."""
    B, wl, ctx = env
    keys = _keys_for_all(B, wl, ctx, 2)
    specs = [(i % 3, [16, 100, 33, 200, 64, 300][i % 6], i % 2, 40 + i) for i in range(8)]
    reqs, keep = _make_requests(B, wl, ctx, specs, keys, cplx=True)
    Ws = {wid: wl.serving_weights(wid, SHAPES[wid]) for wid in SHAPES}
    B.blb_ctx_set_knob(ctx, B.BLB_KNOB_PLAN_FORMAT, 1)  # taken by the server at creation
    srv = None
    try:
        srv = B.blb_server_create(ctx, plan_cache_bytes=600 << 20, max_batch=4, n_streams=2, policy=1, max_wait_ms=50.0)
        for wid, W in Ws.items():
            B.blb_server_add_weights(srv, wid, W, 2, cplx=True)
        # the real-packing output count is refused for a complex-packed weight
        real, keep2 = _make_requests(B, wl, ctx, [(1, 64, 0, 99)], keys)
        r = real[0]
        if len(r["Y"]) > 1:
            with pytest.raises(B.BlbError):
                B.blb_server_submit(srv, keys[0], r["wid"], r["L"], r["X"], r["Y"], 1, -1, None)
        ids = [B.blb_server_submit(srv, keys[r["client"]], r["wid"], r["L"], r["X"], r["Y"], 0, -1, None) for r in reqs]
        B.blb_server_drain(srv, 300)
        assert [B.blb_server_poll(srv, i)[0] for i in ids] == [2] * len(ids)
    finally:
        if srv is not None:
            B.blb_server_destroy(srv)
        B.blb_ctx_set_knob(ctx, B.BLB_KNOB_PLAN_FORMAT, 0)
    dec = torch.empty(2 * 8192, dtype=torch.int64, device="cuda")
    for r in reqs:
        plan = B.blb_plan_matmul_cp_cplx(ctx, Ws[r["wid"]], r["L"], 2)
        n_y = len(r["Y"])
        assert B.blb_plan_info(plan)["n_out"] == n_y
        Ye = []
        for b in range(n_y):
            ct, t = B.new_ct(8192, 1)
            keep.append(t)
            Ye.append(ct)
        B.blb_matmul_cp(ctx, keys[r["client"]], plan, list(r["X"]), Ye)
        torch.cuda.synchronize()
        vecs = []
        for b in range(n_y):
            assert np.array_equal(B.blb_export(ctx, r["Y"][b], 8192), B.blb_export(ctx, Ye[b], 8192)), f"output {b}"
            B.blb_decrypt(ctx, keys[r["client"]], r["Y"][b], dec)
            vecs += list(B.blb_decode_cplx(ctx, dec, 1, r["Y"][b].scale, 4096))
        got = wl.unpack_spatial(vecs, r["L"], SHAPES[r["wid"]][1], 4096)
        assert np.abs(got - r["Xm"] @ Ws[r["wid"]]).max() < 2.0 ** -20
        B.blb_plan_destroy(plan)
    for k in keys:
        B.blb_keys_destroy(k)
