"""Batched matmul_cp over independent instances (own keys, shared plans, uneven lengths):
batched == per-instance calls, word for word; one instance against the oracle; and the
one-graph-launch executor of the batch replays to the same words."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env(orc):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_19525_amd as B
    from paper_2508_19525_amd import workloads as wl
    ctx = B.blb_ctx_create(13, 3, 1, 3, 0, torch.cuda.current_stream().cuda_stream)
    yield B, wl, ctx
    torch.cuda.synchronize()
    B.blb_ctx_destroy(ctx)


def _build(B, wl, ctx, shapes, level=2, scale=2.0 ** 40):
    n = 8192
    keep, inst, plans = [], [], {}
    Ws = {}
    for i, (L, D) in enumerate(shapes):
        lp = wl.lp_of(L)
        if D not in Ws:
            Ws[D] = wl.batch_weights(D)
        if (D, lp) not in plans:
            plans[(D, lp)] = B.blb_plan_matmul_cp(ctx, Ws[D], lp, level)
        plan = plans[(D, lp)]
        g = B.blb_plan_info(plan)
        steps = [k * g["Lp"] for k in range(1, g["B"])] + [j * g["B"] * g["Lp"] for j in range(1, g["G"])]
        keys = B.blb_keygen(ctx, 900 + i, steps)
        X = wl.batch_activations(i, L, D)
        pt = torch.empty((level + 1) * n, dtype=torch.int64, device="cuda")
        keep.append(pt)
        xs = []
        for a in range(g["n_in"]):
            B.blb_encode(ctx, wl.pack_spatial(X, n // 2, a), scale, level, pt)
            ct, t = B.new_ct(n, level)
            keep.append(t)
            B.blb_encrypt(ctx, keys, pt, level, scale, 4000 + i, a, ct)
            xs.append(ct)
        ys, ys2 = [], []
        for b in range(g["n_out"]):
            ct, t = B.new_ct(n, level - 1)
            keep.append(t)
            ys.append(ct)
            ct2, t2 = B.new_ct(n, level - 1)
            keep.append(t2)
            ys2.append(ct2)
        inst.append(dict(keys=keys, plan=plan, X=xs, Y=ys, Y2=ys2, L=L, D=D, Xm=X, g=g))
    return inst, plans, Ws, keep


def _abi_instances(B, inst, key="Y"):
    arrs = []
    out = (B.blb_cp_instance * len(inst))()
    for k, I in enumerate(inst):
        Xa = (B.blb_ct * len(I["X"]))(*I["X"])
        Ya = (B.blb_ct * len(I[key]))(*I[key])
        arrs += [Xa, Ya]
        out[k] = B.blb_cp_instance(I["keys"], I["plan"], C_cast(Xa), len(I["X"]), C_cast(Ya), len(I[key]))
    return out, arrs


def C_cast(a):
    import ctypes
    return ctypes.cast(a, ctypes.c_void_p)


SHAPES = [(16, 96), (40, 64), (100, 96), (33, 64), (16, 96), (200, 96)]


@pytest.mark.parametrize("fmt", [0, 1])
def test_batched_equals_per_instance(env, fmt):
    """With the plans' plaintexts as 64-bit words (fmt 0) or in the 50-bit format (fmt 1)"""
    B, wl, ctx = env
    B.blb_ctx_set_knob(ctx, B.BLB_KNOB_PLAN_FORMAT, fmt)
    try:
        inst, plans, Ws, keep = _build(B, wl, ctx, SHAPES)
    finally:
        B.blb_ctx_set_knob(ctx, B.BLB_KNOB_PLAN_FORMAT, 0)
    for I in inst:
        B.blb_matmul_cp(ctx, I["keys"], I["plan"], I["X"], I["Y2"])
    arr, hold = _abi_instances(B, inst)
    B.blb_batch_matmul_cp(ctx, arr)
    torch.cuda.synchronize()
    for k, I in enumerate(inst):
        for b in range(len(I["Y"])):
            assert arr[k].Y is not None
            got = B.blb_export(ctx, B.blb_ct.from_address(arr[k].Y + b * B.C.sizeof(B.blb_ct)), 8192)
            want = B.blb_export(ctx, I["Y2"][b], 8192)
            assert np.array_equal(got, want), f"instance {k} output {b}"
    # decoded accuracy of every instance
    for k, I in enumerate(inst):
        vecs = []
        dec = torch.empty(2 * 8192, dtype=torch.int64, device="cuda")
        for b in range(len(I["Y2"])):
            B.blb_decrypt(ctx, I["keys"], I["Y2"][b], dec)
            vecs.append(B.blb_decode(ctx, dec, 1, I["Y2"][b].scale, 4096))
        got = wl.unpack_spatial(vecs, I["L"], I["D"], 4096)
        assert np.abs(got - I["Xm"] @ Ws[I["D"]]).max() < 2.0 ** -20
    # knobs never change bits: MAC shape, persistent grid, limbs per work item
    for var in range(B.BLB_BATCH_VARIANTS):
        B.blb_ctx_set_knob(ctx, B.BLB_KNOB_BATCH_VARIANT, var)
        B.blb_ctx_set_knob(ctx, B.BLB_KNOB_BATCH_GRID, [7, 256, 2048, 100000, 13, 1024, 300, 64, 4096][var])
        B.blb_ctx_set_knob(ctx, B.BLB_KNOB_BATCH_LIMBS, [1, 2, 0, 3, 1, 0, 2, 1, 0][var])
        B.blb_batch_matmul_cp(ctx, arr)
        torch.cuda.synchronize()
        for k, I in enumerate(inst):
            for b in (0, len(I["Y"]) - 1):
                got = B.blb_export(ctx, B.blb_ct.from_address(arr[k].Y + b * B.C.sizeof(B.blb_ct)), 8192)
                assert np.array_equal(got, B.blb_export(ctx, I["Y2"][b], 8192)), f"variant {var} instance {k} output {b}"
    B.blb_ctx_set_knob(ctx, B.BLB_KNOB_BATCH_VARIANT, 0)
    B.blb_ctx_set_knob(ctx, B.BLB_KNOB_BATCH_GRID, 2048)
    B.blb_ctx_set_knob(ctx, B.BLB_KNOB_BATCH_LIMBS, 1)
    # the executor: one graph launch for the batch, every replay equal to the eager words
    share = torch.zeros(sum(len(I["Y"]) for I in inst) * 2 * 8192, dtype=torch.int64, device="cuda")
    ex = B.blb_exec_create_batch_cp(ctx, arr, 1, share)
    for rep in range(2):
        B.blb_exec_run(ex, 77 + rep)
        torch.cuda.synchronize()
        got = [B.blb_export(ctx, B.blb_ct.from_address(arr[k].Y + b * B.C.sizeof(B.blb_ct)), 8192)
               for k, I in enumerate(inst) for b in range(len(I["Y"]))]
        sh = share.cpu().numpy().copy()
        # eager reference with the same concatenated mask call
        for I in inst:
            B.blb_matmul_cp(ctx, I["keys"], I["plan"], I["X"], I["Y2"])
        flat = [y for I in inst for y in I["Y2"]]
        share2 = torch.zeros_like(share)
        B.blb_mask_to_share(ctx, flat, 77 + rep, 1, share2)
        torch.cuda.synchronize()
        for j, y in enumerate(flat):
            assert np.array_equal(got[j], B.blb_export(ctx, y, 8192)), f"replay {rep} output {j}"
        assert np.array_equal(sh, share2.cpu().numpy())
    B.blb_exec_destroy(ex)
    for I in inst:
        B.blb_keys_destroy(I["keys"])
    for p in plans.values():
        B.blb_plan_destroy(p)


def test_batched_instance_matches_oracle(env, orc):
    """One instance of a batch against the oracle (same seeds, same integer inputs)."""
    B, wl, ctx = env
    shapes = [(20, 64), (50, 64)]
    inst, plans, Ws, keep = _build(B, wl, ctx, shapes)
    arr, hold = _abi_instances(B, inst)
    B.blb_batch_matmul_cp(ctx, arr)
    torch.cuda.synchronize()
    o = orc.Context(13, 3, 1, 3)
    I = inst[1]
    g = o.cp_geometry(I["L"], I["D"], I["D"])
    keys_o = orc.Keys(o, 901, o.cp_galois(I["L"], I["D"], I["D"]))
    xw = np.stack([B.blb_export(ctx, x, 8192) for x in I["X"]])
    # the GPU's encryption of X equals the oracle's (so the oracle input is the oracle's own)
    for a in range(g["n_in"]):
        want = keys_o.encrypt(o.encode_rns(o.pack_spatial(I["Xm"], a), 2.0 ** 40, 2), 2, 4001, a)
        assert np.array_equal(xw[a], want)
    want = keys_o.matmul_cp(xw, 2, Ws[I["D"]], wl.lp_of(I["L"]))
    for b in range(g["n_out"]):
        got = B.blb_export(ctx, B.blb_ct.from_address(arr[1].Y + b * B.C.sizeof(B.blb_ct)), 8192)
        assert np.array_equal(got, want[b]), f"output {b}"
    for I in inst:
        B.blb_keys_destroy(I["keys"])
    for p in plans.values():
        B.blb_plan_destroy(p)


def test_batched_refuses_mixed_plan_formats(env):
    """One batched call takes plans of one plaintext format: a 64-bit-word plan beside a 50-bit
    one is refused before any work is enqueued"""
    B, wl, ctx = env
    inst, plans, Ws, keep = _build(B, wl, ctx, [(20, 64), (50, 64)])
    B.blb_ctx_set_knob(ctx, B.BLB_KNOB_PLAN_FORMAT, 1)
    try:
        p50 = B.blb_plan_matmul_cp(ctx, Ws[64], wl.lp_of(50), 2)
    finally:
        B.blb_ctx_set_knob(ctx, B.BLB_KNOB_PLAN_FORMAT, 0)
    inst[1]["plan"] = p50
    arr, hold = _abi_instances(B, inst)
    with pytest.raises(B.BlbError) as e:
        B.blb_batch_matmul_cp(ctx, arr)
    assert e.value.code == B.BLB_EINVAL
    torch.cuda.synchronize()
    for I in inst:
        B.blb_keys_destroy(I["keys"])
    for p in list(plans.values()) + [p50]:
        B.blb_plan_destroy(p)


def test_batched_c4_geometry_against_oracle(env, orc):
    """The batched workload's largest geometry: an instance with L = 500 (L' = 512) and hidden
    1024 at N = 8192, batched with a small hidden-768 instance.  Two sampled outputs equal the
    oracle's words (SHA-256 of the oracle's outputs written by tests/golden/make_cp_sampled_hashes.py,
    since the full oracle product takes minutes), and every output of both instances decodes to
    X W in FP64 within 2^-20."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    import make_cp_sampled_hashes as gold
    B, wl, ctx = env
    n, level, scale = 8192, 2, 2.0 ** 40
    prm, lvl, L, src, xseed, kseed, eseed, outs = gold.CASES["c4_L500_D1024"]
    assert prm == (13, 3, 1, 3) and lvl == level
    table = gold.load()
    W, X = gold.inputs("c4_L500_D1024")
    W2, X2 = wl.batch_weights(768), wl.batch_activations(3, 37, 768)
    keep, inst, hold = [], [], []
    pt = torch.empty((level + 1) * n, dtype=torch.int64, device="cuda")
    for (Wm, Xm, ks, es) in ((W, X, kseed, eseed), (W2, X2, 955, 4955)):
        lp = wl.lp_of(Xm.shape[0])
        plan = B.blb_plan_matmul_cp(ctx, Wm, lp, level)
        g = B.blb_plan_info(plan)
        steps = [k * g["Lp"] for k in range(1, g["B"])] + [j * g["B"] * g["Lp"] for j in range(1, g["G"])]
        keys = B.blb_keygen(ctx, ks, steps)
        xs, ys = [], []
        for a in range(g["n_in"]):
            B.blb_encode(ctx, wl.pack_spatial(Xm, n // 2, a), scale, level, pt)
            ct, t = B.new_ct(n, level)
            keep.append(t)
            B.blb_encrypt(ctx, keys, pt, level, scale, es, a, ct)
            xs.append(ct)
        for b in range(g["n_out"]):
            ct, t = B.new_ct(n, level - 1)
            keep.append(t)
            ys.append(ct)
        inst.append(dict(keys=keys, plan=plan, X=xs, Y=ys, Xm=Xm, W=Wm, g=g))
    assert (inst[0]["g"]["Lp"], inst[0]["g"]["n_in"], inst[0]["g"]["n_out"]) == (512, 128, 128)
    arr, hold = _abi_instances(B, inst)
    B.blb_batch_matmul_cp(ctx, arr)
    torch.cuda.synchronize()
    # the library's encryption of X equals the oracle's, so the hashed oracle outputs share its inputs
    o = orc.Context(*prm)
    keys_o = orc.Keys(o, kseed, [])
    assert np.array_equal(B.blb_export(ctx, inst[0]["X"][0], n),
                          keys_o.encrypt(o.encode_rns(o.pack_spatial(X, 0), scale, level), level, eseed, 0))
    for b in outs:
        got = B.blb_export(ctx, B.blb_ct.from_address(arr[0].Y + b * B.C.sizeof(B.blb_ct)), n)
        assert gold.words_hash(got) == table[("c4_L500_D1024", b)], f"output {b}"
    dec = torch.empty(level * n, dtype=torch.int64, device="cuda")
    for k, I in enumerate(inst):
        vecs = []
        for b in range(I["g"]["n_out"]):
            y = B.blb_ct.from_address(arr[k].Y + b * B.C.sizeof(B.blb_ct))
            B.blb_decrypt(ctx, I["keys"], y, dec)
            vecs.append(B.blb_decode(ctx, dec, level - 1, y.scale, n // 2))
        got = wl.unpack_spatial(vecs, I["Xm"].shape[0], I["W"].shape[1], n // 2)
        assert np.abs(got - I["Xm"] @ I["W"]).max() < 2.0 ** -20, f"instance {k}"
    for I in inst:
        B.blb_keys_destroy(I["keys"])
        B.blb_plan_destroy(I["plan"])
