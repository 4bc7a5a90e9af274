"""Identity and Expansion operators on the GPU (element-wise ct-ct / ct-pt addition and
multiplication; scalar addition / multiplication by broadcast and straight after a summation)
against the CPU oracle, word for word, through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env(orc):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_19525_amd as B
    ctx = B.blb_ctx_create(13, 3, 1, 3, 0, torch.cuda.current_stream().cuda_stream)
    o = orc.Context(13, 3, 1, 3)
    blk, D = 32, 128
    steps = []
    st = blk
    while st < blk * D:
        steps += [st, -st]
        st *= 2
    keys = B.blb_keygen(ctx, 71, steps)
    keys_o = orc.Keys(o, 71, sorted({o.galois_elt(x) for x in steps}))
    yield B, ctx, o, keys, keys_o, blk, D
    torch.cuda.synchronize()
    B.blb_keys_destroy(keys)
    B.blb_ctx_destroy(ctx)


N = 8192


def _imp(B, ctx, keep, words, level, scale):
    c, t = B.new_ct(N, level)
    keep.append(t)
    B.blb_import(ctx, np.ascontiguousarray(words, dtype=np.uint64), c)
    c.scale = scale
    return c


def _out(B, keep, level):
    c, t = B.new_ct(N, level)
    keep.append(t)
    return c


def _enc(o, keys_o, v, scale, level, seed, i):
    return keys_o.encrypt(o.encode_rns(v, scale, level), level, seed, i)


def test_elementwise_ops_match_oracle(env):
    B, ctx, o, keys, keys_o, blk, D = env
    rng = np.random.default_rng(5)
    keep = []
    for level in (2, 1):
        scale = 2.0 ** 40
        aw = [_enc(o, keys_o, rng.uniform(-1, 1, N // 2), scale, level, 11, i) for i in range(3)]
        bw = [_enc(o, keys_o, rng.uniform(-1, 1, N // 2), scale, level, 12, i) for i in range(3)]
        mods = [int(q) for q in o.moduli[:level + 1]]
        pw = [np.stack([rng.integers(0, q, N, dtype=np.uint64) for q in mods]) for _ in range(3)]
        pt = torch.from_numpy(np.stack(pw).view(np.int64).reshape(-1).copy()).cuda()
        A = [_imp(B, ctx, keep, w, level, scale) for w in aw]
        Bc = [_imp(B, ctx, keep, w, level, scale) for w in bw]
        outs = {name: [_out(B, keep, level) for _ in range(3)] for name in ("add", "addp", "mulp", "mulr")}
        B.blb_ew_add(ctx, A, Bc, outs["add"])
        B.blb_ew_add_plain(ctx, A, pt, outs["addp"])
        B.blb_ew_mul_plain(ctx, A, pt, 2.0 ** 20, outs["mulp"])
        B.blb_ew_mul_relin(ctx, keys, A, Bc, outs["mulr"])
        torch.cuda.synchronize()
        for i in range(3):
            assert np.array_equal(B.blb_export(ctx, outs["add"][i], N), o.ew_add(aw[i], bw[i], level)), f"add {level} {i}"
            assert np.array_equal(B.blb_export(ctx, outs["addp"][i], N), o.ew_add_plain(aw[i], pw[i], level)), f"add_plain {level} {i}"
            assert np.array_equal(B.blb_export(ctx, outs["mulp"][i], N), o.ew_mul_plain(aw[i], pw[i], level)), f"mul_plain {level} {i}"
            assert np.array_equal(B.blb_export(ctx, outs["mulr"][i], N), keys_o.ew_mul_relin(aw[i], bw[i], level)), f"mul_relin {level} {i}"
        assert outs["mulp"][0].scale == scale * 2.0 ** 20 and outs["mulr"][0].scale == scale * scale
        assert outs["add"][0].level == level and outs["mulr"][0].degree == 1
    # in place (out = the first operand)
    a_inplace = _imp(B, ctx, keep, aw[0], 1, 2.0 ** 40)
    B.blb_ew_add(ctx, [a_inplace], [Bc[0]], [a_inplace])
    torch.cuda.synchronize()
    assert np.array_equal(B.blb_export(ctx, a_inplace, N), o.ew_add(aw[0], bw[0], 1))


@pytest.mark.parametrize("op,from_sum", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_scalar_ops_match_oracle(env, op, from_sum):
    """sadd / smul with a broadcast scalar column, and the fused form straight after a summation,
    word for word against the oracle, and decoded against the closed form.  The rotate-and-sum
    doubles its key-switch noise at each of its log2 D = 7 steps (no noise boost: nothing
    follows that could undo one), about 2^14 x D absolute at these parameters, so the inputs are
    encoded at 2^45 for the 2^-20 decoded bound."""
    B, ctx, o, keys, keys_o, blk, D = env
    rng = np.random.default_rng(op * 2 + from_sum)
    keep = []
    level, scale, S = 2, 2.0 ** 45, N // 2
    idx = np.arange(S)
    a = rng.uniform(-1, 1, (2, S))
    z = rng.uniform(-1, 1, (2, S)) / 16
    if not from_sum:
        z = np.where(idx < blk, z, 0.0)
    aw = [_enc(o, keys_o, a[i], scale, level, 21, i) for i in range(2)]
    zw = [_enc(o, keys_o, z[i], scale, level, 22, i) for i in range(2)]
    A = [_imp(B, ctx, keep, w, level, scale) for w in aw]
    Z = [_imp(B, ctx, keep, w, level, scale) for w in zw]
    out = [_out(B, keep, level) for _ in range(2)]
    B.blb_scalar_op(ctx, keys, A, Z, blk, D, op, from_sum, out)
    torch.cuda.synchronize()
    dec = torch.empty((level + 1) * N, dtype=torch.int64, device="cuda")
    for i in range(2):
        want = keys_o.scalar_op(aw[i], zw[i], level, blk, D, op, from_sum=bool(from_sum))
        assert np.array_equal(B.blb_export(ctx, out[i], N), want), f"ciphertext {i}"
        B.blb_decrypt(ctx, keys, out[i], dec)
        got = B.blb_decode(ctx, dec, level, out[i].scale, S)
        v = sum(z[i][(idx % blk) + k * blk] for k in range(D)) if from_sum else z[i][idx % blk]
        ref = a[i] + v if op == 0 else a[i] * v
        assert np.abs(got - ref).max() < 2.0 ** -20


def test_elementwise_argument_errors(env):
    B, ctx, o, keys, keys_o, blk, D = env
    keep = []
    rng = np.random.default_rng(9)
    a2 = _imp(B, ctx, keep, _enc(o, keys_o, rng.uniform(-1, 1, N // 2), 2.0 ** 40, 2, 31, 0), 2, 2.0 ** 40)
    a1 = _imp(B, ctx, keep, _enc(o, keys_o, rng.uniform(-1, 1, N // 2), 2.0 ** 40, 1, 31, 1), 1, 2.0 ** 40)
    b2 = _imp(B, ctx, keep, _enc(o, keys_o, rng.uniform(-1, 1, N // 2), 2.0 ** 30, 2, 31, 2), 2, 2.0 ** 30)
    out = _out(B, keep, 2)
    for fn, args, code in [(B.blb_ew_add, ([a2], [a1], [out]), B.BLB_ELEVEL), (B.blb_ew_add, ([a2], [b2], [out]), B.BLB_ESCALE),
                           (B.blb_scalar_op, (keys, [a2], [a2], 32, 64, 0, 1, [out]), B.BLB_EINVAL)]:
        with pytest.raises(B.BlbError) as e:
            fn(ctx, *args)
        assert e.value.code == code
    bare = B.blb_keygen(ctx, 3, [])
    with pytest.raises(B.BlbError) as e:
        B.blb_scalar_op(ctx, bare, [a2], [a2], blk, D, 0, 0, [out])
    assert e.value.code == B.BLB_ENOKEY
    B.blb_keys_destroy(bare)
