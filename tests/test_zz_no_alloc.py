"""The allocation-free rotation (blb_rotate_noalloc) against blb_rotate, word for word.

Its temporaries live in one fixed per-device array that the library holds until the process
ends; two calls in a row (the second with a smaller input, so stale words from the first are in
the array) must both equal the allocating entry point, and an input that needs more than the
array is refused with its output untouched.
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


def _ctx(B, log_n, n_q, n_sp, dnum):
    return B.blb_ctx_create(log_n, n_q, n_sp, dnum, 0, torch.cuda.current_stream().cuda_stream)


def _encrypted(B, h, keys, n, level, seed):
    pt = torch.empty((level + 1) * n, dtype=torch.int64, device="cuda")
    m = np.random.default_rng(seed).normal(0, 1, n // 2)
    B.blb_encode(h, m, 2.0 ** 40, level, pt)
    ct, t = B.new_ct(n, level)
    B.blb_encrypt(h, keys, pt, level, 2.0 ** 40, seed, 0, ct)
    return ct, t


def test_rotate_noalloc_matches_rotate_twice(blb, orc):
    B = blb
    n = 1 << 14
    h = _ctx(B, 14, 4, 2, 2)
    try:
        steps = [128, -3]
        keys = B.blb_keygen(h, 31, steps)
        keys_o = orc.Keys(orc.Context(14, 4, 2, 2), 31, [B.blb_galois_elt(h, s) for s in steps])
        for level, s, seed in ((3, 128, 5), (1, -3, 6)):  # second call: a smaller input
            x, xt = _encrypted(B, h, keys, n, level, seed)
            want, wt = B.new_ct(n, level)
            got, gt = B.new_ct(n, level)
            gt.fill_(-1)
            B.blb_rotate(h, keys, x, s, want)
            B.blb_rotate_noalloc(h, keys, x, s, got)
            torch.cuda.synchronize()
            w = B.blb_export(h, want, n)
            g = B.blb_export(h, got, n)
            assert got.level == level and got.degree == 1 and got.scale == x.scale
            assert np.array_equal(g, w), f"level {level}, steps {s}"
            assert np.array_equal(g, keys_o.rotate(B.blb_export(h, x, n), level, s)), f"oracle, level {level}"
        B.blb_keys_destroy(keys)
    finally:
        torch.cuda.synchronize()
        B.blb_ctx_destroy(h)


def test_rotate_noalloc_refuses_inputs_beyond_its_scratch(blb):
    """Ten primes + two special at dnum 5: the top level needs about 15 MB of temporaries, more
    than the fixed 8 MiB array, and is refused with the output untouched; level 3 fits and equals
    blb_rotate."""
    B = blb
    n = 1 << 14
    h = _ctx(B, 14, 10, 2, 5)
    try:
        keys = B.blb_keygen(h, 33, [1])
        x, xt = _encrypted(B, h, keys, n, 9, 7)
        out, ot = B.new_ct(n, 9)
        ot.fill_(12345)
        with pytest.raises(B.BlbError) as e:
            B.blb_rotate_noalloc(h, keys, x, 1, out)
        assert e.value.code == B.BLB_ETOOBIG
        torch.cuda.synchronize()
        assert bool((ot == 12345).all())
        x3, x3t = _encrypted(B, h, keys, n, 3, 8)
        want, wt = B.new_ct(n, 3)
        got, gt = B.new_ct(n, 3)
        B.blb_rotate(h, keys, x3, 1, want)
        B.blb_rotate_noalloc(h, keys, x3, 1, got)
        torch.cuda.synchronize()
        assert np.array_equal(B.blb_export(h, got, n), B.blb_export(h, want, n))
        B.blb_keys_destroy(keys)
    finally:
        torch.cuda.synchronize()
        B.blb_ctx_destroy(h)
