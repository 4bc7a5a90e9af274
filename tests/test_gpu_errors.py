"""Fault paths forced from the host: malformed arguments, level and scale mismatches, missing
keys and an exhausted HBM budget return their error codes before any work is enqueued, and
the outputs are left untouched."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_19525_amd as B
    ctx = B.blb_ctx_create(12, 2, 1, 2, 0, torch.cuda.current_stream().cuda_stream)
    keys = B.blb_keygen(ctx, 3, [1])
    yield B, ctx, keys
    torch.cuda.synchronize()
    B.blb_keys_destroy(keys)
    B.blb_ctx_destroy(ctx)


def _fresh_ct(B, ctx, keys, level=1, scale=2.0 ** 30):
    n = 4096
    pt = torch.empty((level + 1) * n, dtype=torch.int64, device="cuda")
    B.blb_encode(ctx, np.linspace(-1, 1, 100), scale, level, pt)
    ct, t = B.new_ct(n, level)
    B.blb_encrypt(ctx, keys, pt, level, scale, 1, 0, ct)
    return ct, t


def _code(fn, *a):
    import paper_2508_19525_amd as B
    with pytest.raises(B.BlbError) as e:
        fn(*a)
    return e.value.code


def test_bad_parameters_rejected(env):
    B, ctx, keys = env
    assert _code(B.blb_ctx_create, 11, 2, 1, 2) == B.BLB_EINVAL  # N below the supported range
    assert _code(B.blb_ctx_create, 13, 3, 1, 4) == B.BLB_EINVAL  # dnum > n_q
    assert _code(B.blb_ctx_create, 13, 0, 1, 1) == B.BLB_EINVAL
    # knob values out of range, unknown knobs
    assert _code(B.blb_ctx_set_knob, ctx, B.BLB_KNOB_PLAN_FORMAT, 2) == B.BLB_EINVAL
    assert _code(B.blb_ctx_set_knob, ctx, B.BLB_KNOB_MAC_VARIANT, B.BLB_MAC_VARIANTS) == B.BLB_EINVAL
    assert _code(B.blb_ctx_set_knob, ctx, 8, 0) == B.BLB_EINVAL
    assert B.blb_ctx_get_knob(ctx, B.BLB_KNOB_PLAN_FORMAT) == 0


def test_missing_key_and_untouched_output(env):
    B, ctx, keys = env
    ct, t = _fresh_ct(B, ctx, keys)
    out, to = B.new_ct(4096, 1)
    to.fill_(7)
    torch.cuda.synchronize()
    assert _code(B.blb_rotate, ctx, keys, ct, 3, out) == B.BLB_ENOKEY  # only step 1 was generated
    torch.cuda.synchronize()
    assert bool((to == 7).all())
    # aliasing input and output is rejected
    assert _code(B.blb_rotate, ctx, keys, ct, 1, ct) == B.BLB_EINVAL


def test_level_errors(env):
    B, ctx, keys = env
    ct, t = _fresh_ct(B, ctx, keys, level=0)
    out, to = B.new_ct(4096, 0)
    assert _code(B.blb_rescale, ctx, ct, out) == B.BLB_ELEVEL  # no limb left to drop
    plan = B.blb_plan_matmul_cp(ctx, np.eye(32) * 0.1, 32, 1)
    try:
        y, ty = B.new_ct(4096, 0)
        assert _code(B.blb_matmul_cp, ctx, keys, plan, [ct], [y]) in (B.BLB_ELEVEL, B.BLB_ENOKEY)
    finally:
        B.blb_plan_destroy(plan)
    share = torch.zeros(2 * 4096, dtype=torch.int64, device="cuda")
    assert _code(B.blb_mask_to_share, ctx, [ct], 1, 1, share) == B.BLB_ELEVEL  # target above the level


def test_scale_mismatch(env):
    B, ctx, keys = env
    plan = B.blb_plan_matmul_cp(ctx, np.eye(64)[:, :32] * 0.1, 32, 1)
    try:
        g = B.blb_plan_info(plan)
        assert g["n_in"] == 1
        a, ta = _fresh_ct(B, ctx, keys, scale=2.0 ** 30)
        y, ty = B.new_ct(4096, 0)
        ty.fill_(5)
        # the plan needs keys for its baby/giant steps, which these keys lack
        assert _code(B.blb_matmul_cp, ctx, keys, plan, [a], [y]) == B.BLB_ENOKEY
        torch.cuda.synchronize()
        assert bool((ty == 5).all())
    finally:
        B.blb_plan_destroy(plan)


def test_hbm_budget_exhausted():
    """A context with a small HBM budget refuses plans and keys beyond it (forced from the host)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_19525_amd as B
    ctx = B.blb_ctx_create(13, 3, 1, 3, 0, torch.cuda.current_stream().cuda_stream, 64 << 20)
    try:
        used = B.blb_ctx_device_bytes(ctx)
        assert used < 64 << 20
        assert _code(B.blb_plan_matmul_cp, ctx, np.zeros((768, 768)), 128, 2) == B.BLB_ENOMEM
        assert B.blb_ctx_device_bytes(ctx) == used  # nothing leaked by the failed call
        steps = list(range(1, 60))
        assert _code(B.blb_keygen, ctx, 1, steps) == B.BLB_ENOMEM
        assert B.blb_ctx_device_bytes(ctx) == used
    finally:
        B.blb_ctx_destroy(ctx)


def test_temporaries_reused_and_trimmed(env):
    """Eager calls take their temporaries from the context's per-stream stack: once it has
    grown, repeating a call allocates nothing more, and trimming hands the stack back (the
    next call grows it again and still gives the same words)."""
    B, ctx, keys = env
    ct, t = _fresh_ct(B, ctx, keys)
    outs = []
    used = []
    for _ in range(4):
        out, to = B.new_ct(4096, 1)
        B.blb_rotate(ctx, keys, ct, 1, out)
        torch.cuda.synchronize()
        outs.append(B.blb_export(ctx, out, 4096))
        used.append(B.blb_ctx_device_bytes(ctx))
    assert used[2] == used[3], f"device bytes still changing: {used}"
    B.blb_ctx_trim(ctx)
    assert B.blb_ctx_device_bytes(ctx) < used[3]  # the idle stack was released
    out, to = B.new_ct(4096, 1)
    B.blb_rotate(ctx, keys, ct, 1, out)
    torch.cuda.synchronize()
    for o in outs + [B.blb_export(ctx, out, 4096)]:
        assert np.array_equal(o, outs[0])


def test_attention_and_share_entry_points_reject_bad_arguments(env):
    """The entry points of the attention operators, rotate-and-sum and the share addition refuse
    malformed arguments before enqueuing work, leaving outputs untouched."""
    B, ctx, keys = env
    ct, t = _fresh_ct(B, ctx, keys)
    out, to = B.new_ct(4096, 1)
    to.fill_(9)
    torch.cuda.synchronize()
    # rotate-and-sum: n_blocks not a power of two, a masked broadcast, a width beyond N/2, a missing key
    assert _code(B.blb_rotate_sum, ctx, keys, [ct], [out], 32, 6, 0) == B.BLB_EINVAL
    assert _code(B.blb_rotate_sum, ctx, keys, [ct], [out], 32, 8, 1, True) == B.BLB_EINVAL
    assert _code(B.blb_rotate_sum, ctx, keys, [ct], [out], 1024, 4, 0) == B.BLB_EINVAL
    assert _code(B.blb_rotate_sum, ctx, keys, [ct], [out], 32, 8, 0) == B.BLB_ENOKEY
    torch.cuda.synchronize()
    assert bool((to == 9).all())
    # share addition: ciphertexts at different levels
    c0, t0 = _fresh_ct(B, ctx, keys, level=0)
    share = torch.zeros(2 * 2 * 4096, dtype=torch.int64, device="cuda")
    assert _code(B.blb_add_share, ctx, [ct, c0], share) == B.BLB_ELEVEL
    # a Softmax x V plan below its three levels; a diagonal-input plan with d_v' > L'; a
    # reordered-column plan whose head group needs more columns per ciphertext than L'
    assert _code(B.blb_plan_matmul_cc_sv, ctx, 4, 16, 32, 1) == B.BLB_EINVAL
    assert _code(B.blb_plan_matmul_cp_diag, ctx, np.zeros((128, 8)), 1, 128, 64, 1) == B.BLB_EINVAL
    assert _code(B.blb_plan_matmul_cp_mhp, ctx, np.zeros((8, 16)), 1, 16, 8, 1) == B.BLB_EINVAL


def test_executors_refuse_undersized_share_buffers(env):
    """The binding checks the share tensor of an executor with mask-to-share against the words the
    replays write (n_out (target + 1) N) before recording anything."""
    B, ctx, keys = env
    W = np.random.default_rng(2).normal(0, 0.02, (32, 32))
    plan = B.blb_plan_matmul_cp(ctx, W, 32, 1)
    try:
        x, xt = _fresh_ct(B, ctx, keys)
        y, yt = B.new_ct(4096, 0)
        small = torch.zeros(4096 - 1, dtype=torch.int64, device="cuda")
        assert _code(B.blb_exec_create_cp, ctx, keys, plan, [x], [y], 0, small) == B.BLB_EINVAL
        arr = (B.blb_cp_instance * 1)()
        Xa, Ya = (B.blb_ct * 1)(x), (B.blb_ct * 1)(y)
        arr[0] = B.blb_cp_instance(keys, plan, B.C.cast(Xa, B.C.c_void_p), 1, B.C.cast(Ya, B.C.c_void_p), 1)
        assert _code(B.blb_exec_create_batch_cp, ctx, arr, 0, small) == B.BLB_EINVAL
    finally:
        B.blb_plan_destroy(plan)
