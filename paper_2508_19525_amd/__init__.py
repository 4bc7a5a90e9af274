"""Python binding of the gfx950 RNS-CKKS engine (``libblb.so``, C ABI in ``include/blb.h``).

Argument marshalling only: every step runs in the HIP library.  Device buffers are torch
tensors (``torch.int64`` viewed as the uint64 residues) or raw device pointers; the context's
HIP stream is passed at creation (torch's current stream by default).  If the shared library
is missing the import of any entry point raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libblb.so")

BLB_OK, BLB_EINVAL, BLB_ELEVEL, BLB_ESCALE, BLB_ENOKEY, BLB_ENOMEM, BLB_EDEVICE, BLB_EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
BLB_ETOOBIG = -8


class BlbError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {status_str(code)} ({code})")
        self.code = code


class blb_ct(C.Structure):
    _fields_ = [("data", C.c_void_p), ("level", C.c_int32), ("degree", C.c_int32), ("scale", C.c_double)]


class blb_cp_instance(C.Structure):
    _fields_ = [("keys", C.c_void_p), ("plan", C.c_void_p), ("X", C.c_void_p), ("n_in", C.c_int), ("Y", C.c_void_p),
                ("n_out", C.c_int)]


class blb_server_config(C.Structure):
    _fields_ = [("plan_cache_bytes", C.c_uint64), ("max_batch", C.c_int), ("max_queue", C.c_int), ("n_streams", C.c_int),
                ("policy", C.c_int), ("max_wait_ms", C.c_double)]


class blb_params(C.Structure):
    _fields_ = [("log_n", C.c_int32), ("n_q", C.c_int32), ("n_special", C.c_int32), ("dnum", C.c_int32),
                ("device", C.c_int32), ("stream", C.c_void_p), ("hbm_budget_bytes", C.c_uint64)]


_lib = None

_SIGS = {
    "blb_status_str": (C.c_char_p, [C.c_int]),
    "blb_ctx_create": (C.c_int, [C.POINTER(blb_params), C.POINTER(C.c_void_p)]),
    "blb_ctx_destroy": (None, [C.c_void_p]),
    "blb_ctx_moduli": (C.c_int, [C.c_void_p, C.c_void_p]),
    "blb_ctx_device_bytes": (C.c_uint64, [C.c_void_p]),
    "blb_ctx_trim": (C.c_int, [C.c_void_p]),
    "blb_ctx_set_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "blb_ctx_read_timing": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    "blb_ctx_reset_timing": (C.c_int, [C.c_void_p]),
    "blb_ctx_counters": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "blb_ctx_set_knob": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "blb_ctx_get_knob": (C.c_int, [C.c_void_p, C.c_int]),
    "blb_keygen": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p, C.c_int, C.POINTER(C.c_void_p)]),
    "blb_keys_destroy": (None, [C.c_void_p]),
    "blb_galois_elt": (C.c_uint64, [C.c_void_p, C.c_int32]),
    "blb_encode": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_int, C.c_void_p]),
    "blb_encrypt": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_uint64, C.c_uint32,
                              C.POINTER(blb_ct)]),
    "blb_decrypt": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(blb_ct), C.c_void_p]),
    "blb_decode": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_int64]),
    "blb_export": (C.c_int, [C.c_void_p, C.POINTER(blb_ct), C.c_void_p]),
    "blb_import": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(blb_ct)]),
    "blb_rotate": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(blb_ct), C.c_int32, C.POINTER(blb_ct)]),
    "blb_rotate_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(blb_ct), C.c_int32, C.POINTER(blb_ct)]),
    "blb_ew_add": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "blb_ew_add_plain": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "blb_ew_mul_plain": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_double, C.c_void_p]),
    "blb_ew_mul_relin": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "blb_scalar_op": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                C.c_void_p]),
    "blb_rescale": (C.c_int, [C.c_void_p, C.POINTER(blb_ct), C.POINTER(blb_ct)]),
    "blb_ntt": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32]),
    "blb_rerandomize": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(blb_ct), C.c_int, C.c_uint64, C.c_int]),
    "blb_plan_matmul_cp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)]),
    "blb_plan_destroy": (None, [C.c_void_p]),
    "blb_plan_info": (C.c_int, [C.c_void_p, C.c_void_p]),
    "blb_matmul_cp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(blb_ct), C.c_int, C.POINTER(blb_ct), C.c_int]),
    "blb_mask_to_share": (C.c_int, [C.c_void_p, C.POINTER(blb_ct), C.c_int, C.c_uint64, C.c_int, C.c_void_p]),
    "blb_cc_rotations": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int]),
    "blb_plan_matmul_cc": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int32, C.POINTER(C.c_void_p)]),
    "blb_add_share": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "blb_rotate_sum": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "blb_plan_matmul_cc_sv": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int32, C.POINTER(C.c_void_p)]),
    "blb_plan_matmul_cp_mhp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                         C.POINTER(C.c_void_p)]),
    "blb_plan_matmul_cp_diag": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                          C.POINTER(C.c_void_p)]),
    "blb_plan_cc_info": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "blb_plan_matmul_cp_cplx": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_void_p)]),
    "blb_plan_matmul_cp_diag_cplx": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                               C.POINTER(C.c_void_p)]),
    "blb_decode_cplx": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_int64]),
    "blb_cc_rotations_sched": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int32, C.c_int32, C.c_void_p, C.c_int]),
    "blb_plan_matmul_cc_sched": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int32, C.c_int32,
                                           C.POINTER(C.c_void_p)]),
    "blb_plan_matmul_cc_sv_sched": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int32, C.c_int32,
                                              C.POINTER(C.c_void_p)]),
    "blb_matmul_cc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(blb_ct), C.POINTER(blb_ct), C.c_int,
                                C.POINTER(blb_ct), C.c_int]),
    "blb_exec_create_cp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(blb_ct), C.c_int, C.POINTER(blb_ct), C.c_int,
                                     C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "blb_exec_create_cc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(blb_ct), C.POINTER(blb_ct), C.c_int,
                                     C.POINTER(blb_ct), C.c_int, C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "blb_exec_run": (C.c_int, [C.c_void_p, C.c_uint64]),
    "blb_exec_run_stream": (C.c_int, [C.c_void_p, C.c_uint64, C.c_void_p]),
    "blb_batch_matmul_cp": (C.c_int, [C.c_void_p, C.POINTER(blb_cp_instance), C.c_int]),
    "blb_server_create": (C.c_int, [C.c_void_p, C.POINTER(blb_server_config), C.POINTER(C.c_void_p)]),
    "blb_server_add_weights": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "blb_server_add_weights_cplx": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_int]),
    "blb_server_submit": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_int,
                                    C.c_uint64, C.c_int, C.c_void_p, C.POINTER(C.c_int64)]),
    "blb_server_poll": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "blb_server_drain": (C.c_int, [C.c_void_p, C.c_double]),
    "blb_server_stats": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int]),
    "blb_server_destroy": (None, [C.c_void_p]),
    "blb_exec_create_batch_cp": (C.c_int, [C.c_void_p, C.POINTER(blb_cp_instance), C.c_int, C.c_int, C.c_void_p,
                                           C.POINTER(C.c_void_p)]),
    "blb_exec_device_bytes": (C.c_uint64, [C.c_void_p]),
    "blb_exec_destroy": (None, [C.c_void_p]),
}


def lib():
    """Loads libblb.so (built by ``paper_2508_19525_amd.build``); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2508_19525_amd.build.build_lib()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def status_str(code: int) -> str:
    return lib().blb_status_str(code).decode()


def _check(rc, what):
    if rc != BLB_OK:
        raise BlbError(rc, what)


def _ptr(x):
    """device pointer of a torch tensor, or an int"""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _host_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------------------------------
# C ABI, one function per entry point
# ---------------------------------------------------------------------------------------
_CTX_N = {}  # ring degree of each live context, for the buffer-size checks below
_SRV_CTX = {}  # server handle -> its context


def _need(ctx, buf, words, what):
    """A torch tensor passed as device words must hold at least `words` 64-bit words (raw integer
    pointers are taken as given)."""
    if buf is None or isinstance(buf, int) or not hasattr(buf, "numel"):
        return
    if buf.numel() * buf.element_size() < words * 8:
        raise BlbError(BLB_EINVAL, f"{what}: buffer of {buf.numel() * buf.element_size()} bytes, {words * 8} needed")


def blb_ctx_create(log_n, n_q, n_special, dnum, device=0, stream=None, hbm_budget_bytes=0):
    p = blb_params(log_n, n_q, n_special, dnum, device, stream, hbm_budget_bytes)
    out = C.c_void_p()
    _check(lib().blb_ctx_create(C.byref(p), C.byref(out)), "blb_ctx_create")
    _CTX_N[out.value] = 1 << log_n
    return out.value


def blb_ctx_destroy(ctx):
    _CTX_N.pop(ctx, None)
    lib().blb_ctx_destroy(ctx)


def blb_ctx_moduli(ctx, count):
    out = np.zeros(count, np.uint64)
    _check(lib().blb_ctx_moduli(ctx, _host_ptr(out)), "blb_ctx_moduli")
    return out


def blb_ctx_device_bytes(ctx):
    return int(lib().blb_ctx_device_bytes(ctx))


def blb_ctx_trim(ctx):
    _check(lib().blb_ctx_trim(ctx), "blb_ctx_trim")


BLB_T_CP_MAC, BLB_T_NTT, BLB_T_KS_INNER, BLB_T_MODUP, BLB_T_MODDOWN, BLB_T_MASK, BLB_T_EW, BLB_T_CC_TENSOR = range(8)


def blb_ctx_set_timing(ctx, enable):
    _check(lib().blb_ctx_set_timing(ctx, 1 if enable else 0), "blb_ctx_set_timing")


def blb_ctx_read_timing(ctx, kind):
    """(total_ms, launches, units) for one kernel family"""
    ms, n, u = C.c_double(), C.c_int64(), C.c_double()
    _check(lib().blb_ctx_read_timing(ctx, kind, C.byref(ms), C.byref(n), C.byref(u)), "blb_ctx_read_timing")
    return ms.value, n.value, u.value


COUNTER_NAMES = ["key_switches", "ntt_polys", "ct_pt_products", "tensor_products", "relinearisations", "rescaled_cts",
                 "modup_sources", "plaintext_bytes"]


def blb_ctx_counters(ctx, reset=False):
    out = np.zeros(8, np.int64)
    _check(lib().blb_ctx_counters(ctx, _host_ptr(out), 1 if reset else 0), "blb_ctx_counters")
    return dict(zip(COUNTER_NAMES, [int(x) for x in out]))


def blb_ctx_reset_timing(ctx):
    _check(lib().blb_ctx_reset_timing(ctx), "blb_ctx_reset_timing")


BLB_KNOB_MAC_VARIANT, BLB_KNOB_BATCH_VARIANT, BLB_KNOB_BATCH_GRID, BLB_KNOB_NTT_VARIANT, BLB_KNOB_KS_VARIANT = 0, 1, 2, 3, 4
BLB_KNOB_NTT_RADIX, BLB_KNOB_BATCH_LIMBS, BLB_KNOB_PLAN_FORMAT = 5, 6, 7
BLB_MAC_VARIANTS = 18
BLB_BATCH_VARIANTS = 9


def blb_ctx_set_knob(ctx, knob, value):
    _check(lib().blb_ctx_set_knob(ctx, knob, value), "blb_ctx_set_knob")


def blb_ctx_get_knob(ctx, knob):
    return int(lib().blb_ctx_get_knob(ctx, knob))


def blb_keygen(ctx, seed, rot_steps=()):
    steps = np.ascontiguousarray(rot_steps, dtype=np.int32)
    out = C.c_void_p()
    _check(lib().blb_keygen(ctx, seed, _host_ptr(steps) if steps.size else None, int(steps.size), C.byref(out)), "blb_keygen")
    return out.value


def blb_keys_destroy(keys):
    lib().blb_keys_destroy(keys)


def blb_galois_elt(ctx, steps):
    return int(lib().blb_galois_elt(ctx, steps))


def blb_encode(ctx, values, scale, level, pt_dev):
    v = np.ascontiguousarray(values, dtype=np.float64)
    _need(ctx, pt_dev, (level + 1) * _CTX_N.get(ctx, 0), "blb_encode")
    _check(lib().blb_encode(ctx, _host_ptr(v), v.size, float(scale), level, _ptr(pt_dev)), "blb_encode")


def blb_encrypt(ctx, keys, pt_dev, level, scale, seed, ct_id, ct: blb_ct):
    _need(ctx, pt_dev, (level + 1) * _CTX_N.get(ctx, 0), "blb_encrypt")
    _check(lib().blb_encrypt(ctx, keys, _ptr(pt_dev), level, float(scale), seed, ct_id, C.byref(ct)), "blb_encrypt")


def blb_decrypt(ctx, keys, ct: blb_ct, pt_dev):
    _need(ctx, pt_dev, (ct.level + 1) * _CTX_N.get(ctx, 0), "blb_decrypt")
    _check(lib().blb_decrypt(ctx, keys, C.byref(ct), _ptr(pt_dev)), "blb_decrypt")


def blb_decode(ctx, pt_dev, level, scale, n_vals):
    _need(ctx, pt_dev, (level + 1) * _CTX_N.get(ctx, 0), "blb_decode")
    out = np.zeros(n_vals, np.float64)
    _check(lib().blb_decode(ctx, _ptr(pt_dev), level, float(scale), _host_ptr(out), n_vals), "blb_decode")
    return out


def blb_decode_cplx(ctx, pt_dev, level, scale, n_vals):
    """(real parts, imaginary parts) of the first n_vals slots"""
    _need(ctx, pt_dev, (level + 1) * _CTX_N.get(ctx, 0), "blb_decode_cplx")
    re = np.zeros(n_vals, np.float64)
    im = np.zeros(n_vals, np.float64)
    _check(lib().blb_decode_cplx(ctx, _ptr(pt_dev), level, float(scale), _host_ptr(re), _host_ptr(im), n_vals), "blb_decode_cplx")
    return re, im


def blb_export(ctx, ct: blb_ct, n):
    out = np.zeros((ct.degree + 1, ct.level + 1, n), np.uint64)
    _check(lib().blb_export(ctx, C.byref(ct), _host_ptr(out)), "blb_export")
    return out


def blb_import(ctx, words: np.ndarray, ct: blb_ct):
    w = np.ascontiguousarray(words, dtype=np.uint64)
    _check(lib().blb_import(ctx, _host_ptr(w), C.byref(ct)), "blb_import")


def blb_rotate(ctx, keys, ct_in: blb_ct, steps, ct_out: blb_ct):
    _check(lib().blb_rotate(ctx, keys, C.byref(ct_in), steps, C.byref(ct_out)), "blb_rotate")


def blb_rotate_noalloc(ctx, keys, ct_in: blb_ct, steps, ct_out: blb_ct):
    """blb_rotate with every temporary in the library's fixed per-device scratch (allocates nothing)"""
    _check(lib().blb_rotate_noalloc(ctx, keys, C.byref(ct_in), steps, C.byref(ct_out)), "blb_rotate_noalloc")


def _cts_call(fn, what, out_cts, *args):
    """call fn with blb_ct arrays; copies the outputs' (level, degree, scale) back"""
    arrs = [(blb_ct * len(a))(*a) if isinstance(a, (list, tuple)) else a for a in args]
    oa = (blb_ct * len(out_cts))(*out_cts)
    _check(fn(*[C.cast(a, C.c_void_p) if isinstance(a, C.Array) else a for a in arrs], C.cast(oa, C.c_void_p)), what)
    for i in range(len(out_cts)):
        out_cts[i].level, out_cts[i].degree, out_cts[i].scale = oa[i].level, oa[i].degree, oa[i].scale


def blb_ew_add(ctx, a_cts, b_cts, out_cts):
    _cts_call(lambda *x: lib().blb_ew_add(ctx, x[0], x[1], len(a_cts), x[2]), "blb_ew_add", out_cts, a_cts, b_cts)


def blb_ew_add_plain(ctx, a_cts, pt_dev, out_cts):
    if a_cts:
        _need(ctx, pt_dev, len(a_cts) * (a_cts[0].level + 1) * _CTX_N.get(ctx, 0), "blb_ew_add_plain")
    _cts_call(lambda *x: lib().blb_ew_add_plain(ctx, x[0], len(a_cts), _ptr(pt_dev), x[1]), "blb_ew_add_plain", out_cts, a_cts)


def blb_ew_mul_plain(ctx, a_cts, pt_dev, pt_scale, out_cts):
    if a_cts:
        _need(ctx, pt_dev, len(a_cts) * (a_cts[0].level + 1) * _CTX_N.get(ctx, 0), "blb_ew_mul_plain")
    _cts_call(lambda *x: lib().blb_ew_mul_plain(ctx, x[0], len(a_cts), _ptr(pt_dev), float(pt_scale), x[1]), "blb_ew_mul_plain",
              out_cts, a_cts)


def blb_ew_mul_relin(ctx, keys, a_cts, b_cts, out_cts):
    _cts_call(lambda *x: lib().blb_ew_mul_relin(ctx, keys, x[0], x[1], len(a_cts), x[2]), "blb_ew_mul_relin", out_cts, a_cts, b_cts)


def blb_scalar_op(ctx, keys, a_cts, s_cts, block, n_blocks, op, from_sum, out_cts):
    """op 0: a + V, 1: a x V (relinearised); V = broadcast of s's first block, or (from_sum) the
    unmasked rotate-and-sum of s"""
    _cts_call(lambda *x: lib().blb_scalar_op(ctx, keys, x[0], x[1], len(a_cts), block, n_blocks, op, 1 if from_sum else 0, x[2]),
              "blb_scalar_op", out_cts, a_cts, s_cts)


def blb_rescale(ctx, ct_in: blb_ct, ct_out: blb_ct):
    _check(lib().blb_rescale(ctx, C.byref(ct_in), C.byref(ct_out)), "blb_rescale")


def blb_ntt(ctx, data_dev, n_polys, n_limbs, inverse=False):
    """In-place batched NTT of device words [n_polys][n_limbs][N] (int64 tensor or pointer)."""
    _need(ctx, data_dev, n_polys * n_limbs * _CTX_N.get(ctx, 0), "blb_ntt")
    _check(lib().blb_ntt(ctx, _ptr(data_dev), n_polys, n_limbs, 1 if inverse else 0), "blb_ntt")


def blb_plan_matmul_cp(ctx, W: np.ndarray, L, level):
    Wc = np.ascontiguousarray(W, dtype=np.float64)
    out = C.c_void_p()
    _check(lib().blb_plan_matmul_cp(ctx, _host_ptr(Wc), Wc.shape[0], Wc.shape[1], L, level, C.byref(out)), "blb_plan_matmul_cp")
    return out.value


def blb_plan_matmul_cp_cplx(ctx, W: np.ndarray, L, level):
    """complex-slot output packing: output b holds column blocks 2b and 2b + 1"""
    Wc = np.ascontiguousarray(W, dtype=np.float64)
    out = C.c_void_p()
    _check(lib().blb_plan_matmul_cp_cplx(ctx, _host_ptr(Wc), Wc.shape[0], Wc.shape[1], L, level, C.byref(out)),
           "blb_plan_matmul_cp_cplx")
    return out.value


def blb_plan_destroy(plan):
    lib().blb_plan_destroy(plan)


def blb_plan_info(plan):
    out = np.zeros(8, np.int32)
    _check(lib().blb_plan_info(plan, _host_ptr(out)), "blb_plan_info")
    return dict(zip(["Lp", "c", "c_eff", "c_out", "n_in", "n_out", "B", "G"], [int(x) for x in out]))


def blb_matmul_cp(ctx, keys, plan, X_cts, Y_cts):
    Xa = (blb_ct * len(X_cts))(*X_cts)
    Ya = (blb_ct * len(Y_cts))(*Y_cts)
    _check(lib().blb_matmul_cp(ctx, keys, plan, Xa, len(X_cts), Ya, len(Y_cts)), "blb_matmul_cp")
    for i in range(len(Y_cts)):
        Y_cts[i].level, Y_cts[i].degree, Y_cts[i].scale = Ya[i].level, Ya[i].degree, Ya[i].scale


def blb_mask_to_share(ctx, cts, seed, target_level, share_dev):
    _need(ctx, share_dev, len(cts) * (target_level + 1) * _CTX_N.get(ctx, 0), "blb_mask_to_share")
    arr = (blb_ct * len(cts))(*cts)
    _check(lib().blb_mask_to_share(ctx, arr, len(cts), seed, target_level, _ptr(share_dev)), "blb_mask_to_share")
    for i in range(len(cts)):
        cts[i].level = arr[i].level


def blb_add_share(ctx, cts, share_dev):
    if cts:
        _need(ctx, share_dev, len(cts) * (cts[0].level + 1) * _CTX_N.get(ctx, 0), "blb_add_share")
    arr = (blb_ct * len(cts))(*cts)
    _check(lib().blb_add_share(ctx, arr, len(cts), _ptr(share_dev)), "blb_add_share")


def blb_rotate_sum(ctx, keys, in_cts, out_cts, block, n_blocks, direction=0, mask=None):
    """rotate-and-sum summation (direction 0, first-block mask unless mask=False) or broadcast"""
    if mask is None:
        mask = direction == 0
    ia = (blb_ct * len(in_cts))(*in_cts)
    oa = (blb_ct * len(out_cts))(*out_cts)
    if len(in_cts) != len(out_cts):
        raise BlbError(BLB_EINVAL, "blb_rotate_sum")
    _check(lib().blb_rotate_sum(ctx, keys, ia, len(in_cts), block, n_blocks, direction, 1 if mask else 0, oa), "blb_rotate_sum")
    for i in range(len(out_cts)):
        out_cts[i].level, out_cts[i].degree, out_cts[i].scale = oa[i].level, oa[i].degree, oa[i].scale


def blb_rerandomize(ctx, keys, cts, seed, flood_bits):
    arr = (blb_ct * len(cts))(*cts)
    _check(lib().blb_rerandomize(ctx, keys, arr, len(cts), seed, flood_bits), "blb_rerandomize")


def blb_cc_rotations(ctx, n_heads, L, schedule=0, b_prerotated=True):
    """Rotation steps matmul_cc needs (schedule 0: plain, 1: BSGS; b_prerotated=False adds the
    server-side step 1's steps)"""
    pre = 1 if b_prerotated else 0
    k = lib().blb_cc_rotations_sched(ctx, n_heads, L, pre, schedule, None, 0)
    if k < 0:
        raise BlbError(k, "blb_cc_rotations")
    out = np.zeros(max(k, 1), np.int32)
    _check(0 if lib().blb_cc_rotations_sched(ctx, n_heads, L, pre, schedule, _host_ptr(out), k) >= 0 else BLB_EINVAL,
           "blb_cc_rotations")
    return [int(x) for x in out[:k]]


def blb_plan_matmul_cc(ctx, n_heads, L, d_head, level, b_prerotated=True, schedule=0):
    out = C.c_void_p()
    _check(lib().blb_plan_matmul_cc_sched(ctx, n_heads, L, d_head, level, 1 if b_prerotated else 0, schedule, C.byref(out)),
           "blb_plan_matmul_cc")
    return out.value


def blb_plan_matmul_cc_sv(ctx, n_heads, L, d_v, level, b_prerotated=True, schedule=0):
    out = C.c_void_p()
    _check(lib().blb_plan_matmul_cc_sv_sched(ctx, n_heads, L, d_v, level, 1 if b_prerotated else 0, schedule, C.byref(out)),
           "blb_plan_matmul_cc_sv")
    return out.value


def blb_plan_matmul_cp_mhp(ctx, W: np.ndarray, n_heads, d_head, L, level):
    Wc = np.ascontiguousarray(W, dtype=np.float64)
    if Wc.shape[1] != n_heads * d_head:
        raise BlbError(BLB_EINVAL, "blb_plan_matmul_cp_mhp")
    out = C.c_void_p()
    _check(lib().blb_plan_matmul_cp_mhp(ctx, _host_ptr(Wc), Wc.shape[0], n_heads, d_head, L, level, C.byref(out)),
           "blb_plan_matmul_cp_mhp")
    return out.value


def blb_plan_matmul_cp_diag(ctx, W: np.ndarray, n_heads, d_v, L, level):
    Wc = np.ascontiguousarray(W, dtype=np.float64)
    if Wc.shape[0] != n_heads * d_v:
        raise BlbError(BLB_EINVAL, "blb_plan_matmul_cp_diag")
    out = C.c_void_p()
    _check(lib().blb_plan_matmul_cp_diag(ctx, _host_ptr(Wc), n_heads, d_v, Wc.shape[1], L, level, C.byref(out)),
           "blb_plan_matmul_cp_diag")
    return out.value


def blb_plan_matmul_cp_diag_cplx(ctx, W: np.ndarray, n_heads, d_v, L, level):
    Wc = np.ascontiguousarray(W, dtype=np.float64)
    if Wc.shape[0] != n_heads * d_v:
        raise BlbError(BLB_EINVAL, "blb_plan_matmul_cp_diag_cplx")
    out = C.c_void_p()
    _check(lib().blb_plan_matmul_cp_diag_cplx(ctx, _host_ptr(Wc), n_heads, d_v, Wc.shape[1], L, level, C.byref(out)),
           "blb_plan_matmul_cp_diag_cplx")
    return out.value


def blb_plan_cc_info(plan):
    buf = np.zeros(64, np.int32)
    ng = lib().blb_plan_cc_info(plan, _host_ptr(buf), 64)
    if ng < 0:
        raise BlbError(ng, "blb_plan_cc_info")
    groups = [dict(zip(["H", "c", "n_ct", "n_out", "ct0"], [int(x) for x in buf[3 + 5 * i: 8 + 5 * i]])) for i in range(ng)]
    return {"Lp": int(buf[0]), "n_ct": int(buf[1]), "n_out": int(buf[2]), "groups": groups}


def blb_matmul_cc(ctx, keys, plan, A_cts, Bp_cts, C_cts):
    Aa = (blb_ct * len(A_cts))(*A_cts)
    Ba = (blb_ct * len(Bp_cts))(*Bp_cts)
    Ca = (blb_ct * len(C_cts))(*C_cts)
    _check(lib().blb_matmul_cc(ctx, keys, plan, Aa, Ba, len(A_cts), Ca, len(C_cts)), "blb_matmul_cc")
    for i in range(len(C_cts)):
        C_cts[i].level, C_cts[i].degree, C_cts[i].scale = Ca[i].level, Ca[i].degree, Ca[i].scale


class Exec:
    """A recorded graph executor; keeps the ctypes arrays it was created with alive."""

    def __init__(self, handle, arrays, outs, out_arr):
        self.h, self._arrays, self._outs, self._out_arr = handle, arrays, outs, out_arr

    def sync_outputs(self):
        for i in range(len(self._outs)):
            self._outs[i].level, self._outs[i].degree, self._outs[i].scale = (
                self._out_arr[i].level, self._out_arr[i].degree, self._out_arr[i].scale)


def _need_share(ctx, share_dev, n_out, mask_target_level, what):
    if mask_target_level >= 0:
        _need(ctx, share_dev, n_out * (mask_target_level + 1) * _CTX_N.get(ctx, 0), what)


def blb_exec_create_cp(ctx, keys, plan, X_cts, Y_cts, mask_target_level=-1, share_dev=None):
    _need_share(ctx, share_dev, len(Y_cts), mask_target_level, "blb_exec_create_cp")
    Xa = (blb_ct * len(X_cts))(*X_cts)
    Ya = (blb_ct * len(Y_cts))(*Y_cts)
    out = C.c_void_p()
    _check(lib().blb_exec_create_cp(ctx, keys, plan, Xa, len(X_cts), Ya, len(Y_cts), mask_target_level, _ptr(share_dev),
                                    C.byref(out)), "blb_exec_create_cp")
    e = Exec(out.value, (Xa,), Y_cts, Ya)
    e.sync_outputs()
    return e


def blb_exec_create_cc(ctx, keys, plan, A_cts, Bp_cts, C_cts, mask_target_level=-1, share_dev=None):
    _need_share(ctx, share_dev, len(C_cts), mask_target_level, "blb_exec_create_cc")
    Aa = (blb_ct * len(A_cts))(*A_cts)
    Ba = (blb_ct * len(Bp_cts))(*Bp_cts)
    Ca = (blb_ct * len(C_cts))(*C_cts)
    out = C.c_void_p()
    _check(lib().blb_exec_create_cc(ctx, keys, plan, Aa, Ba, len(A_cts), Ca, len(C_cts), mask_target_level, _ptr(share_dev),
                                    C.byref(out)), "blb_exec_create_cc")
    e = Exec(out.value, (Aa, Ba), C_cts, Ca)
    e.sync_outputs()
    return e


def blb_batch_matmul_cp(ctx, instances):
    """instances: a ctypes array of blb_cp_instance (X / Y point at blb_ct arrays kept alive by the caller)"""
    _check(lib().blb_batch_matmul_cp(ctx, instances, len(instances)), "blb_batch_matmul_cp")


def blb_exec_create_batch_cp(ctx, instances, mask_target_level=-1, share_dev=None):
    _need_share(ctx, share_dev, sum(int(instances[k].n_out) for k in range(len(instances))), mask_target_level,
                "blb_exec_create_batch_cp")
    out = C.c_void_p()
    _check(lib().blb_exec_create_batch_cp(ctx, instances, len(instances), mask_target_level, _ptr(share_dev), C.byref(out)),
           "blb_exec_create_batch_cp")
    return Exec(out.value, (instances,), [], [])


def blb_exec_run(ex, mask_seed=0):
    _check(lib().blb_exec_run(ex.h if isinstance(ex, Exec) else ex, mask_seed), "blb_exec_run")


def blb_exec_run_stream(ex, mask_seed, stream):
    """replay on a given hipStream_t (int handle, e.g. torch.cuda.Stream().cuda_stream)"""
    _check(lib().blb_exec_run_stream(ex.h if isinstance(ex, Exec) else ex, mask_seed, stream), "blb_exec_run_stream")


def blb_exec_device_bytes(ex):
    return int(lib().blb_exec_device_bytes(ex.h if isinstance(ex, Exec) else ex))


def blb_exec_destroy(ex):
    lib().blb_exec_destroy(ex.h if isinstance(ex, Exec) else ex)


SERVE_FIFO, SERVE_RESIDENT_FIRST = 0, 1


def blb_server_create(ctx, plan_cache_bytes, max_batch=16, max_queue=4096, n_streams=2, policy=SERVE_RESIDENT_FIRST,
                      max_wait_ms=1000.0):
    cfg = blb_server_config(plan_cache_bytes, max_batch, max_queue, n_streams, policy, max_wait_ms)
    out = C.c_void_p()
    _check(lib().blb_server_create(ctx, C.byref(cfg), C.byref(out)), "blb_server_create")
    _SRV_CTX[out.value] = ctx
    return out.value


def blb_server_add_weights(server, weight_id, W, level, cplx=False):
    """register W (d_in x d_out); cplx: complex-slot output packing for requests on it"""
    Wc = np.ascontiguousarray(W, dtype=np.float64)
    fn = lib().blb_server_add_weights_cplx if cplx else lib().blb_server_add_weights
    _check(fn(server, weight_id, _host_ptr(Wc), Wc.shape[0], Wc.shape[1], level),
           "blb_server_add_weights_cplx" if cplx else "blb_server_add_weights")


def blb_server_submit(server, keys, weight_id, L, X_arr, Y_arr, mask_seed=0, mask_target_level=-1, share_dev=None):
    """X_arr / Y_arr: ctypes arrays of blb_ct kept alive by the caller until completion"""
    _need_share(_SRV_CTX.get(server), share_dev, len(Y_arr), mask_target_level, "blb_server_submit")
    rid = C.c_int64()
    rc = lib().blb_server_submit(server, keys, weight_id, L, C.cast(X_arr, C.c_void_p), len(X_arr), C.cast(Y_arr, C.c_void_p),
                                 len(Y_arr), mask_seed, mask_target_level, _ptr(share_dev), C.byref(rid))
    _check(rc, "blb_server_submit")
    return rid.value


def blb_server_poll(server, req_id):
    st, lat = C.c_int(), C.c_double()
    _check(lib().blb_server_poll(server, req_id, C.byref(st), C.byref(lat)), "blb_server_poll")
    return st.value, lat.value


def blb_server_drain(server, timeout_s=600.0):
    _check(lib().blb_server_drain(server, timeout_s), "blb_server_drain")


def blb_server_stats(server):
    out = np.zeros(16, np.float64)
    _check(lib().blb_server_stats(server, _host_ptr(out), 16), "blb_server_stats")
    keys = ["completed", "rejected", "p50_ms", "p99_ms", "mean_ms", "plan_hits", "plan_misses", "batches", "plan_gen_s",
            "plan_bytes", "failed", "gen_deferred_room", "gen_deferred_mem", "plan_bytes_generated", "launch_retries",
            "stall_s"]
    return dict(zip(keys, [float(x) for x in out]))


def blb_server_destroy(server):
    lib().blb_server_destroy(server)
    _SRV_CTX.pop(server, None)


# ---------------------------------------------------------------------------------------
# small conveniences over the ABI (buffer allocation with torch)
# ---------------------------------------------------------------------------------------
def new_ct(n, level, degree=1, device="cuda"):
    """(blb_ct, backing tensor) for a ciphertext at `level`"""
    import torch
    t = torch.empty((degree + 1) * (level + 1) * n, dtype=torch.int64, device=device)
    return blb_ct(t.data_ptr(), level, degree, 0.0), t
