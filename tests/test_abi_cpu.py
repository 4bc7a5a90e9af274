"""CPU-side checks of the C ABI library: it loads and exports every symbol include/blb.h declares
(no compute calls: those need a GPU)."""
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _declared():
    src = open(os.path.join(ROOT, "include", "blb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(blb_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import ctypes
    import paper_2508_19525_amd as B
    L = B.lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
        assert callable(getattr(L, n))
    # the binding marshals exactly the declared entry points
    assert sorted(B.exported_symbols()) == names


def test_binding_constants_match_header_enums():
    """Every BLB_* enum constant the binding defines has the header's value (knobs, timing kinds,
    variant counts, status codes)."""
    import paper_2508_19525_amd as B
    src = open(os.path.join(ROOT, "include", "blb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    header = {}
    for body in re.findall(r"enum\s*\{(.*?)\}", src, flags=re.S):
        for name, val in re.findall(r"\b(BLB_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            header[name] = int(val)
    assert {"BLB_KNOB_PLAN_FORMAT", "BLB_MAC_VARIANTS", "BLB_BATCH_VARIANTS", "BLB_T_CP_MAC"} <= set(header)
    shared = [n for n in header if hasattr(B, n)]
    assert len(shared) >= 20
    for n in shared:
        assert getattr(B, n) == header[n], n


def test_status_strings():
    import paper_2508_19525_amd as B
    assert B.status_str(0) == "ok"
    assert "key" in B.status_str(B.BLB_ENOKEY)
    assert B.status_str(-99) == "unknown status"


def test_package_has_no_cpu_fallback():
    """The product path never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2508_19525_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert not re.search(r"^\s*(import|from)\s+oracle", src, flags=re.M), fn


def test_binding_refuses_undersized_device_buffers():
    """The binding checks torch buffers against the words a call reads or writes ((level + 1) N
    for a decryption, n_ct (target + 1) N for shares, ...) before calling into the library."""
    import torch
    import paper_2508_19525_amd as B
    fake_ctx = 0x1234
    B._CTX_N[fake_ctx] = 4096
    try:
        ct = B.blb_ct()
        ct.level, ct.degree = 1, 1
        small = torch.empty(4096, dtype=torch.int64)
        for fn, args in [(B.blb_decrypt, (fake_ctx, None, ct, small)),
                         (B.blb_decode, (fake_ctx, small, 1, 1.0, 8)),
                         (B.blb_encode, (fake_ctx, np.zeros(4), 1.0, 1, small)),
                         (B.blb_mask_to_share, (fake_ctx, [ct], 1, 1, small)),
                         (B.blb_add_share, (fake_ctx, [ct], small)),
                         (B.blb_ntt, (fake_ctx, small, 2, 1))]:
            try:
                fn(*args)
            except B.BlbError as e:
                assert e.code == B.BLB_EINVAL
            else:
                raise AssertionError(f"{fn.__name__} accepted an undersized buffer")
    finally:
        B._CTX_N.pop(fake_ctx, None)
