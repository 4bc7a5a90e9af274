"""CPU-side checks of the C ABI library: it loads and exports every symbol include/blb.h declares
(no compute calls: those need a GPU)."""
import os
import re

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
