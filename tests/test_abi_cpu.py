"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/at.h declares, the binding covers them, and parameter
validation rejects what the reversible hash cannot support."""
import ctypes as C
import os
import re

import pytest

from paper_1807_01527_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    hdr = open(os.path.join(ROOT, "include", "at.h")).read()
    return re.findall(r"^\s*(?:int|const char \*)\s*(at_\w+)\s*\(", hdr, re.M)


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = _header_symbols()
    assert {"at_create", "at_ingest_slice", "at_close_slice", "at_estimate", "at_restore",
            "at_destroy"} <= set(names)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.SIGNATURES)


def test_strerror_and_null_handles():
    lib = binding.load()
    assert lib.at_strerror(binding.AT_E_BUDGET).decode() == "restore tuple budget exceeded"
    assert lib.at_destroy(None) == binding.AT_OK
    assert lib.at_close_slice(None, 1) == binding.AT_E_INVAL
    assert lib.at_ingest_slice(None, None, None, 0) == binding.AT_E_INVAL


@pytest.mark.parametrize("bad", [
    dict(k=4, r=4, c=9, s=7, u=0, log2g=9),      # c + s(r-1) < W: incomplete
    dict(k=4, r=4, c=7, s=7, u=4, log2g=9),      # c*r <= W: no redundancy
    dict(k=0, r=4, c=9, s=8, u=0, log2g=9),
    dict(k=32768, r=4, c=9, s=8, u=0, log2g=9),  # 2k no longer fits a 16-bit AT
    dict(k=4, r=9, c=9, s=4, u=0, log2g=9),      # more rows than supported
    dict(k=4, r=4, c=9, s=10, u=0, log2g=9),     # s > c
    dict(k=4, r=4, c=9, s=8, u=0, log2g=3),      # g below 16
    dict(k=4, r=4, c=9, s=8, u=0, log2g=9, theta=-1.0),
])
def test_create_rejects_invalid_geometry(bad):
    lib = binding.load()
    p = binding.Params(bad["k"], bad["r"], bad["c"], bad["s"], bad["u"], bad["log2g"], bad.get("theta", 1024.0),
                       0, 0)
    h = C.c_void_p()
    assert lib.at_create(C.byref(p), None, C.byref(h)) == binding.AT_E_INVAL
    assert not h.value


def test_binding_constants_match_header():
    """Limits the binding checks against are the header's own #defines."""
    import re
    with open(os.path.join(ROOT, "include", "at.h")) as f:
        text = f.read()
    defs = dict(re.findall(r"#define\s+(AT_[A-Z_]+)\s+\(?([0-9a-z<>ul ]+?)\)?\s*$", text, re.M))
    assert eval(defs["AT_HIST_MAX_K"]) == binding.AT_HIST_MAX_K
    assert eval(defs["AT_NOALLOC_MAX_PAIRS"].replace("ull", "")) == binding.NOALLOC_MAX_PAIRS
    assert eval(defs["AT_MAX_WINDOWS"]) == 8
