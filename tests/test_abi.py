"""Host-side checks of the C ABI: the library loads, exports every function
include/tsk.h declares, and its host-only size and validation logic agrees
with the paper's rules.  No GPU is touched."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import ROOT, read_golden

HEADER = os.path.join(ROOT, "include", "tsk.h")
TEST_HEADER = os.path.join(ROOT, "include", "tsk_test.h")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:tsk|tucker)_\w+)\s*\(", text)))


def exported_functions():
    """Dynamic symbols the built library defines with the ABI's prefixes."""
    import subprocess
    from paper_2603_13532_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    names = set()
    for line in out.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[1] in ("T", "t") and re.match(r"(tsk|tucker)_", parts[2]):
            names.add(parts[2])
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2603_13532_amd import _lib
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "tucker_sum_sketch" in names and "tucker_sum_recompress" in names
    for name in names:
        assert hasattr(lib, name), name


def test_every_export_is_declared(lib):
    """No undeclared entry points: every exported tsk_* / tucker_sum_*
    symbol is declared in the public header or in the test header, and every
    test-header function is exported."""
    public, testing = set(declared_functions()), set(declared_functions(TEST_HEADER))
    assert not public & testing
    exported = exported_functions()
    assert exported - public - testing == set()
    assert testing <= exported


def test_binding_prototypes_cover_header():
    from paper_2603_13532_amd import _lib
    assert set(_lib.PROTOTYPES) == set(declared_functions())


def test_status_strings(lib):
    for code, name in {0: b"TSK_OK", 1: b"TSK_ERR_INVALID_ARG", 4: b"TSK_ERR_WORKSPACE_TOO_SMALL",
                       6: b"TSK_ERR_RANK_DEFICIENT"}.items():
        assert lib.tsk_status_string(code) == name


def test_kron_sizes_match_golden_and_oracle():
    import paper_2603_13532_amd as tsk
    from oracle.recompress import kron_sizes
    for row in read_golden("kron_sketch_sizes.txt"):
        d = int(row[0])
        ell = [int(x) for x in row[1:1 + d]]
        want = [int(x) for x in row[1 + d:1 + 2 * d]]
        assert tsk.kron_sizes(ell) == want
    rng = np.random.default_rng(0)
    for _ in range(200):
        d = int(rng.integers(2, 7))
        ell = [int(x) for x in rng.integers(1, 200, size=d)]
        assert tsk.kron_sizes(ell) == kron_sizes(ell), ell


def test_krp_width():
    import paper_2603_13532_amd as tsk
    assert tsk.krp_width([3, 74, 12]) == 74


def _fake_sum(lib, d=3, s=2, dims=(10, 11, 12), rank=3, kind=0, sizes=(5,), dtype=0):
    from paper_2603_13532_amd import _lib
    keep = {}
    keep["dims"] = (ctypes.c_int64 * d)(*dims)
    keep["ranks"] = (ctypes.c_int32 * (s * d))(*([rank] * (s * d)))
    keep["cores"] = (ctypes.c_void_p * s)(*([0x1000] * s))
    keep["factors"] = (ctypes.c_void_p * (s * d))(*([0x2000] * (s * d)))
    keep["sizes"] = (ctypes.c_int32 * len(sizes))(*sizes)
    tsum = _lib.TuckerSum(d, s, keep["dims"], keep["ranks"], keep["cores"], keep["factors"], None,
                          dtype)
    spec = _lib.SketchSpec(kind, keep["sizes"], 7, None, 0, 0, 0)
    return tsum, spec, keep


def test_sketch_widths_krp_and_kron(lib):
    sw = (ctypes.c_int64 * 3)()
    bw = (ctypes.c_int64 * 3)()
    tsum, spec, keep = _fake_sum(lib, dims=(10, 40, 40), sizes=(12,))
    assert lib.tsk_sketch_widths(ctypes.byref(tsum), ctypes.byref(spec), sw, bw) == 0
    assert list(sw) == [12, 12, 12] and list(bw) == [10, 12, 12]   # economy width min(n, m)
    tsum, spec, keep = _fake_sum(lib, dims=(10, 40, 40), kind=1, sizes=(2, 3, 4))
    assert lib.tsk_sketch_widths(ctypes.byref(tsum), ctypes.byref(spec), sw, bw) == 0
    assert list(sw) == [12, 8, 6] and list(bw) == [10, 8, 6]


@pytest.mark.parametrize("field,value", [("order", 1), ("order", 99), ("num_terms", 0),
                                         ("dtype", 7)])
def test_validation_rejects_bad_sums(lib, field, value):
    tsum, spec, keep = _fake_sum(lib)
    setattr(tsum, field, value)
    sw = (ctypes.c_int64 * 3)()
    assert lib.tsk_sketch_widths(ctypes.byref(tsum), ctypes.byref(spec), sw, None) == 1


def test_validation_rejects_bad_ranks_sizes_and_pointers(lib):
    sw = (ctypes.c_int64 * 3)()
    tsum, spec, keep = _fake_sum(lib)
    keep["ranks"][4] = 0
    assert lib.tsk_sketch_widths(ctypes.byref(tsum), ctypes.byref(spec), sw, None) == 1
    tsum, spec, keep = _fake_sum(lib, sizes=(0,))
    assert lib.tsk_sketch_widths(ctypes.byref(tsum), ctypes.byref(spec), sw, None) == 1
    tsum, spec, keep = _fake_sum(lib)
    keep["factors"][3] = None
    assert lib.tsk_sketch_widths(ctypes.byref(tsum), ctypes.byref(spec), sw, None) == 1
    tsum, spec, keep = _fake_sum(lib)
    spec.kind = 5
    assert lib.tsk_sketch_widths(ctypes.byref(tsum), ctypes.byref(spec), sw, None) == 1
    tsum, spec, keep = _fake_sum(lib)
    spec.sketch_prec = 9
    assert lib.tsk_sketch_widths(ctypes.byref(tsum), ctypes.byref(spec), sw, None) == 1
    tsum, spec, keep = _fake_sum(lib)
    spec.qr_policy = 3
    assert lib.tsk_sketch_widths(ctypes.byref(tsum), ctypes.byref(spec), sw, None) == 1
    assert lib.tsk_sketch_widths(None, ctypes.byref(spec), sw, None) == 1


def test_null_handle_calls_fail_cleanly(lib):
    tsum, spec, keep = _fake_sum(lib)
    nbytes = ctypes.c_size_t()
    assert lib.tucker_sum_workspace_size(None, ctypes.byref(tsum), ctypes.byref(spec),
                                         ctypes.byref(nbytes)) == 1
    assert lib.tsk_destroy(None) == 1
    assert lib.tsk_last_error_detail(None) == b""


def test_product_has_no_oracle_dependency():
    """The package never imports the oracle (no CPU fallback path)."""
    pkg = os.path.join(ROOT, "paper_2603_13532_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
