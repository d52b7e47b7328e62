"""The autotuner's JSON cache format (host-only): what the library writes it
reads back to the same table; malformed files, unknown kernels, values out
of range and caches of another GPU architecture are rejected."""
import ctypes

import pytest


def check(text, arch="gfx950"):
    from paper_2603_13532_amd import _lib
    fn = _lib.load().tsk_tune_json_check
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_size_t]
    out = ctypes.create_string_buffer(1 << 16)
    rc = fn(text.encode(), arch.encode(), out, 1 << 16)
    return rc, out.value.decode()


GOOD = """{"arch": "gfx950", "entries": [
  {"kernel": "proj_final", "param": "split_target", "prec": "fp64", "tiles_log2": 9,
   "ktiles_log2": 4, "value": 1024, "us": 101.5},
  {"us": 7, "value": 2, "kernel": "krp_core_sketch", "param": "waves_per_quadrant",
   "prec": "fp32", "tiles_log2": 12, "ktiles_log2": 6},
  {"kernel": "krp_core_sketch", "param": "split_target", "prec": "bf16x6", "tiles_log2": 0,
   "ktiles_log2": 0, "value": 128, "us": 0.5}
]}"""


def test_round_trip():
    rc, text = check(GOOD)
    assert rc == 0, text
    rc2, text2 = check(text)
    assert rc2 == 0 and text2 == text
    assert text.count('"kernel"') == 3 and '"value": 1024' in text
    assert '"waves_per_quadrant"' in text and '"bf16x6"' in text


def test_empty_table():
    rc, text = check('{"arch": "gfx950", "entries": []}')
    assert rc == 0 and '"entries": [' in text


@pytest.mark.parametrize("bad", [
    GOOD.replace('"gfx950"', '"gfx942"'),                      # another architecture
    GOOD.replace('"proj_final"', '"warp_gemm"'),                # unknown kernel
    GOOD.replace('"value": 2', '"value": 3'),                   # waves per quadrant not 1/2/4
    GOOD.replace('"value": 1024', '"value": 0'),                # split target out of range
    GOOD.replace('"prec": "fp64"', '"prec": "fp16"'),           # unknown precision
    GOOD.replace('"tiles_log2": 9', '"tiles_log2": 9.5'),       # non-integer bucket
    GOOD[:-3],                                                  # truncated
    '{"arch": "gfx950"}',                                       # no entries
    GOOD.replace('"us": 101.5', '"speed": 101.5'),              # unknown field
])
def test_rejects(bad):
    rc, msg = check(bad)
    assert rc != 0 and msg
