"""The C ABI without a GPU: the library loads, exports every function the
header declares, its struct layouts match the ctypes mirror, and parameter
validation answers with the documented status codes before touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sft.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1407_8315_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_1407_8315_amd import build

        build.build(verbose=False)
    return _lib.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sft_\w+)\s*\(", text)))


def test_every_declared_function_is_exported(lib):
    from paper_1407_8315_amd import _lib

    declared = header_functions()
    assert sorted(_lib.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name), name


def test_version_and_status_strings(lib):
    from paper_1407_8315_amd import _lib

    assert lib.sft_abi_version() == 3
    assert lib.sft_status_str(_lib.SFT_E_CAPACITY) == b"SFT_E_CAPACITY"
    assert lib.sft_status_str(99) == b"unknown status"


def test_struct_layouts_match_c(tmp_path):
    from paper_1407_8315_amd import _lib

    prog = tmp_path / "layout.c"
    prog.write_text("""
#include <stddef.h>
#include <stdio.h>
#include "sft.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(sft_params), sizeof(sft_sparse_out), sizeof(sft_stats), sizeof(sft_plan_info));
  printf("%zu %zu %zu\\n", offsetof(sft_params, seed), offsetof(sft_params, delta_mag), offsetof(sft_plan_info, rshifts));
  printf("%zu %zu %zu\\n", offsetof(sft_plan_info, tau_zero), offsetof(sft_stats, stage_ms), offsetof(sft_stats, gather_ms));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = list(map(int, out))
    want = [ctypes.sizeof(_lib.Params), ctypes.sizeof(_lib.SparseOut), ctypes.sizeof(_lib.Stats),
            ctypes.sizeof(_lib.PlanInfo), _lib.Params.seed.offset, _lib.Params.delta_mag.offset,
            _lib.PlanInfo.rshifts.offset, _lib.PlanInfo.tau_zero.offset, _lib.Stats.stage_ms.offset,
            _lib.Stats.gather_ms.offset]
    assert got == want


def _plan_status(lib, **kw):
    from paper_1407_8315_amd import _lib, make_params

    p = make_params(**kw)
    h = ctypes.c_void_p()
    st = lib.sft_plan(ctypes.byref(h), ctypes.byref(p), 1, None)
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(n=1000, k=10), "SFT_E_UNSUPPORTED"),                 # N not a power of two
    (dict(n=1 << 14, k=0), "SFT_E_INVALID"),                   # K <= 0
    (dict(n=1 << 14, k=(1 << 14) + 1), "SFT_E_INVALID"),       # K > N
    (dict(n=1 << 14, k=50, m=100), "SFT_E_UNSUPPORTED"),       # M not a power of two
    (dict(n=1 << 14, k=50, m=1 << 15), "SFT_E_UNSUPPORTED"),   # M does not divide N
    (dict(n=1 << 14, k=50, l=5), "SFT_E_UNSUPPORTED"),         # L outside 1..4
    (dict(n=1 << 24, k=50, m=1 << 23), "SFT_E_UNSUPPORTED"),   # M above 2^22
    (dict(n=1 << 14, k=50, r=3), "SFT_E_INVALID"),             # R in exact mode
    (dict(n=1 << 14, k=50, mode="general", r=40), "SFT_E_UNSUPPORTED"),
    (dict(n=1 << 14, k=50, flags=1 << 10), "SFT_E_INVALID"),   # unknown flag
    (dict(n=1 << 14, k=50, tau_res=-1.0), "SFT_E_INVALID"),
    (dict(n=1 << 14, k=50, m=128, flags=8), "SFT_E_INVALID"),                 # autotune with a fixed M
    (dict(n=1 << 14, k=50, mode="general", flags=8), "SFT_E_INVALID"),        # autotune in general mode
    (dict(n=1 << 14, k=50, target_recovery=0.99), "SFT_E_INVALID"),           # target without autotune
    (dict(n=1 << 14, k=50, flags=8, target_recovery=1.5), "SFT_E_INVALID"),   # target outside [0, 1)
    (dict(n=1 << 14, k=50, m=4, l=4, mode="iterative"), "SFT_E_UNSUPPORTED"),   # M_0 < 2^(L-1)
    (dict(n=1 << 24, k=50, m=2, l=4, mode="iterative"), "SFT_E_UNSUPPORTED"),   # d_0 2^(L-1) above 2^22
    (dict(n=1 << 14, k=50, mode="iterative", flags=1), "SFT_E_UNSUPPORTED"),    # learned order: exact mode only
    (dict(n=1 << 14, k=50, mode="iterative", flags=8), "SFT_E_INVALID"),        # autotune: exact mode only
    (dict(n=1 << 14, k=50, mode="iterative", r=2), "SFT_E_INVALID"),            # R: general mode only
    (dict(n=1 << 14, k=50, flags=32), "SFT_E_INVALID"),                          # SP on every bin: general mode only
    (dict(n=1 << 14, k=1, mode="general", flags=64), "SFT_E_INVALID"),           # unknown K: exact mode only
    (dict(n=1 << 14, k=1, flags=64 | 8), "SFT_E_INVALID"),                       # unknown K and autotune
])
def test_parameter_validation(lib, kw, status):
    st, h = _plan_status(lib, **kw)
    assert lib.sft_status_str(st).decode() == status
    assert h.value is None
    assert lib.sft_last_error()


def test_mixed_iterative_plan_is_rejected(lib):
    """A plan's signals are all iterative or none is (checked before any device call)."""
    from paper_1407_8315_amd import make_params

    arr = (type(make_params(n=64, k=1)) * 2)(make_params(n=1 << 12, k=8, mode="iterative"),
                                             make_params(n=1 << 12, k=8, mode="exact"))
    h = ctypes.c_void_p()
    st = lib.sft_plan(ctypes.byref(h), arr, 2, None)
    assert lib.sft_status_str(st).decode() == "SFT_E_UNSUPPORTED"
    assert h.value is None
    assert b"ITERATIVE" in lib.sft_last_error()


def test_mixed_fft64_plan_is_rejected(lib):
    from paper_1407_8315_amd import make_params

    arr = (type(make_params(n=64, k=1)) * 2)(make_params(n=1 << 12, k=8, flags=16), make_params(n=1 << 12, k=8))
    h = ctypes.c_void_p()
    st = lib.sft_plan(ctypes.byref(h), arr, 2, None)
    assert lib.sft_status_str(st).decode() == "SFT_E_UNSUPPORTED"
    assert b"FFT64" in lib.sft_last_error()


def test_null_arguments(lib):
    from paper_1407_8315_amd import _lib

    assert lib.sft_plan(None, None, 1, None) == _lib.SFT_E_INVALID
    h = ctypes.c_void_p()
    assert lib.sft_plan(ctypes.byref(h), None, 1, None) == _lib.SFT_E_INVALID
    assert lib.sft_exact(None, None, None, None) == _lib.SFT_E_INVALID
    assert lib.sft_iterative(None, None, None, None) == _lib.SFT_E_INVALID
    assert lib.sft_unknown_k(None, None, None, None, None) == _lib.SFT_E_INVALID
    assert lib.sft_batch(None, None, None, None) == _lib.SFT_E_INVALID
    assert lib.sft_plan_get(None, 0, None) == _lib.SFT_E_INVALID
    lib.sft_destroy(None)


@pytest.mark.parametrize("kw,flags,status,text", [
    (dict(n=1 << 20, k=1000, m=16384, l=4), 0, 2, "limit 8192"),
    (dict(n=1 << 20, k=1000, m=8192, l=4, dtype="c128"), 0, 2, "limit 4096"),
    (dict(n=1 << 30, k=1000, m=8192, l=4), 0, 2, "limit 65536"),
    (dict(n=1 << 20, k=1000, m=4096, l=4), 1, 2, "not available"),     # SFT_FLAG_LEARNED
    (dict(n=1 << 20, k=1000, m=4096, l=4), 2, 2, "not available"),     # SFT_FLAG_SYNC
    (dict(n=1 << 20, k=1000, m=4096, l=4, mode="general"), 0, 1, "SFT_MODE_EXACT"),
    (dict(n=1000, k=10, m=8, l=4), 0, 2, "power of two"),
])
def test_noalloc_rejects_before_any_device_call(lib, kw, flags, status, text):
    """sft_exact_noalloc validates on the host and refuses sizes beyond its
    static workspace with the limit in the error text (no GPU is touched)."""
    from paper_1407_8315_amd import _lib, make_params

    p = make_params(flags=flags, **kw)
    o = _lib.SparseOut()
    o.loc_dev, o.val_dev, o.capacity, o.count_dev = 8, 8, 1, 8   # never dereferenced
    st = lib.sft_exact_noalloc(ctypes.byref(p), ctypes.c_void_p(8), ctypes.byref(o), None)
    assert st == status
    assert text in lib.sft_last_error().decode()
