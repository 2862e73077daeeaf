"""The C-ABI library loads on a machine without a GPU, exports every function that
include/rlwe.h declares, and rejects invalid parameters before touching a device."""

import ctypes
import os
import re

import pytest

from paper_2505_07329_amd import rlwe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlwe.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rlwe_params_init", "ct_matmul_clear", "ct_modswitch"):
        assert must in names
    assert set(names) == set(rlwe.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = rlwe.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_binding_declares_every_signature():
    """Every exported function has its argument types declared in the binding (an
    undeclared pointer argument would be passed as a 32-bit int)."""
    L = rlwe.lib()
    for name in rlwe.EXPORTS:
        assert getattr(L, name).argtypes is not None, name


P4096 = (18014398509309953, 18014398509293569)


@pytest.mark.parametrize("N,primes,log2_t,q_out,code", [
    (1000, P4096, 26, 32, -2),                      # N not a power of two
    (32, P4096, 26, 32, -2),                        # N too small
    (65536, P4096, 26, 32, -2),                     # N too large
    (4096, (18014398509309953, 18014398509309953), 26, 32, -2),  # repeated prime
    (4096, (18014398509309951,), 26, 32, -2),       # not prime / not 1 mod 2N
    (4096, ((1 << 54) + 1,), 26, 32, -2),           # >= 2^54
    (4096, (40961,), 26, 32, -2),                   # 40961 = 1 mod 8192 is prime but t > q
    (4096, (12289,), 8, 32, -2),                    # 12289 is prime but not 1 mod 8192
    (4096, P4096, 26, 0, -2),                       # q_out = 2^0
    (4096, P4096, 26, 33, -2),                      # q_out above 2^32
    (4096, P4096, 0, 32, -2),                       # log2_t out of range
    (4096, P4096 + (12289,), 26, 32, -2),           # three primes
])
def test_params_validation(N, primes, log2_t, q_out, code):
    with pytest.raises(rlwe.RlweError) as ei:
        rlwe.rlwe_params_init(N, primes, log2_t, log2_q_out=q_out)
    assert ei.value.code == code


def test_null_arguments_rejected():
    L = rlwe.lib()
    assert L.rlwe_params_init(None, 0, None) == -1
    assert L.ct_matmul_clear(None, None, 0, None, 0, None, 0, None) == -1
    assert L.ct_modswitch(None, None, 0, None, None) == -1
    assert L.rlwe_weights_load(None, None, 1, 1, 1, None, None) == -1
    assert L.rlwe_params_destroy(None) == 0
    assert L.rlwe_weights_free(None) == 0
    assert b"null" in L.rlwe_last_error() or L.rlwe_last_error() == b""


def test_keyswitch_entry_points_reject_null_arguments():
    L = rlwe.lib()
    assert L.rlwe_ksk_load(None, None, 54, 1, None, None) == -1
    assert L.ct_keyswitch_pack(None, None, None, 0, 1, None, 0, None) == -1
    assert L.rlwe_ksk_free(None) == 0
    assert L.rlwe_keyswitch_workspace_bytes(None, None, 1, 1) == 0
    assert L.ct_matmul_pack(None, None, 0, None, 0, None, 1, None, 0, None) == -1
    assert L.rlwe_matmul_pack_workspace_bytes(None, None, 0, 1, None, 1) == 0
    assert L.rlwe_packed_count(10, 4) == 3
    assert L.rlwe_packed_count(8192, 4096) == 2
    assert L.rlwe_packed_count(10, 0) == 0
