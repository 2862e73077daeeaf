"""Thin Python binding of the C ABI in include/rlwe.h (argument marshalling only).

Every computation runs in the HIP library ``librlwe.so`` next to this file;
PyTorch provides device memory and streams. If the library is missing the
binding raises instead of computing anything on the CPU.

Tensor conventions (torch has no unsigned 64/32-bit arithmetic, only storage):
uint64 buffers are passed as torch.int64 tensors holding the same bits, uint32
buffers as torch.int32 tensors.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlwe.so")

RLWE_OK = 0
RLWE_EINVAL, RLWE_EPARAM, RLWE_ESHAPE, RLWE_EOVERFLOW, RLWE_ENOMEM, RLWE_EHIP = -1, -2, -3, -4, -5, -6
ERRORS = {-1: "RLWE_EINVAL", -2: "RLWE_EPARAM", -3: "RLWE_ESHAPE", -4: "RLWE_EOVERFLOW",
          -5: "RLWE_ENOMEM", -6: "RLWE_EHIP"}
RLWE_W_FWD = 1
RLWE_W_TRANSPOSE = 2
RLWE_W_NTT = 4
RLWE_W_TOEPLITZ = 8
RLWE_W_ROWPACK = 16
RLWE_METHOD_TOEPLITZ = 0
RLWE_METHOD_NTT = 1
RLWE_OUT_SWITCHED = 0
RLWE_OUT_RAW_Q = 1
RLWE_OUT_FORCE_EXACT = 2
RLWE_IN_SEEDED = 4
RLWE_LAUNCH_PERSISTENT = 8
RLWE_LAUNCH_GROUPED = 16

EXPORTS = ("rlwe_params_init", "rlwe_params_destroy", "rlwe_weights_load", "rlwe_weights_free",
           "ct_matmul_clear", "ct_modswitch", "rlwe_workspace_bytes", "rlwe_workspace_reserve",
           "rlwe_profile_begin", "rlwe_profile_end", "rlwe_weights_digits", "ct_matmul_batch",
           "rlwe_batch_workspace_bytes", "rlwe_graph_capture_batch", "rlwe_graph_launch",
           "rlwe_graph_destroy", "rlwe_weights_method", "ct_pack_bits", "rlwe_packed_words",
           "rlwe_weights_rows_per_product", "rlwe_ksk_load", "rlwe_ksk_free",
           "rlwe_packed_count", "rlwe_keyswitch_workspace_bytes", "ct_keyswitch_pack",
           "rlwe_matmul_pack_workspace_bytes", "ct_matmul_pack", "ct_matmul_clear_noalloc",
           "rlwe_tuner_create", "rlwe_tuner_destroy", "rlwe_tuner_size", "rlwe_tune_key",
           "rlwe_tuner_put", "rlwe_tuner_get", "rlwe_tuner_lookup", "rlwe_tuner_save",
           "rlwe_tuner_load", "rlwe_device_key", "rlwe_ctx_set_tuner", "rlwe_autotune_product",
           "rlwe_autotune_batch", "rlwe_measure_peaks", "rlwe_last_error")
RLWE_NOALLOC_SCRATCH_BYTES = 64 << 20


class RlweError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class KernelTimes(ctypes.Structure):
    _fields_ = [("prep_ms", ctypes.c_double), ("mask_ms", ctypes.c_double),
                ("body_ms", ctypes.c_double), ("modswitch_ms", ctypes.c_double),
                ("ntt_ms", ctypes.c_double), ("pack_ms", ctypes.c_double),
                ("prep_n", ctypes.c_uint32), ("mask_n", ctypes.c_uint32),
                ("body_n", ctypes.c_uint32), ("modswitch_n", ctypes.c_uint32),
                ("ntt_n", ctypes.c_uint32), ("pack_n", ctypes.c_uint32),
                ("dropped", ctypes.c_uint32),
                ("ksdig_ms", ctypes.c_double), ("ksacc_ms", ctypes.c_double),
                ("ksfin_ms", ctypes.c_double), ("ksdig_n", ctypes.c_uint32),
                ("ksacc_n", ctypes.c_uint32), ("ksfin_n", ctypes.c_uint32),
                ("persist_ms", ctypes.c_double), ("persist_n", ctypes.c_uint32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class CtMatmulDesc(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("transpose", ctypes.c_uint32),
                ("ct_in", ctypes.c_void_p), ("tokens", ctypes.c_uint32), ("out", ctypes.c_void_p)]


class Schedule(ctypes.Structure):
    _fields_ = [("method", ctypes.c_uint32), ("tt_log2", ctypes.c_uint32),
                ("order", ctypes.c_uint32), ("launch", ctypes.c_uint32), ("ms", ctypes.c_float)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class Peaks(ctypes.Structure):
    _fields_ = [("mul32_lane_ops", ctypes.c_double), ("modmul", ctypes.c_double),
                ("butterfly", ctypes.c_double), ("mfma_int8_ops", ctypes.c_double),
                ("clock_mhz", ctypes.c_double), ("compute_units", ctypes.c_uint32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class _Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("num_primes", ctypes.c_uint32),
                ("primes", ctypes.POINTER(ctypes.c_uint64)), ("log2_t", ctypes.c_uint32),
                ("log2_q_out", ctypes.c_uint32)]


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """Load librlwe.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_07329_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.rlwe_params_init.argtypes = [ctypes.POINTER(_Params), ctypes.c_int, ctypes.POINTER(vp)]
    L.rlwe_params_destroy.argtypes = [vp]
    L.rlwe_weights_load.argtypes = [vp, vp, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, vp,
                                    ctypes.POINTER(vp)]
    L.rlwe_weights_free.argtypes = [vp]
    L.ct_matmul_clear.argtypes = [vp, vp, ctypes.c_uint32, vp, ctypes.c_uint32, vp,
                                  ctypes.c_uint32, vp]
    L.ct_matmul_clear_noalloc.argtypes = [vp, vp, ctypes.c_uint32, vp, ctypes.c_uint32, vp,
                                          ctypes.c_uint32, vp]
    L.ct_modswitch.argtypes = [vp, vp, ctypes.c_size_t, vp, vp]
    L.ct_pack_bits.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_uint32, vp, vp]
    L.rlwe_packed_words.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    L.rlwe_packed_words.restype = ctypes.c_size_t
    L.rlwe_workspace_bytes.argtypes = [vp, vp, ctypes.c_uint32, ctypes.c_uint32]
    L.rlwe_workspace_bytes.restype = ctypes.c_size_t
    L.rlwe_workspace_reserve.argtypes = [vp, ctypes.c_size_t]
    L.rlwe_profile_begin.argtypes = [vp]
    L.rlwe_profile_end.argtypes = [vp, ctypes.POINTER(KernelTimes)]
    L.rlwe_weights_digits.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                      ctypes.POINTER(ctypes.c_uint32)]
    L.rlwe_weights_method.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
    L.rlwe_weights_rows_per_product.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
    L.ct_matmul_batch.argtypes = [vp, ctypes.POINTER(CtMatmulDesc), ctypes.c_uint32,
                                  ctypes.c_uint32, vp]
    L.rlwe_batch_workspace_bytes.argtypes = [vp, ctypes.POINTER(CtMatmulDesc), ctypes.c_uint32]
    L.rlwe_batch_workspace_bytes.restype = ctypes.c_size_t
    L.rlwe_graph_capture_batch.argtypes = [vp, ctypes.POINTER(CtMatmulDesc), ctypes.c_uint32,
                                           ctypes.c_uint32, ctypes.POINTER(vp)]
    L.rlwe_graph_launch.argtypes = [vp, vp]
    L.rlwe_graph_destroy.argtypes = [vp]
    L.rlwe_ksk_load.argtypes = [vp, vp, ctypes.c_uint32, ctypes.c_uint32, vp, ctypes.POINTER(vp)]
    L.rlwe_ksk_free.argtypes = [vp]
    L.rlwe_packed_count.argtypes = [ctypes.c_size_t, ctypes.c_uint32]
    L.rlwe_packed_count.restype = ctypes.c_size_t
    L.rlwe_keyswitch_workspace_bytes.argtypes = [vp, vp, ctypes.c_size_t, ctypes.c_uint32]
    L.rlwe_keyswitch_workspace_bytes.restype = ctypes.c_size_t
    L.ct_keyswitch_pack.argtypes = [vp, vp, vp, ctypes.c_size_t, ctypes.c_uint32, vp,
                                    ctypes.c_uint32, vp]
    L.rlwe_matmul_pack_workspace_bytes.argtypes = [vp, vp, ctypes.c_uint32, ctypes.c_uint32, vp,
                                                   ctypes.c_uint32]
    L.rlwe_matmul_pack_workspace_bytes.restype = ctypes.c_size_t
    L.ct_matmul_pack.argtypes = [vp, vp, ctypes.c_uint32, vp, ctypes.c_uint32, vp,
                                 ctypes.c_uint32, vp, ctypes.c_uint32, vp]
    u32, sz = ctypes.c_uint32, ctypes.c_size_t
    L.rlwe_tuner_create.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
    L.rlwe_tuner_destroy.argtypes = [vp]
    L.rlwe_tuner_size.argtypes = [vp]
    L.rlwe_tuner_size.restype = sz
    L.rlwe_tune_key.argtypes = [u32, u32, u32, u32, u32, u32, u32, ctypes.c_char_p, sz]
    L.rlwe_tuner_put.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(Schedule)]
    L.rlwe_tuner_get.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(Schedule)]
    L.rlwe_tuner_lookup.argtypes = [vp, u32, u32, u32, u32, u32, u32, u32, ctypes.POINTER(Schedule)]
    L.rlwe_tuner_save.argtypes = [vp, ctypes.c_char_p]
    L.rlwe_tuner_load.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(sz)]
    L.rlwe_device_key.argtypes = [ctypes.c_int, ctypes.c_char_p, sz]
    L.rlwe_ctx_set_tuner.argtypes = [vp, vp]
    L.rlwe_autotune_product.argtypes = [vp, vp, u32, u32, u32, u32, u32, vp, ctypes.POINTER(Schedule)]
    L.rlwe_autotune_batch.argtypes = [vp, vp, ctypes.POINTER(CtMatmulDesc), u32, u32, vp,
                                      ctypes.POINTER(Schedule)]
    L.rlwe_measure_peaks.argtypes = [ctypes.c_int, ctypes.POINTER(Peaks)]
    L.rlwe_last_error.argtypes = []
    L.rlwe_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("rlwe_last_error", "rlwe_workspace_bytes", "rlwe_batch_workspace_bytes",
                        "rlwe_packed_words", "rlwe_packed_count", "rlwe_tuner_size",
                        "rlwe_keyswitch_workspace_bytes", "rlwe_matmul_pack_workspace_bytes"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int) -> None:
    if rc != RLWE_OK:
        raise RlweError(rc, lib().rlwe_last_error().decode())


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t) -> int:
    if t is None:
        return 0
    assert t.is_contiguous(), "buffers must be contiguous"
    return t.data_ptr()


# ------------------------------------------------------------------ ABI names

def rlwe_params_init(N: int, primes: Sequence[int], log2_t: int, device: int = 0,
                     log2_q_out: int = 32) -> int:
    arr = (ctypes.c_uint64 * len(primes))(*[int(p) for p in primes])
    p = _Params(N, len(primes), ctypes.cast(arr, ctypes.POINTER(ctypes.c_uint64)), log2_t, log2_q_out)
    h = ctypes.c_void_p()
    _check(lib().rlwe_params_init(ctypes.byref(p), device, ctypes.byref(h)))
    return h.value


def rlwe_params_destroy(ctx: int) -> None:
    _check(lib().rlwe_params_destroy(ctx))


def rlwe_weights_load(ctx: int, W, flags: int = RLWE_W_FWD, stream=None) -> int:
    """W: torch.int8 CUDA tensor (d_out, d_in)."""
    d_out, d_in = W.shape
    h = ctypes.c_void_p()
    _check(lib().rlwe_weights_load(ctx, _ptr(W), d_out, d_in, flags, _stream(stream),
                                   ctypes.byref(h)))
    return h.value


def rlwe_weights_free(w: int) -> None:
    _check(lib().rlwe_weights_free(w))


def ct_matmul_clear(ctx: int, w: int, ct, tokens: int, out, transpose: bool = False,
                    flags: int = RLWE_OUT_SWITCHED, stream=None) -> None:
    """ct: int64 tensor [tokens][L][2][P][N]; out: int32 [tokens][M][N+1] (switched) or
    int64 [tokens][M][P][N+1] (RLWE_OUT_RAW_Q)."""
    _check(lib().ct_matmul_clear(ctx, w, int(bool(transpose)), _ptr(ct), tokens, _ptr(out), flags,
                                 _stream(stream)))


def ct_matmul_clear_noalloc(ctx: int, w: int, ct, tokens: int, out, transpose: bool = False,
                            flags: int = RLWE_OUT_SWITCHED, stream=None) -> None:
    """ct_matmul_clear with its workspace in the library's fixed device array (no
    allocation); same buffers and flags."""
    _check(lib().ct_matmul_clear_noalloc(ctx, w, int(bool(transpose)), _ptr(ct), tokens,
                                         _ptr(out), flags, _stream(stream)))


def ct_modswitch(ctx: int, raw, count: int, out, stream=None) -> None:
    """raw: int64 [count][P][N+1]; out: int32 [count][N+1]."""
    _check(lib().ct_modswitch(ctx, _ptr(raw), count, _ptr(out), _stream(stream)))


def ct_pack_bits(ctx: int, inp, count: int, length: int, out, stream=None) -> None:
    """inp: int32 [count][length] switched coefficients; out: int32 [count][rlwe_packed_words]."""
    _check(lib().ct_pack_bits(ctx, _ptr(inp), count, length, _ptr(out), _stream(stream)))


def rlwe_packed_words(length: int, bits: int) -> int:
    return int(lib().rlwe_packed_words(length, bits))


def rlwe_workspace_bytes(ctx: int, w: int, transpose: bool, tokens: int) -> int:
    return int(lib().rlwe_workspace_bytes(ctx, w, int(bool(transpose)), tokens))


def rlwe_workspace_reserve(ctx: int, nbytes: int) -> None:
    _check(lib().rlwe_workspace_reserve(ctx, nbytes))


def rlwe_weights_digits(w: int, transpose: bool = False) -> tuple[int, int]:
    kept, total = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().rlwe_weights_digits(w, int(bool(transpose)), ctypes.byref(kept), ctypes.byref(total)))
    return kept.value, total.value


def rlwe_weights_method(w: int, transpose: bool = False) -> int:
    m = ctypes.c_uint32()
    _check(lib().rlwe_weights_method(w, int(bool(transpose)), ctypes.byref(m)))
    return m.value


def rlwe_weights_rows_per_product(w: int, transpose: bool = False) -> int:
    n = ctypes.c_uint32()
    _check(lib().rlwe_weights_rows_per_product(w, int(bool(transpose)), ctypes.byref(n)))
    return n.value


def _descs(items):
    """items: sequence of (weights_handle, transpose, ct_tensor, tokens, out_tensor)."""
    arr = (CtMatmulDesc * len(items))()
    for i, (w, tr, ct, tokens, out) in enumerate(items):
        arr[i] = CtMatmulDesc(w, int(bool(tr)), _ptr(ct), tokens, _ptr(out))
    return arr


def ct_matmul_batch(ctx: int, items, flags: int = RLWE_OUT_SWITCHED, stream=None) -> None:
    arr = _descs(items)
    _check(lib().ct_matmul_batch(ctx, arr, len(items), flags, _stream(stream)))


def rlwe_batch_workspace_bytes(ctx: int, items) -> int:
    arr = _descs(items)
    return int(lib().rlwe_batch_workspace_bytes(ctx, arr, len(items)))


def rlwe_graph_capture_batch(ctx: int, items, flags: int = RLWE_OUT_SWITCHED) -> int:
    arr = _descs(items)
    h = ctypes.c_void_p()
    _check(lib().rlwe_graph_capture_batch(ctx, arr, len(items), flags, ctypes.byref(h)))
    return h.value


def rlwe_graph_launch(graph: int, stream=None) -> None:
    _check(lib().rlwe_graph_launch(graph, _stream(stream)))


def rlwe_graph_destroy(graph: int) -> None:
    _check(lib().rlwe_graph_destroy(graph))


def rlwe_ksk_load(ctx: int, ksk, log2_base: int, levels: int, stream=None) -> int:
    """ksk: int64 CUDA tensor [N][levels][2][P][N] (uint64 residues of KSK_{i,m})."""
    h = ctypes.c_void_p()
    _check(lib().rlwe_ksk_load(ctx, _ptr(ksk), log2_base, levels, _stream(stream), ctypes.byref(h)))
    return h.value


def rlwe_ksk_free(k: int) -> None:
    _check(lib().rlwe_ksk_free(k))


def rlwe_packed_count(count: int, n_pack: int) -> int:
    return int(lib().rlwe_packed_count(count, n_pack))


def rlwe_keyswitch_workspace_bytes(ctx: int, k: int, count: int, n_pack: int) -> int:
    return int(lib().rlwe_keyswitch_workspace_bytes(ctx, k, count, n_pack))


def ct_keyswitch_pack(ctx: int, k: int, lwe, count: int, n_pack: int, out,
                      flags: int = RLWE_OUT_SWITCHED, stream=None) -> None:
    """lwe: int64 [count][P][N+1] raw LWE ciphertexts; out: int32 [G][2][N] (switched) or
    int64 [G][2][P][N] (RLWE_OUT_RAW_Q), G = rlwe_packed_count(count, n_pack)."""
    _check(lib().ct_keyswitch_pack(ctx, k, _ptr(lwe), count, n_pack, _ptr(out), flags,
                                   _stream(stream)))


def rlwe_matmul_pack_workspace_bytes(ctx: int, w: int, transpose: bool, tokens: int, k: int,
                                     n_pack: int) -> int:
    return int(lib().rlwe_matmul_pack_workspace_bytes(ctx, w, int(bool(transpose)), tokens, k,
                                                      n_pack))


def ct_matmul_pack(ctx: int, w: int, ct, tokens: int, k: int, n_pack: int, out,
                   transpose: bool = False, flags: int = RLWE_OUT_SWITCHED, stream=None) -> None:
    """ct as for ct_matmul_clear; out as for ct_keyswitch_pack with count = tokens * rows."""
    _check(lib().ct_matmul_pack(ctx, w, int(bool(transpose)), _ptr(ct), tokens, k, n_pack,
                                _ptr(out), flags, _stream(stream)))


def rlwe_tuner_create(device_key: str) -> int:
    h = ctypes.c_void_p()
    _check(lib().rlwe_tuner_create(device_key.encode(), ctypes.byref(h)))
    return h.value


def rlwe_tuner_destroy(t: int) -> None:
    _check(lib().rlwe_tuner_destroy(t))


def rlwe_tuner_size(t: int) -> int:
    return int(lib().rlwe_tuner_size(t))


def rlwe_tune_key(N: int, P: int, K: int, M: int, n_o: int = 1, raw: bool = False,
                  tokens: int = 1) -> str:
    buf = ctypes.create_string_buffer(160)
    _check(lib().rlwe_tune_key(N, P, K, M, n_o, int(bool(raw)), tokens, buf, len(buf)))
    return buf.value.decode()


def rlwe_tuner_put(t: int, key: str, sched: dict) -> None:
    s = Schedule(**{k: sched[k] for k in ("method", "tt_log2", "order", "launch", "ms")})
    _check(lib().rlwe_tuner_put(t, key.encode(), ctypes.byref(s)))


def rlwe_tuner_get(t: int, key: str) -> dict:
    s = Schedule()
    _check(lib().rlwe_tuner_get(t, key.encode(), ctypes.byref(s)))
    return s.as_dict()


def rlwe_tuner_lookup(t: int, N: int, P: int, K: int, M: int, n_o: int = 1, raw: bool = False,
                      tokens: int = 1):
    """The entry a product call uses (nearest token bucket of its shape), or None."""
    s = Schedule()
    rc = lib().rlwe_tuner_lookup(t, N, P, K, M, n_o, int(bool(raw)), tokens, ctypes.byref(s))
    if rc < 0:
        _check(rc)
    return s.as_dict() if rc == 1 else None


def rlwe_tuner_save(t: int, path: str) -> None:
    _check(lib().rlwe_tuner_save(t, os.fsencode(path)))


def rlwe_tuner_load(t: int, path: str) -> int:
    n = ctypes.c_size_t()
    _check(lib().rlwe_tuner_load(t, os.fsencode(path), ctypes.byref(n)))
    return n.value


def rlwe_device_key(device: int = 0) -> str:
    buf = ctypes.create_string_buffer(512)
    _check(lib().rlwe_device_key(device, buf, len(buf)))
    return buf.value.decode()


def rlwe_ctx_set_tuner(ctx: int, t) -> None:
    _check(lib().rlwe_ctx_set_tuner(ctx, t or None))


def rlwe_autotune_product(ctx: int, t: int, K: int, M: int, tokens: int, wflags: int = 0,
                          oflags: int = RLWE_OUT_SWITCHED, stream=None) -> dict:
    s = Schedule()
    _check(lib().rlwe_autotune_product(ctx, t, K, M, wflags, tokens, oflags, _stream(stream),
                                       ctypes.byref(s)))
    return s.as_dict()


def rlwe_autotune_batch(ctx: int, t: int, items, flags: int = RLWE_OUT_SWITCHED, stream=None) -> dict:
    arr = _descs(items)
    s = Schedule()
    _check(lib().rlwe_autotune_batch(ctx, t, arr, len(items), flags, _stream(stream), ctypes.byref(s)))
    return s.as_dict()


def rlwe_measure_peaks(device: int = 0) -> dict:
    """Measured peak rates of the device (microbenchmarks in the library)."""
    pk = Peaks()
    _check(lib().rlwe_measure_peaks(device, ctypes.byref(pk)))
    return pk.as_dict()


def rlwe_profile_begin(ctx: int) -> None:
    _check(lib().rlwe_profile_begin(ctx))


def rlwe_profile_end(ctx: int) -> dict:
    kt = KernelTimes()
    _check(lib().rlwe_profile_end(ctx, ctypes.byref(kt)))
    return kt.as_dict()


# ------------------------------------------------------------------ conveniences

class Context:
    """Owns an rlwe_ctx handle."""

    def __init__(self, N: int, primes: Sequence[int], log2_t: int, device: int = 0,
                 log2_q_out: int = 32):
        self.N, self.primes, self.log2_t = N, tuple(int(p) for p in primes), log2_t
        self.P = len(self.primes)
        self.log2_q_out = log2_q_out
        self.handle = rlwe_params_init(N, self.primes, log2_t, device, log2_q_out)

    def close(self) -> None:
        if self.handle:
            rlwe_params_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Tuner:
    """Owns an rlwe_tuner handle (measured launch choices for one device)."""

    def __init__(self, device_key: str):
        self.handle = rlwe_tuner_create(device_key)

    def close(self) -> None:
        if self.handle:
            rlwe_tuner_destroy(self.handle)
            self.handle = 0

    def __len__(self) -> int:
        return rlwe_tuner_size(self.handle)

    def load(self, path: str) -> int:
        return rlwe_tuner_load(self.handle, path)

    def save(self, path: str) -> None:
        rlwe_tuner_save(self.handle, path)


class Weights:
    """Owns an rlwe_weights handle for a (d_out, d_in) int8 matrix."""

    def __init__(self, ctx: Context, W, flags: int = RLWE_W_FWD, stream=None):
        self.ctx = ctx
        self.d_out, self.d_in = W.shape
        self.handle = rlwe_weights_load(ctx.handle, W, flags, stream)

    def close(self) -> None:
        if self.handle:
            rlwe_weights_free(self.handle)
            self.handle = 0

    def out_rows(self, transpose: bool) -> int:
        return self.d_in if transpose else self.d_out

    def in_len(self, transpose: bool) -> int:
        return self.d_out if transpose else self.d_in


def matmul(ctx: Context, w: Weights, ct, transpose: bool = False, raw: bool = False,
           force_exact: bool = False, out=None, stream=None, seeded: bool = False):
    """Allocate the output (torch, on ct's device) and run ct_matmul_clear. seeded: ct is
    in the seeded layout (tokens, L, P N + 2)."""
    import torch
    T = ct.shape[0]
    M = w.out_rows(transpose)
    if out is None:
        shape = (T, M, ctx.P, ctx.N + 1) if raw else (T, M, ctx.N + 1)
        out = torch.empty(shape, dtype=torch.int64 if raw else torch.int32, device=ct.device)
    flags = (RLWE_OUT_RAW_Q if raw else 0) | (RLWE_OUT_FORCE_EXACT if force_exact else 0)
    flags |= RLWE_IN_SEEDED if seeded else 0
    ct_matmul_clear(ctx.handle, w.handle, ct, T, out, transpose, flags, stream)
    return out


def pack_bits(ctx: Context, switched, out=None, stream=None):
    """Bit-pack switched ciphertexts (..., len) int32 -> (..., words) int32 (torch)."""
    import torch
    length = switched.shape[-1]
    count = switched.numel() // length
    words = rlwe_packed_words(length, ctx.log2_q_out)
    if out is None:
        out = torch.empty(switched.shape[:-1] + (words,), dtype=torch.int32, device=switched.device)
    ct_pack_bits(ctx.handle, switched, count, length, out, stream)
    return out


def modswitch(ctx: Context, raw, out=None, stream=None):
    import torch
    count = raw.numel() // (ctx.P * (ctx.N + 1))
    if out is None:
        out = torch.empty(raw.shape[:-2] + (ctx.N + 1,), dtype=torch.int32, device=raw.device)
    ct_modswitch(ctx.handle, raw, count, out, stream)
    return out


class KeySwitchKey:
    """Owns an rlwe_ksk handle: the key-switching key made resident in the NTT domain."""

    def __init__(self, ctx: Context, ksk, log2_base: int, levels: int, stream=None):
        self.ctx = ctx
        self.log2_base, self.levels = log2_base, levels
        self.handle = rlwe_ksk_load(ctx.handle, ksk, log2_base, levels, stream)

    def close(self) -> None:
        if self.handle:
            rlwe_ksk_free(self.handle)
            self.handle = 0


def keyswitch_pack(ctx: Context, k: KeySwitchKey, lwe, n_pack: int | None = None,
                   raw: bool = False, out=None, stream=None):
    """Pack raw LWE ciphertexts (..., P, N+1) int64 into RLWE ciphertexts (torch): (G, 2, N)
    int32 switched, or (G, 2, P, N) int64 with raw=True."""
    import torch
    n_pack = ctx.N if n_pack is None else int(n_pack)
    count = lwe.numel() // (ctx.P * (ctx.N + 1))
    G = rlwe_packed_count(count, n_pack)
    if out is None:
        shape = (G, 2, ctx.P, ctx.N) if raw else (G, 2, ctx.N)
        out = torch.empty(shape, dtype=torch.int64 if raw else torch.int32, device=lwe.device)
    ct_keyswitch_pack(ctx.handle, k.handle, lwe, count, n_pack, out,
                      RLWE_OUT_RAW_Q if raw else RLWE_OUT_SWITCHED, stream)
    return out


def matmul_pack(ctx: Context, w: Weights, ct, k: KeySwitchKey, n_pack: int | None = None,
                transpose: bool = False, raw: bool = False, force_exact: bool = False,
                seeded: bool = False, out=None, stream=None):
    """ct_matmul_pack (torch): the product's LWE outputs, in (token, row) order, packed into
    RLWE ciphertexts (G, 2, N) int32 switched, or (G, 2, P, N) int64 with raw=True."""
    import torch
    n_pack = ctx.N if n_pack is None else int(n_pack)
    T = ct.shape[0]
    G = rlwe_packed_count(T * w.out_rows(transpose), n_pack)
    if out is None:
        shape = (G, 2, ctx.P, ctx.N) if raw else (G, 2, ctx.N)
        out = torch.empty(shape, dtype=torch.int64 if raw else torch.int32, device=ct.device)
    flags = (RLWE_OUT_RAW_Q if raw else 0) | (RLWE_OUT_FORCE_EXACT if force_exact else 0)
    flags |= RLWE_IN_SEEDED if seeded else 0
    ct_matmul_pack(ctx.handle, w.handle, ct, T, k.handle, n_pack, out, transpose, flags, stream)
    return out
