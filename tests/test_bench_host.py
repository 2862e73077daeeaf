"""Host logic of bench.py (no GPU): the roofline accounting of both methods, the
algorithmic bytes of the NTT products, the source-hash guard of the measured traffic
records, and the one-GPU contract."""

import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

PEAKS = {"modmul_G": 3000.0, "mfma_int8_TOPS": 4400.0, "mul32_lane_ops_T": 37.5,
         "butterfly_G": 2400.0}


def test_roofline_ntt_counts_butterflies_and_pointwise_products():
    N, P, T, M, K = 4096, 2, 128, 2048, 2048
    prod = dict(T=T, M=M, K=K, kept=9, ntt=True, n_o=1)
    dom, other = bench.roofline([prod], {"ntt_ms": 8.0, "mask_ms": 0.0}, N, P, PEAKS)
    work = T * M * P * ((N // 2) * math.log2(N) + N)  # one block: N pointwise products
    assert dom["bound"] == "alu" and other is None
    assert dom["achieved"] == pytest.approx(work / 8e-3 / 1e9)
    assert dom["frac"] == pytest.approx(dom["achieved"] / PEAKS["modmul_G"])
    # two input blocks: twice the pointwise products; packed rows: fewer polynomials
    two = dict(prod, K=8192)
    dom2, _ = bench.roofline([two], {"ntt_ms": 8.0, "mask_ms": 0.0}, N, P, PEAKS)
    assert dom2["achieved"] == pytest.approx(T * M * P * ((N // 2) * 12 + 2 * N) / 8e-3 / 1e9)
    packed = dict(prod, n_o=2)
    dom3, _ = bench.roofline([packed], {"ntt_ms": 8.0, "mask_ms": 0.0}, N, P, PEAKS)
    assert dom3["achieved"] == pytest.approx(dom["achieved"] / 2)


def test_roofline_matrix_cores_and_the_dominant_kernel():
    N, P = 4096, 2
    mf = dict(T=128, M=2048, K=512, kept=9, ntt=False, n_o=1)
    nt = dict(T=128, M=2048, K=2048, kept=9, ntt=True, n_o=1)
    kt = {"ntt_ms": 8.0, "mask_ms": 7.0}
    dom, other = bench.roofline([mf, nt], kt, N, P, PEAKS)
    assert dom["bound"] == "alu" and other["bound"] == "mfma"  # the longer kernel dominates
    ops = 2.0 * 128 * 2048 * N * 512 * 9
    assert other["achieved"] == pytest.approx(ops / 7e-3 / 1e12)
    assert other["peak"] == bench.INT8_PEAK_TOPS
    assert other["frac_of_measured"] == pytest.approx(other["achieved"] / PEAKS["mfma_int8_TOPS"])


def test_algorithmic_bytes_of_the_ntt_products():
    N, P = 4096, 2
    prod = dict(T=128, M=2048, K=2048, kept=9, ntt=True, n_o=1)
    out = 128 * 2048 * (N + 1) * 4         # switched outputs, u32
    masks = 128 * 1 * P * N * 16           # transformed masks with Shoup companions
    weights = 2048 * 1 * P * N * 8         # transformed weight polynomials
    assert bench.ntt_algorithmic_bytes([prod], N, P) == out + masks + weights == 4447010816
    two = dict(prod, K=8192)               # two input blocks: twice the masks and weights
    assert bench.ntt_algorithmic_bytes([two], N, P) == out + 2 * masks + 2 * weights
    packed = dict(prod, n_o=2)             # half the weight polynomials
    assert bench.ntt_algorithmic_bytes([packed], N, P) == out + masks + weights // 2
    mf = dict(prod, ntt=False)             # matrix-core products are not counted
    assert bench.ntt_algorithmic_bytes([prod, mf], N, P) == out + masks + weights


def test_traffic_records_follow_their_sources(monkeypatch):
    for kind, rec in bench.KERNEL_TRAFFIC.items():
        good = dict(rec, sha256=bench.source_sha256(kind))
        monkeypatch.setitem(bench.KERNEL_TRAFFIC, kind, good)
        assert bench.kernel_traffic(kind) == rec["fetch_bytes"] + rec["write_bytes"]
        monkeypatch.setitem(bench.KERNEL_TRAFFIC, kind, dict(rec, sha256="0" * 64))
        assert bench.kernel_traffic(kind) is None  # sources changed since the measurement
    assert bench.kernel_traffic("no such kernel") is None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert "one GPU" in (r.stdout + r.stderr)
