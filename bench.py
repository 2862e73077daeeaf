#!/usr/bin/env python3
"""Throughput and latency of the encrypted clear-weight product W.[x]_HE on one MI355X.

Workloads (--workload):
  serve (default)  requests from 16 clients (Poisson arrivals) over a resident 16-layer
                   Llama-3.2-1B-shaped model, each one projection forward or backward with
                   1..512 encrypted tokens, N = 4096, two 54-bit primes; HBM-budget
                   admission. Reports the sustained encrypted MACs/s of the request loop,
                   the same requests as plain per-call products, and p50/p99 latency at
                   fractions of the saturated rate.
  attn             one 2048 x 2048 projection, 128 tokens, t = 2^26 (a single
                   ct_matmul_clear per step; options for seeded input, bit-packing, packed
                   rows, KeySwitch packing).
  layer            the 14 products of one layer (7 projections forward and transposed),
                   uneven token counts, one captured graph per step, against plain calls.
  mlp              gate/up/down forward and transposed over 2048 tokens in chunks.

Every step computes Eq. (LWEdot) and the ModulusSwitch of Sec. 3.2 on synthetic, seeded
inputs resident in HBM before the timed region: int8 weights uniform in [-127, 127] and
ciphertext residues uniform in [0, q_p) (the distribution of RLWE ciphertexts under a
uniform mask). The kernels are data-oblivious apart from a rare exact-rounding route.

Prints one JSON line: value = encrypted MACs/s (d_in * d_out * tokens / s), the roofline
of the dominant kernel (its time from HIP events on its launch stream over the timed
region, its peak measured on the device by the library's microbenchmarks) and the CPU
oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

INT8_PEAK_TOPS = 5000.0  # MI355X published dense int8 matrix peak, 5.0 POP/s
# The NTT method is bound by VALU issue. Its algorithmic work is counted in 54-bit modular
# products: one per butterfly of the inverse transforms and one per pointwise product. The
# peak is the device's measured rate of that product (rlwe_measure_peaks: the kernel's
# truncated-quotient Shoup product in register-only chains). A lazy Gentleman-Sande
# butterfly is that product plus a sum and a biased difference, 15 VALU instructions
# against the product's 11 (the kernels' form); the butterfly rate at the measured issue
# rate is reported as a kernel-model ceiling beside it.
BFLY_MODEL_INSTR = 15


def measured_peaks():
    from paper_2505_07329_amd import rlwe
    pk = rlwe.rlwe_measure_peaks(0)
    return {"mul32_lane_ops_T": pk["mul32_lane_ops"] / 1e12, "modmul_G": pk["modmul"] / 1e9,
            "butterfly_G": pk["butterfly"] / 1e9, "mfma_int8_TOPS": pk["mfma_int8_ops"] / 1e12,
            "clock_mhz": pk["clock_mhz"], "compute_units": pk["compute_units"],
            "source": "rlwe_measure_peaks (register-only microbenchmarks on this GPU)"}


def tuner_path():
    """The autotuner's cache for this device, next to the package."""
    from paper_2505_07329_amd import tune
    return tune.cache_path(0)


def attach_tuner(rlwe, ctx):
    """Attach the committed autotuner cache of this device, if there is one."""
    path = tuner_path()
    t = rlwe.Tuner(rlwe.rlwe_device_key(0))
    n = t.load(path) if os.path.exists(path) else 0
    if n:
        rlwe.rlwe_ctx_set_tuner(ctx.handle, t.handle)
    info = {"file": os.path.relpath(path, ROOT), "entries": n}
    return t, info


def method_flag(args):
    from paper_2505_07329_amd import rlwe
    flag = {"auto": 0, "ntt": rlwe.RLWE_W_NTT, "toeplitz": rlwe.RLWE_W_TOEPLITZ}[args.method]
    return flag | (rlwe.RLWE_W_ROWPACK if getattr(args, "rowpack", False) else 0)


def ntt_algorithmic_bytes(products, N, P):
    """HBM bytes the NTT product kernels must move for a set of products (dicts as for
    roofline): the switched outputs (u32, N + 1 per LWE), the transformed masks
    (residue and Shoup companion per coefficient, block and prime) and the transformed
    weights (per weight polynomial, block and prime), each once."""
    total = 0
    for p in products:
        if not p["ntt"]:
            continue
        L = (p["K"] + N - 1) // N
        groups = -(-p["M"] // p.get("n_o", 1))
        total += p["T"] * p["M"] * (N + 1) * 4 + p["T"] * L * P * N * 16 + groups * L * P * N * 8
    return total


def copy_calibration(torch, dev, gib):
    """A plain copy kernel of known size (gib GiB read, the same written), run once so that a
    counter pass can scale FETCH_SIZE and WRITE_SIZE by what they read for it."""
    n = int(gib * (1 << 30)) // 4
    src = torch.zeros(n, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def product_info(rlwe, w, tr, T, M, K):
    kept, _ = rlwe.rlwe_weights_digits(w.handle, tr)
    ntt = rlwe.rlwe_weights_method(w.handle, tr) == rlwe.RLWE_METHOD_NTT
    n_o = rlwe.rlwe_weights_rows_per_product(w.handle, tr)
    return dict(T=T, M=M, K=K, kept=kept, ntt=ntt, n_o=n_o)


def roofline(products, kt, N, P, peaks, traffic=None):
    """Roofline of the dominant mask kernel of a set of products, each a dict with
    T, M (outputs per token), K, kept (digits on the matrix cores), ntt (method), n_o
    (outputs per weight polynomial, 1 unless rows are packed). Matrix cores: 2 T M N K
    kept int8 ops against the published int8 peak; NTT: per weight polynomial, token and
    prime (N/2) log2 N butterflies and L N pointwise products, one 54-bit modular product
    each, against the measured modular-product rate (the persistent launch's time counts
    as the NTT product's: its transforms and bodies are a few per cent of it). traffic:
    measured HBM bytes per launch by kernel kind ("mfma", "alu"), where known."""
    traffic = traffic or {}
    import math
    mf_ops = sum(2.0 * p["T"] * p["M"] * N * p["K"] * p["kept"] for p in products if not p["ntt"])
    nt_ops = sum(p["T"] * -(-p["M"] // p.get("n_o", 1)) * P
                 * ((N // 2) * math.log2(N) + ((p["K"] + N - 1) // N) * N)
                 for p in products if p["ntt"])
    bfly = sum(p["T"] * -(-p["M"] // p.get("n_o", 1)) * P * (N // 2) * math.log2(N)
               for p in products if p["ntt"])
    parts = {}
    if mf_ops and kt["mask_ms"] > 0:
        a = mf_ops / (kt["mask_ms"] * 1e-3) / 1e12
        parts["mfma"] = {"bound": "mfma", "achieved": a, "peak": INT8_PEAK_TOPS,
                         "unit": "TOP/s (int8)", "frac": a / INT8_PEAK_TOPS,
                         "traffic": traffic.get("mfma"), "ms": kt["mask_ms"],
                         "measured_peak": peaks["mfma_int8_TOPS"],
                         "frac_of_measured": a / peaks["mfma_int8_TOPS"]}
    ntt_ms = kt.get("ntt_ms", 0) + kt.get("persist_ms", 0)
    if nt_ops and ntt_ms > 0:
        a = nt_ops / (ntt_ms * 1e-3) / 1e9
        model = peaks["mul32_lane_ops_T"] * 1e3 / BFLY_MODEL_INSTR
        parts["alu"] = {"bound": "alu", "achieved": a, "peak": peaks["modmul_G"],
                        "unit": "G modmul/s (54-bit modular products: one per butterfly and "
                                "per pointwise product, NTT method)",
                        "frac": a / peaks["modmul_G"], "traffic": traffic.get("alu"), "ms": ntt_ms,
                        "peak_source": "measured: rlwe_measure_peaks modmul",
                        "kernel_model": {"butterflies_G_per_s": bfly / (ntt_ms * 1e-3) / 1e9,
                                         "instr_per_butterfly": BFLY_MODEL_INSTR,
                                         "ceiling_G_per_s": model,
                                         "measured_butterfly_G_per_s": peaks["butterfly_G"],
                                         "frac_of_ceiling": a / model}}
    if not parts:
        return None, None
    dom = max(parts.values(), key=lambda x: x["ms"])
    other = [v for v in parts.values() if v is not dom]
    return ({k: v for k, v in dom.items() if k != "ms"},
            {k: v for k, v in other[0].items() if k != "ms"} if other else None)

# HBM bytes moved by one launch of each mask kernel on the default workload: two
# rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by
# the ratio of known to counted bytes of a plain copy kernel in the same run
# (--copy-calibration). Valid for the kernel source it was taken on (sha256); for any
# other source the roofline reports traffic as null.
KERNEL_TRAFFIC = {
    "mask": {"sources": ["k_mask.hip"], "fetch_bytes": 4382826959, "write_bytes": 4766587301,
             "sha256": "d31818600eff6cf99abfb69ae5fdda8bf673103f1a029ac55bbd206c5b7eaf12"},
    "ntt": {"sources": ["k_ntt.hip", "ntt_product.hpp", "ntt_device.hpp", "ks_round.hpp"],
            "fetch_bytes": 5427843915,
            "write_bytes": 4331271291,
            "sha256": "4b63e1dcc950517b63600462b23f1938014968164bad10c23eb08ca900a89691"},
    # the product with masks rounded for KeySwitch packing (ct_matmul_pack, --keyswitch)
    "ntt_ks": {"sources": ["k_ntt.hip", "ntt_product.hpp", "ntt_device.hpp", "ks_round.hpp"],
               "fetch_bytes": 6331299466, "write_bytes": 8669613432,
               "sha256": "4b63e1dcc950517b63600462b23f1938014968164bad10c23eb08ca900a89691"},
    "ksacc": {"sources": ["k_keyswitch.hip", "ntt_device.hpp", "ks_round.hpp"],
              "fetch_bytes": 13007274145, "write_bytes": 536870912,
              "sha256": "282d0a1962e40c1e3caffecc5b42429e11efa078d072ba147b2bc9f0fa450cf4"},
    # the serving workload's NTT product launches (both block classes), averaged over the
    # 396 launches of the timed region of the profiled run (the grouping follows timing)
    "serve_ntt": {"sources": ["k_ntt.hip", "ntt_product.hpp", "ntt_device.hpp", "ks_round.hpp"],
                  "fetch_bytes": 118117667758, "write_bytes": 14331846432,
                  "sha256": "4b63e1dcc950517b63600462b23f1938014968164bad10c23eb08ca900a89691"},
}


def keyswitch_roofline(M, N, P, ell, acc_s, peaks):
    """Roofline of the KeySwitch accumulate kernel for M LWE ciphertexts packed N per RLWE
    ciphertext: per packed ciphertext, key coefficient, level and prime one forward
    transform ((N/2) log2 N butterflies) and 2 N pointwise products (mask and body of the
    key), one 54-bit modular product each, against the measured modular-product rate."""
    import math
    G = -(-M // N)
    work = G * N * ell * P * ((N // 2) * math.log2(N) + 2 * N)
    a = work / acc_s / 1e9
    return {"bound": "alu", "achieved": a, "peak": peaks["modmul_G"],
            "unit": "G modmul/s (54-bit modular products, KeySwitch transforms)",
            "frac": a / peaks["modmul_G"], "traffic": None,
            "peak_source": "measured: rlwe_measure_peaks modmul"}


def keyswitch_cpu_baseline(prod, N, primes, d_in, beta, ell):
    """Oracle rate of the whole path: the product rate measured by cpu_baseline and the
    oracle's packing (digits, NTT-form KeySwitch, Rotate) timed on one packed ciphertext
    of N uniform LWE ciphertexts; combined per encrypted MAC."""
    import numpy as np

    from oracle import oracle as orc
    from paper_2505_07329_amd import synth
    g = synth.rng(2, synth.P_MISC, 5)
    lwe = synth.uniform_mod_primes(g, primes, (N,), N + 1)
    ksk = synth.uniform_mod_primes(g, primes, (N, ell, 2), N)
    t0 = time.perf_counter()
    orc.keyswitch_pack(N, primes, beta, ell, lwe, ksk, N)
    el = time.perf_counter() - t0
    pack_rate = N * d_in / el  # MAC/s of the outputs packed per second
    value = 1.0 / (1.0 / prod["value"] + 1.0 / pack_rate)
    return {"value": value, "unit": "encrypted MAC/s", "cores": prod["cores"], "kind": "oracle",
            "sample": prod["sample"] + f"; plus the oracle's packing of {N} LWE ciphertexts "
                      f"into one RLWE ciphertext ({el:.1f} s, {N * d_in / el:.3g} MAC/s of outputs "
                      "packed); rates combined per MAC"}


def clear_gemm_context(torch, dev, T, d_in, d_out, he_value):
    """Context only: the same product on clear int8 data (torch._int_mm, int32 results) on the
    same GPU, and the encrypted product's slowdown against it (the HE overhead factor)."""
    try:
        a = torch.randint(-127, 128, (T, d_in), dtype=torch.int8, device=dev)
        b = torch.randint(-127, 128, (d_in, d_out), dtype=torch.int8, device=dev)
        kind = "int8 torch._int_mm"
        f = lambda: torch._int_mm(a, b)  # noqa: E731
        f()
    except Exception:  # no int8 GEMM in this build of torch: half precision instead
        a = torch.randn((T, d_in), dtype=torch.float16, device=dev)
        b = torch.randn((d_in, d_out), dtype=torch.float16, device=dev)
        kind = "fp16 torch.matmul (no int8 GEMM available)"
        f = lambda: a @ b  # noqa: E731
    for _ in range(5):
        f()
    reps = 200
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        f()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    value = T * d_in * d_out / (ms * 1e-3)
    return {"kind": kind, "value": value, "unit": "MAC/s", "ms": ms,
            "he_overhead": value / he_value}


def kernel_traffic(kind):
    import hashlib
    rec = KERNEL_TRAFFIC.get(kind)
    if not rec:
        return None
    h = hashlib.sha256()
    for name in rec["sources"]:
        with open(os.path.join(ROOT, "paper_2505_07329_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sha256"]:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def source_sha256(kind):
    """sha256 of the sources a traffic record is tied to (printed by --print-hashes)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, "paper_2505_07329_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


KERNEL_SOURCES = {"mask": ["k_mask.hip"],
                  "ntt": ["k_ntt.hip", "ntt_product.hpp", "ntt_device.hpp", "ks_round.hpp"],
                  "ntt_ks": ["k_ntt.hip", "ntt_product.hpp", "ntt_device.hpp", "ks_round.hpp"],
                  "serve_ntt": ["k_ntt.hip", "ntt_product.hpp", "ntt_device.hpp", "ks_round.hpp"],
                  "ksacc": ["k_keyswitch.hip", "ntt_device.hpp", "ks_round.hpp"]}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20; mlp: 1 pass over all 2048 tokens of 6 products)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 3; mlp: 1)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target CPU time of the oracle baseline sample (0 disables it)")
    ap.add_argument("--chunk", type=int, default=256, help="mlp: tokens per call")
    ap.add_argument("--method", choices=["auto", "ntt", "toeplitz"], default="auto",
                    help="mask-product method of every weight matrix (auto: the library's choice "
                         "by estimated time per output)")
    ap.add_argument("--q-out-bits", type=int, default=32,
                    help="attn: switched outputs modulo 2^K (the paper's output modulus is 26 bits)")
    ap.add_argument("--seeded", action="store_true",
                    help="attn: inputs in the seeded layout [seed, 0, B] per block; the masks are "
                         "expanded on the GPU")
    ap.add_argument("--pack", action="store_true",
                    help="attn: every step also bit-packs the switched outputs (ct_pack_bits), "
                         "reported with its own HBM roofline")
    ap.add_argument("--keyswitch", action="store_true",
                    help="attn: pack the outputs into RLWE ciphertexts (KeySwitch and Rotate, "
                         "Eq. (pack_rotate)), N per ciphertext, switched to 2^q-out-bits")
    ap.add_argument("--ks-base-bits", type=int, default=54, help="KeySwitch: digit bits")
    ap.add_argument("--ks-levels", type=int, default=1, help="KeySwitch: gadget levels")
    ap.add_argument("--d-in", type=int, default=None,
                    help="attn: contraction length K instead of 2048 (shape studies; the bench "
                         "line is then not the attention workload's)")
    ap.add_argument("--d-out", type=int, default=None, help="attn: output rows M instead of 2048")
    ap.add_argument("--rowpack", action="store_true",
                    help="load every weight matrix with RLWE_W_ROWPACK (floor(N / K) rows per "
                         "weight polynomial where the contraction length K <= N/2; NTT method)")
    ap.add_argument("--print-hashes", action="store_true",
                    help="print the sha256 of each kernel's sources and exit")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="attn: before the timed region, run one plain elementwise copy kernel "
                         "(int32 bitwise not) reading and writing GIB GiB each, as the known-size "
                         "reference for the FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--workload", choices=["attn", "layer", "mlp", "serve", "table4"], default="serve",
                    help="serve (default): Poisson requests from 16 clients over a resident "
                         "16-layer model, vs plain per-call kernels, p50/p99; "
                         "attn: one 2048x2048 projection, 128 tokens; layer: the 14 "
                         "products of a Llama-3.2-1B layer, forward and transposed, with uneven "
                         "token counts, captured once as a graph and replayed; mlp: gate/up/down "
                         "forward and transposed over 2048 tokens in chunks; table4: the paper's "
                         "Table 4 shapes at N = 2048, one and 16 tokens per call")
    ap.add_argument("--requests", type=int, default=500,
                    help="serve: requests per load point of the latency sweep")
    ap.add_argument("--max-tokens", type=int, default=16,
                    help="layer: token counts drawn uniformly in 1..max-tokens")
    ap.add_argument("--budget-gib", type=float, default=128.0,
                    help="serve: HBM budget of the output arena")
    ap.add_argument("--round-macs", type=float, default=1e9,
                    help="serve: MACs after which a scheduling round stops adding requests")
    ap.add_argument("--no-rowpack-run", action="store_true",
                    help="serve: skip the second saturated run with packed rows")
    ap.add_argument("--loads", default="0.5,0.8,0.95",
                    help="serve: arrival rates as fractions of the saturated request rate")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 1 if args.workload == "mlp" else 20
    if args.warmup is None:
        args.warmup = 1 if args.workload == "mlp" else 3
    return args


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_rates(sample, target_s, label):
    """The oracle's rate in its two modes (NTT: a psi-twisted transform per output and
    prime; schoolbook: the closed form of Eq. (LWEdot), d_in (N + 1) products per output
    and prime), each on all host threads and on one thread, plus the exact switch.
    sample(mode) runs one chunk of the workload's sampled outputs and returns the MACs
    it credits; each of the four runs takes about target_s / 4 seconds. value = NTT mode
    on all threads (the fastest plain-CPU form)."""
    from oracle import oracle as orc
    orc.lib()
    all_threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or (os.cpu_count() or 1)
    rates, notes = {}, []
    for mode, mname in ((1, "ntt"), (0, "schoolbook")):
        for threads, tname in ((all_threads, "all_cores"), (1, "one_core")):
            orc.set_threads(threads)
            macs, el = 0, 0.0
            while el < target_s / 4:
                t0 = time.perf_counter()
                macs += sample(mode)
                el += time.perf_counter() - t0
            rates[f"{mname}_{tname}"] = macs / el
            notes.append(f"{mname} on {threads} thread(s) {el:.1f} s")
    orc.set_threads(all_threads)
    return {"value": rates["ntt_all_cores"], "unit": "encrypted MAC/s", "cores": all_threads,
            "kind": "oracle", "cpu_model": cpu_model(), "modes": rates,
            "sample": f"{label}; oracle plus exact switch to 2^32, " + ", ".join(notes)
                      + "; scaled per MAC (the cost is linear in tokens and outputs)"}


def cpu_baseline(W, ct_np, N, primes, T, d_out, d_in, target_s, n_o=1):
    """The oracle on sampled (token, row) outputs of the same workload (same weights and
    ciphertexts); with packed rows (n_o > 1), on sampled (token, group of n_o rows)
    products by the oracle's packed-row product (one form: both mode entries are it)."""
    import numpy as np

    from oracle import oracle as orc
    g = np.random.default_rng(7)
    groups = -(-d_out // n_o)

    def sample(mode):
        if n_o > 1:
            t, gr = int(g.integers(0, T)), int(g.integers(0, groups))
            rows = W[gr * n_o:(gr + 1) * n_o]
            orc.modswitch(primes, orc.matmul_rowpacked(N, primes, rows, ct_np[t:t + 1]))
            return rows.shape[0] * d_in
        pairs = np.stack([g.integers(0, T, 16), g.integers(0, d_out, 16)], 1).astype(np.uint32)
        orc.modswitch(primes, orc.matmul_clear(N, primes, W, ct_np, pairs=pairs, mode=mode))
        return len(pairs) * d_in

    label = ("sampled (token, row) outputs of the same workload, 16 per chunk" if n_o == 1 else
             f"sampled (token, group of {n_o} packed rows) products of the same workload")
    return oracle_rates(sample, target_s, label)


def mix_cpu_baseline(shapes, N, primes, target_s, label, seed):
    """The oracle on sampled output LWEs of a mix of products (K inputs, M outputs each),
    8 outputs of each product in turn, on seeded random weights and ciphertexts of those
    shapes (the oracle's cost does not depend on the values), credited K MACs per output."""
    import numpy as np

    from oracle import oracle as orc
    g = np.random.default_rng(seed)
    data = {}
    for K, M in shapes:
        if (K, M) not in data:
            W = g.integers(-127, 128, size=(M, K), dtype=np.int64).astype(np.int8)
            L = (K + N - 1) // N
            ct = np.stack([g.integers(0, q, size=(8, L, 2, N), dtype=np.uint64) for q in primes], -2)
            data[(K, M)] = (W, ct)
    order = list(shapes)
    state = {"i": 0}

    def sample(mode):
        K, M = order[state["i"] % len(order)]
        state["i"] += 1
        W, ct = data[(K, M)]
        pairs = np.stack([g.integers(0, 8, 8), g.integers(0, M, 8)], 1).astype(np.uint32)
        orc.modswitch(primes, orc.matmul_clear(N, primes, W, ct, pairs=pairs, mode=mode))
        return len(pairs) * K

    return oracle_rates(sample, target_s, label)


LAYER_BUDGET = 250e9  # output bytes per captured graph


def layer_workload(args):
    """All 7 projections of one Llama-3.2-1B layer, forward and transposed (14 products),
    token counts drawn uniformly in 1..max_tokens (16 by default: the paper's training step
    runs one sequence of 16 tokens per call, Sec. 6.3), one captured graph replayed per
    step (launch shape from the autotuner's cache when it has the batch, else grouped),
    against the same 14 products issued as plain ct_matmul_clear calls."""
    import numpy as np
    import torch

    from paper_2505_07329_amd import rlwe, synth

    cfg = synth.WORKLOADS[4]
    N, primes, log2_t = cfg["N"], cfg["primes"], cfg["log2_t"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    peaks = measured_peaks()
    ctx = rlwe.Context(N, primes, log2_t, device=0)
    tuner, tuner_info = attach_tuner(rlwe, ctx)
    g = synth.rng(4, synth.P_MISC)
    products, weights = [], []
    for pi, (name, (d_in, d_out)) in enumerate(synth.LLAMA_1B_PROJ.items()):
        W = synth.int8_uniform(synth.rng(4, synth.P_WEIGHTS, pi), (d_out, d_in))
        w = rlwe.Weights(ctx, torch.from_numpy(W).to(dev),
                         rlwe.RLWE_W_FWD | rlwe.RLWE_W_TRANSPOSE | method_flag(args))
        weights.append(w)
        for tr in (False, True):
            K, M = (d_out, d_in) if tr else (d_in, d_out)
            T = int(g.integers(1, args.max_tokens + 1))
            products.append(dict(name=name + ("^T" if tr else ""), w=w, tr=tr, K=K, M=M, T=T))
    macs = sum(p["T"] * p["K"] * p["M"] for p in products)
    groups, cur, cur_bytes = [], [], 0
    for p in products:
        ob = p["T"] * p["M"] * (N + 1) * 4
        if cur and cur_bytes + ob > LAYER_BUDGET:
            groups.append(cur)
            cur, cur_bytes = [], 0
        cur.append(p)
        cur_bytes += ob
    groups.append(cur)
    items_per_group = []
    for grp in groups:
        items = []
        for p in grp:
            L = (p["K"] + N - 1) // N
            ct = synth.uniform_mod_primes(synth.rng(4, synth.P_MASK, len(items)), primes, (p["T"], L, 2), N)
            p["ct"] = torch.from_numpy(ct.view(np.int64)).to(dev)
            p["out"] = torch.empty((p["T"], p["M"], N + 1), dtype=torch.int32, device=dev)
            items.append((p["w"].handle, p["tr"], p["ct"], p["T"], p["out"]))
        items_per_group.append(items)
    stream = torch.cuda.current_stream()
    all_ntt = all(rlwe.rlwe_weights_method(p["w"].handle, p["tr"]) == rlwe.RLWE_METHOD_NTT
                  for p in products)

    def capture(flags):
        return [rlwe.rlwe_graph_capture_batch(ctx.handle, items, flags) for items in items_per_group]

    def step_graph(graphs):
        for gr in graphs:
            rlwe.rlwe_graph_launch(gr, stream)

    def step_plain():
        for p in products:
            rlwe.ct_matmul_clear(ctx.handle, p["w"].handle, p["ct"], p["T"], p["out"], p["tr"],
                                 rlwe.RLWE_OUT_SWITCHED, stream)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    rlwe.rlwe_workspace_reserve(ctx.handle, max(
        rlwe.rlwe_workspace_bytes(ctx.handle, p["w"].handle, p["tr"], p["T"]) for p in products))
    t_plain = timed(step_plain, max(1, args.steps // 2), 1)
    shapes = {}
    for name, flags in (("grouped", rlwe.RLWE_LAUNCH_GROUPED),
                        ("persistent", rlwe.RLWE_LAUNCH_PERSISTENT if all_ntt else None)):
        if flags is None:
            continue
        gr = capture(flags)
        shapes[name] = timed(lambda: step_graph(gr), max(1, args.steps // 2), 1) * 1e3
        for x in gr:
            rlwe.rlwe_graph_destroy(x)
    graphs = capture(rlwe.RLWE_OUT_SWITCHED)  # the launch the tuner chose
    t_graph = timed(lambda: step_graph(graphs), args.steps, args.warmup)
    rlwe.rlwe_profile_begin(ctx.handle)
    step_plain()
    torch.cuda.synchronize()
    kt = rlwe.rlwe_profile_end(ctx.handle)
    roof, roof_other = roofline([product_info(rlwe, p["w"], p["tr"], p["T"], p["M"], p["K"])
                                 for p in products], kt, N, len(primes), peaks)
    cpu = None
    if args.cpu_seconds > 0:
        cpu = mix_cpu_baseline([(p["K"], p["M"]) for p in products], N, primes, args.cpu_seconds,
                               "sampled output LWEs, 8 from each of the 14 products in turn", 4)
    value = macs / t_graph
    result = {
        "metric": "encrypted MACs/s (sum d_in*d_out*tokens / s), one Llama-3.2-1B layer, 7 projections "
                  "forward and transposed in one captured graph, vs plain per-call kernels",
        "value": value, "unit": "MAC/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_graph * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64 (54-bit RNS residues)",
        "data": "synthetic (seeded uniform int8 weights, uniform ciphertext residues)",
        "config": {"workload": cfg["name"], "N": N, "primes": len(primes), "log2_t": log2_t,
                   "tokens": f"U{{1..{args.max_tokens}}}",
                   "products": [f'{p["name"]}:{p["K"]}->{p["M"]}x{p["T"]}' for p in products],
                   "graphs": len(graphs),
                   "output_GB": sum(p["T"] * p["M"] * (N + 1) * 4 for p in products) / 1e9},
        "plain_per_call": {"value": macs / t_plain, "ms_per_step": t_plain * 1e3,
                           "speedup_graph": t_plain / t_graph},
        "launch_shapes_ms": shapes, "tuner": tuner_info,
        "methods": {p["name"]: ("ntt" if rlwe.rlwe_weights_method(p["w"].handle, p["tr"]) else "toeplitz")
                    for p in products},
        "roofline": roof, "roofline_other_method": roof_other, "peaks": peaks,
        "cpu_baseline": cpu,
    }
    for gr in graphs:
        rlwe.rlwe_graph_destroy(gr)
    for w in weights:
        w.close()
    rlwe.rlwe_ctx_set_tuner(ctx.handle, None)
    tuner.close()
    ctx.close()
    print(json.dumps(result), flush=True)

MLP_TOKENS = 2048


def mlp_workload(args):
    """Llama-3.2-1B MLP over 2048 encrypted tokens (batch 4 x context 512): gate and up
    (2048 -> 8192) and down (8192 -> 2048) forward, and the backward products with their
    transposes (gate^T, up^T: 8192 -> 2048; down^T: 2048 -> 8192). One step is one pass
    over all six products and all tokens, issued as plain ct_matmul_clear calls of
    `chunk` tokens that alternate between two output slots (one full product's switched
    output is 275 GB; the slots stand in for the transfer buffers of a server)."""
    import numpy as np
    import torch

    from paper_2505_07329_amd import rlwe, synth

    cfg = synth.WORKLOADS[3]
    N, primes, log2_t = cfg["N"], cfg["primes"], cfg["log2_t"]
    T, C = MLP_TOKENS, args.chunk
    if T % C:
        raise SystemExit("--chunk must divide 2048")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    peaks = measured_peaks()
    ctx = rlwe.Context(N, primes, log2_t, device=0)
    tuner, tuner_info = attach_tuner(rlwe, ctx)
    mats = {}
    for pi, name in enumerate(("gate", "up", "down")):
        d_in, d_out = synth.LLAMA_1B_PROJ[name]
        W = synth.int8_uniform_device(3, synth.P_WEIGHTS, pi, (d_out, d_in), dev)
        mats[name] = rlwe.Weights(ctx, W, rlwe.RLWE_W_FWD | rlwe.RLWE_W_TRANSPOSE | method_flag(args))
        del W
    cts = {}
    for L in (1, 2):
        ct = synth.uniform_mod_primes(synth.rng(3, synth.P_MASK, L), primes, (T, L, 2), N)
        cts[L] = torch.from_numpy(ct.view(np.int64)).to(dev)
        del ct
    products = []
    for name in ("gate", "up", "down"):
        w = mats[name]
        for tr in (False, True):
            K, M = (w.d_out, w.d_in) if tr else (w.d_in, w.d_out)
            products.append(dict(name=name + ("^T" if tr else ""), w=w, tr=tr, K=K, M=M,
                                 L=(K + N - 1) // N))
    Mmax = max(p["M"] for p in products)
    slots = [torch.empty((C, Mmax, N + 1), dtype=torch.int32, device=dev) for _ in range(2)]
    rlwe.rlwe_workspace_reserve(ctx.handle, max(
        rlwe.rlwe_workspace_bytes(ctx.handle, p["w"].handle, p["tr"], C) for p in products))
    stream = torch.cuda.current_stream()

    def one_pass(chunks):
        k = 0
        for p in products:
            for c in range(chunks):
                out = slots[k % 2][:, : p["M"]] if p["M"] == Mmax else \
                    slots[k % 2].view(-1)[: C * p["M"] * (N + 1)].view(C, p["M"], N + 1)
                rlwe.ct_matmul_clear(ctx.handle, p["w"].handle, cts[p["L"]][c * C:(c + 1) * C], C,
                                     out, p["tr"], rlwe.RLWE_OUT_SWITCHED, stream)
                k += 1

    for _ in range(args.warmup):
        one_pass(1)
    torch.cuda.synchronize()
    rlwe.rlwe_profile_begin(ctx.handle)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_pass(T // C)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = rlwe.rlwe_profile_end(ctx.handle)
    macs = args.steps * T * sum(p["K"] * p["M"] for p in products)
    roof, roof_other = roofline([product_info(rlwe, p["w"], p["tr"], args.steps * T, p["M"], p["K"])
                                 for p in products], kt, N, len(primes), peaks)
    cpu = None
    if args.cpu_seconds > 0:
        cpu = mix_cpu_baseline([(p["K"], p["M"]) for p in products], N, primes, args.cpu_seconds,
                               "sampled output LWEs, 8 from each of the six products in turn", 9)
    result = {
        "metric": "encrypted MACs/s (sum d_in*d_out*tokens / s), Llama-3.2-1B MLP forward and backward "
                  "through the frozen weights, outputs switched to 2^32",
        "value": macs / wall, "unit": "MAC/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64 (54-bit RNS residues)",
        "data": "synthetic (seeded uniform int8 weights, uniform ciphertext residues)",
        "config": {"workload": cfg["name"], "N": N, "primes": len(primes), "log2_t": log2_t,
                   "tokens": T, "chunk": C,
                   "products": [f'{p["name"]}:{p["K"]}->{p["M"]}' for p in products],
                   "digits_on_matrix_cores": {p["name"]: rlwe.rlwe_weights_digits(p["w"].handle, p["tr"])[0]
                                              for p in products}},
        "kernels_ms": {"prep": kt["prep_ms"], "mask": kt["mask_ms"], "ntt": kt["ntt_ms"],
                       "persistent": kt["persist_ms"], "body": kt["body_ms"]},
        "methods": {p["name"]: ("ntt" if rlwe.rlwe_weights_method(p["w"].handle, p["tr"]) else "toeplitz")
                    for p in products},
        "roofline": roof, "roofline_other_method": roof_other, "peaks": peaks,
        "tuner": tuner_info, "cpu_baseline": cpu,
    }
    for w in mats.values():
        w.close()
    rlwe.rlwe_ctx_set_tuner(ctx.handle, None)
    tuner.close()
    ctx.close()
    print(json.dumps(result), flush=True)


SERVE_LAYERS = 16
SERVE_CLIENTS = 16
SERVE_MAX_TOKENS = 512


# Sec. 6.3, Table 4: latency of one encrypted product W.[x] per shape (d_in -> d_out) on one
# NVIDIA RTX 4060 Laptop GPU at the Table 1 parameters (N = 2048, 39-bit input and
# 26-bit output moduli), seconds. Context only: other hardware, other moduli.
TABLE4_PAPER_S = {(768, 768): 0.0809, (3072, 768): 0.1528, (2048, 2048): 0.2402,
                  (768, 3072): 0.3389, (8192, 2048): 0.6368, (2048, 8192): 1.0539}


def table4_workload(args):
    """The six product shapes of the paper's Table 4 at N = 2048 with one 54-bit prime,
    outputs switched to 2^26 (Table 1's output modulus), t = 2^28 (room for 8192-input
    rows). One step is one call of each shape with one token; the same with 16 tokens
    (the paper's training step runs 16 tokens per call) is timed after it. Each shape's
    launch is tuned on the spot (rlwe_autotune_product)."""
    import numpy as np
    import torch

    from paper_2505_07329_amd import rlwe, synth

    N, primes, log2_t, qbits = 2048, synth.PRIMES_2048, 28, 26
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    peaks = measured_peaks()
    ctx = rlwe.Context(N, primes, log2_t, device=0, log2_q_out=qbits)
    tuner = rlwe.Tuner(rlwe.rlwe_device_key(0))
    for (d_in, d_out) in TABLE4_PAPER_S:
        for T in (1, 16):
            rlwe.rlwe_autotune_product(ctx.handle, tuner.handle, d_in, d_out, T)
    rlwe.rlwe_ctx_set_tuner(ctx.handle, tuner.handle)
    stream = torch.cuda.current_stream()
    shapes = []
    for si, (d_in, d_out) in enumerate(TABLE4_PAPER_S):
        W = synth.int8_uniform(synth.rng(1, synth.P_WEIGHTS, 10 + si), (d_out, d_in))
        w = rlwe.Weights(ctx, torch.from_numpy(W).to(dev), rlwe.RLWE_W_FWD)
        L = (d_in + N - 1) // N
        per_T = {}
        for T in (1, 16):
            ct = synth.uniform_mod_primes(synth.rng(1, synth.P_MASK, 10 + si), primes, (T, L, 2), N)
            per_T[T] = (torch.from_numpy(ct.view(np.int64)).to(dev),
                        torch.empty((T, d_out, N + 1), dtype=torch.int32, device=dev))
        shapes.append(dict(d_in=d_in, d_out=d_out, w=w, per_T=per_T,
                           method="ntt" if rlwe.rlwe_weights_method(w.handle) else "toeplitz"))
    rlwe.rlwe_workspace_reserve(ctx.handle, max(
        rlwe.rlwe_workspace_bytes(ctx.handle, sh["w"].handle, False, 16) for sh in shapes))

    def call(sh, T):
        ct, out = sh["per_T"][T]
        rlwe.ct_matmul_clear(ctx.handle, sh["w"].handle, ct, T, out, False, rlwe.RLWE_OUT_SWITCHED,
                             stream)

    def step(T):
        for sh in shapes:
            call(sh, T)

    for _ in range(args.warmup):
        step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    macs1 = sum(sh["d_in"] * sh["d_out"] for sh in shapes)
    rows = []
    for sh in shapes:
        lat = {}
        for T in (1, 16):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            call(sh, T)
            e0.record(stream)
            for _ in range(args.steps):
                call(sh, T)
            e1.record(stream)
            torch.cuda.synchronize()
            lat[T] = e0.elapsed_time(e1) / args.steps
        paper = TABLE4_PAPER_S[(sh["d_in"], sh["d_out"])]
        rows.append({"d_in": sh["d_in"], "d_out": sh["d_out"], "method": sh["method"],
                     "ms_1_token": lat[1], "ms_16_tokens": lat[16],
                     "macs_per_s_1_token": sh["d_in"] * sh["d_out"] / (lat[1] * 1e-3),
                     "macs_per_s_16_tokens": 16 * sh["d_in"] * sh["d_out"] / (lat[16] * 1e-3),
                     "paper_s": paper, "paper_over_ours_1_token": paper / (lat[1] * 1e-3)})
    cpu = None
    if args.cpu_seconds > 0:
        cpu = mix_cpu_baseline([(sh["d_in"], sh["d_out"]) for sh in shapes], N, primes,
                               args.cpu_seconds, "sampled output LWEs, 8 from each of the six shapes "
                               "in turn", 1)
    result = {
        "metric": "encrypted MACs/s (d_in*d_out*tokens/s), one token per call, over the six product "
                  "shapes of the paper's Table 4",
        "value": args.steps * macs1 / wall, "unit": "MAC/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64 (54-bit residues)",
        "data": "synthetic (seeded uniform int8 weights, uniform ciphertext residues)",
        "config": {"workload": "table4-shapes-N2048-P1", "N": N, "primes": 1, "log2_t": log2_t,
                   "q_out": f"2^{qbits}", "tokens": 1},
        "shapes": rows,
        "context": "paper: one RTX 4060 Laptop GPU, N = 2048, 39-bit input modulus (Sec. 6.3, "
                   "Table 4); here: one MI355X, one 54-bit prime",
        "peaks": peaks, "cpu_baseline": cpu,
    }
    for sh in shapes:
        sh["w"].close()
    rlwe.rlwe_ctx_set_tuner(ctx.handle, None)
    tuner.close()
    ctx.close()
    print(json.dumps(result), flush=True)


SERVE_STEP_REQUESTS = 25  # requests per step of the saturated run


def serve_workload(args):
    """Requests from 16 clients over a resident 16-layer Llama-3.2-1B-shaped model, each one
    projection forward or backward with 1..512 tokens. One step is SERVE_STEP_REQUESTS
    requests; the timed region serves `steps` steps of requests queued at once (saturated:
    grouped launches of up to 16 requests per scheduling round), after `warmup` steps
    served untimed. The same requests as one plain call each are the comparator. Then
    Poisson arrivals at fractions of the saturated request rate, `requests` per load
    point, report p50/p99 latency and sustained MACs/s."""
    import math

    import numpy as np
    import torch

    from paper_2505_07329_amd import rlwe, serve, synth

    cfg = synth.WORKLOADS[5]
    N, primes, log2_t = cfg["N"], cfg["primes"], cfg["log2_t"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    peaks = measured_peaks()
    ctx = rlwe.Context(N, primes, log2_t, device=0)
    tuner, tuner_info = attach_tuner(rlwe, ctx)
    t_setup = time.perf_counter()
    weights = {}
    for layer in range(SERVE_LAYERS):
        for pi, (name, (d_in, d_out)) in enumerate(synth.LLAMA_1B_PROJ.items()):
            W = synth.int8_uniform_device(5, synth.P_WEIGHTS, layer * 16 + pi, (d_out, d_in), dev)
            weights[(layer, name)] = rlwe.Weights(ctx, W, rlwe.RLWE_W_FWD | rlwe.RLWE_W_TRANSPOSE
                                                  | method_flag(args))
            del W
    pools = {}
    for L in (1, 2):
        ct = synth.uniform_mod_primes(synth.rng(5, synth.P_MASK, L), primes, (SERVE_MAX_TOKENS, L, 2), N)
        pools[L] = torch.from_numpy(ct.view(np.int64)).to(dev)
    budget = int(args.budget_gib * (1 << 30))
    arena = torch.empty(budget, dtype=torch.uint8, device=dev)
    # workspace of the largest possible group: 16 requests of 512 tokens with two input blocks
    w_big = weights[(0, "down")]
    big = [(w_big.handle, False, pools[2], SERVE_MAX_TOKENS, arena[:4])] * 16
    rlwe.rlwe_workspace_reserve(ctx.handle, rlwe.rlwe_batch_workspace_bytes(ctx.handle, big))
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    stream = torch.cuda.current_stream()
    backend = serve.GpuBackend(ctx, weights, pools, arena, stream)
    out_bytes = serve.switched_out_bytes(N)

    def requests(n, rate, salt):
        g = synth.rng(5, synth.P_MISC, salt)
        return serve.make_requests(synth.LLAMA_1B_PROJ, SERVE_LAYERS, SERVE_CLIENTS, n,
                                   rate, g, out_bytes, SERVE_MAX_TOKENS)

    def run(reqs, max_batch):
        sched = serve.Scheduler(serve.RingArena(budget), max_batch=max_batch,
                                max_round_macs=args.round_macs)
        return serve.run_loop(reqs, sched, backend, time.perf_counter,
                              lambda dt: time.sleep(min(dt, 0.05)))

    n_sat = args.steps * SERVE_STEP_REQUESTS
    if args.warmup:
        run(requests(args.warmup * SERVE_STEP_REQUESTS, math.inf, 99), 16)
        run(requests(2, math.inf, 98), 1)
    sat_reqs = requests(n_sat, math.inf, 0)
    if args.copy_calibration > 0:
        copy_calibration(torch, dev, args.copy_calibration)
    rlwe.rlwe_profile_begin(ctx.handle)
    torch.cuda.synchronize()  # one GPU: the barrier is this synchronisation
    t0 = time.perf_counter()
    sat = run(sat_reqs, 16)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = rlwe.rlwe_profile_end(ctx.handle)
    print(json.dumps({"progress": "saturated", "requests": sat["requests"], "wall_s": wall}),
          file=sys.stderr, flush=True)
    infos = [product_info(rlwe, weights[(r.layer, r.proj)], r.transpose, r.tokens, r.d_out, r.d_in)
             for r in sat_reqs]
    roof, roof_other = roofline(infos, kt, N, len(primes), peaks,
                                traffic={"alu": kernel_traffic("serve_ntt")})
    if roof is not None and roof["bound"] == "alu" and kt["ntt_n"]:
        # the NTT product launches of the timed region (their number follows the grouping)
        roof["launches"] = kt["ntt_n"]
        roof["algorithmic_bytes"] = ntt_algorithmic_bytes(infos, N, len(primes)) / kt["ntt_n"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plain = run(requests(n_sat, math.inf, 0), 1)
    torch.cuda.synchronize()
    plain_wall = time.perf_counter() - t1
    print(json.dumps({"progress": "plain per call", "wall_s": plain_wall}), file=sys.stderr, flush=True)
    macs = sat["macs"]
    sat_rate = sat["requests"] / wall
    sweep = []
    for i, f in enumerate(float(x) for x in args.loads.split(",") if x):
        res = run(requests(args.requests, f * sat_rate, 1 + i), 16)
        sweep.append({"load": f, "rate_req_s": f * sat_rate, "p50_ms": res["p50_s"] * 1e3,
                      "p99_ms": res["p99_s"] * 1e3, "mean_ms": res["mean_s"] * 1e3,
                      "macs_per_s": res["macs_per_s"], "requests": res["requests"],
                      "rejected": res["rejected"], "expired": res["expired"]})
        print(json.dumps({"progress": "load point", **sweep[-1]}), file=sys.stderr, flush=True)
    head = min(sweep, key=lambda x: abs(x["load"] - 0.8)) if sweep else None
    cpu = None
    if args.cpu_seconds > 0:
        cpu = mix_cpu_baseline([(r.d_in, r.d_out) for r in sat_reqs], N, primes, args.cpu_seconds,
                               "sampled output LWEs, 8 from each request of the served mix in "
                               "turn", 8)
    packed = None
    if not args.rowpack and not args.no_rowpack_run and args.method != "toeplitz":
        # the same saturated requests with the weights reloaded with packed rows (n_o = N / K
        # rows per weight polynomial where K <= N/2; Cheetah-style coefficient packing):
        # same decryptions, other ciphertexts
        for key in list(weights):
            weights[key].close()
        for layer in range(SERVE_LAYERS):
            for pi, (name, (d_in, d_out)) in enumerate(synth.LLAMA_1B_PROJ.items()):
                W = synth.int8_uniform_device(5, synth.P_WEIGHTS, layer * 16 + pi, (d_out, d_in), dev)
                weights[(layer, name)] = rlwe.Weights(
                    ctx, W, rlwe.RLWE_W_FWD | rlwe.RLWE_W_TRANSPOSE | method_flag(args)
                    | rlwe.RLWE_W_ROWPACK)
                del W
        backend.weights = weights
        run(requests(SERVE_STEP_REQUESTS, math.inf, 97), 16)  # warm-up
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        psat = run(requests(n_sat, math.inf, 0), 16)
        torch.cuda.synchronize()
        pwall = time.perf_counter() - t2
        t3 = time.perf_counter()
        run(requests(n_sat, math.inf, 0), 1)
        torch.cuda.synchronize()
        pplain = time.perf_counter() - t3
        packed = {"value": psat["macs"] / pwall, "ms_per_step": pwall * 1e3 / args.steps,
                  "saturated_p50_ms": psat["p50_s"] * 1e3, "saturated_p99_ms": psat["p99_s"] * 1e3,
                  "plain_per_call_value": psat["macs"] / pplain,
                  "speedup_vs_unpacked": wall / pwall,
                  "what": "the same saturated requests with RLWE_W_ROWPACK weights (floor(N/K) "
                          "rows per weight polynomial where K <= N/2): same decryptions, other "
                          "ciphertexts"}
        print(json.dumps({"progress": "packed rows", "wall_s": pwall}), file=sys.stderr, flush=True)
    result = {
        "metric": "encrypted MACs/s (sum d_in*d_out*tokens / s) vs plain kernel; p50/p99 request "
                  "latency",
        "value": macs / wall, "unit": "MAC/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64 (54-bit RNS residues)",
        "data": "synthetic (seeded uniform int8 weights of 16 layers, uniform ciphertext residues, "
                "Poisson arrivals)",
        "config": {"workload": cfg["name"], "N": N, "primes": len(primes), "log2_t": log2_t,
                   "layers": SERVE_LAYERS, "clients": SERVE_CLIENTS, "tokens": "U{1..512}",
                   "requests_per_step": SERVE_STEP_REQUESTS, "requests_per_load_point": args.requests,
                   "budget_GiB": args.budget_gib, "max_batch": 16, "round_macs": args.round_macs,
                   "setup_s": t_setup},
        "latency_ms": ({"load": head["load"], "p50": head["p50_ms"], "p99": head["p99_ms"],
                        "requests": head["requests"]} if head else None),
        "saturated": {"requests": sat["requests"], "p50_ms": sat["p50_s"] * 1e3,
                      "p99_ms": sat["p99_s"] * 1e3, "rate_req_s": sat_rate, "wall_s": wall},
        "plain_per_call": {"value": macs / plain_wall, "ms_per_step": plain_wall * 1e3 / args.steps,
                           "speedup_served": plain_wall / wall,
                           "what": "the same requests, one ct_matmul_clear each, in arrival order"},
        "sweep": sweep, "rowpack_saturated": packed, "tuner": tuner_info,
        "kernels_ms": {"ntt": kt["ntt_ms"], "persistent": kt["persist_ms"], "mask": kt["mask_ms"],
                       "prep": kt["prep_ms"], "body": kt["body_ms"]},
        "roofline": roof, "roofline_other_method": roof_other, "peaks": peaks,
        "cpu_baseline": cpu,
    }
    for w in weights.values():
        w.close()
    rlwe.rlwe_ctx_set_tuner(ctx.handle, None)
    tuner.close()
    ctx.close()
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.print_hashes:
        print(json.dumps({k: source_sha256(k) for k in KERNEL_SOURCES}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the encrypted product shards by tokens or output "
              "rows with no exchange, and it is measured on one MI355X; use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "layer":
        layer_workload(args)
        return
    if args.workload == "serve":
        serve_workload(args)
        return
    if args.workload == "mlp":
        mlp_workload(args)
        return
    if args.workload == "table4":
        table4_workload(args)
        return
    import numpy as np
    import torch

    from paper_2505_07329_amd import rlwe, synth

    cfg = dict(synth.WORKLOADS[2])
    N, primes, log2_t = cfg["N"], cfg["primes"], cfg["log2_t"]
    d_in, d_out, T = args.d_in or cfg["d_in"], args.d_out or cfg["d_out"], cfg["tokens"]
    shape_default = (d_in, d_out) == (cfg["d_in"], cfg["d_out"])
    if not shape_default:  # a shape study: named by its shape, no traffic record applies
        cfg["name"] = f"shape-{d_out}x{d_in}-T{T}-N{N}-P{len(primes)}"
        # t large enough that no row can overflow (127 * row 1-norm < t / 2)
        while (1 << (log2_t - 1)) <= 127 * 127 * d_in:
            log2_t += 1
    L = (d_in + N - 1) // N
    W = synth.int8_uniform(synth.rng(2, synth.P_WEIGHTS), (d_out, d_in))
    ct_np = synth.uniform_mod_primes(synth.rng(2, synth.P_MASK), primes, (T, L, 2), N)
    if args.seeded:  # [seed, 0, B] per block; seeds and bodies seeded and uniform
        g = synth.rng(2, synth.P_MISC)
        in_np = np.zeros((T, L, len(primes) * N + 2), dtype=np.uint64)
        in_np[:, :, 0] = g.integers(0, 2**63, size=(T, L), dtype=np.uint64)
        in_np[:, :, 2:] = ct_np[:, :, 1].reshape(T, L, len(primes) * N)
    else:
        in_np = ct_np

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    peaks = measured_peaks()
    qbits = args.q_out_bits
    ctx = rlwe.Context(N, primes, log2_t, device=0, log2_q_out=qbits)
    tuner, tuner_info = attach_tuner(rlwe, ctx)
    w = rlwe.Weights(ctx, torch.from_numpy(W).to(dev), rlwe.RLWE_W_FWD | method_flag(args))
    ct = torch.from_numpy(in_np.view(np.int64)).to(dev)
    in_flags = rlwe.RLWE_IN_SEEDED if args.seeded else 0
    P = len(primes)
    ks = args.keyswitch
    if ks:  # the product's LWE outputs packed N per RLWE ciphertext, switched (one call)
        G = rlwe.rlwe_packed_count(T * d_out, N)
        rlwe_out = torch.empty((G, 2, N), dtype=torch.int32, device=dev)
        # a key of uniform residues: the kernels are data-oblivious (the tests use real keys)
        gen = torch.Generator(device=dev)
        gen.manual_seed(synth.SEED_BASE + 2000 + synth.P_MISC)
        ksk_t = torch.empty((N, args.ks_levels, 2, P, N), dtype=torch.int64, device=dev)
        for p_, q_ in enumerate(primes):
            ksk_t[:, :, :, p_].random_(0, q_, generator=gen)
        key = rlwe.KeySwitchKey(ctx, ksk_t, args.ks_base_bits, args.ks_levels)
        del ksk_t
        words = rlwe.rlwe_packed_words(N, qbits)
        packed = torch.empty((G, 2, words), dtype=torch.int32, device=dev) if args.pack else None
    else:
        out = torch.empty((T, d_out, N + 1), dtype=torch.int32, device=dev)
        words = rlwe.rlwe_packed_words(N + 1, qbits)
        packed = torch.empty((T, d_out, words), dtype=torch.int32, device=dev) if args.pack else None
    ws = rlwe.rlwe_workspace_bytes(ctx.handle, w.handle, False, T)
    if ks:
        ws = max(ws, rlwe.rlwe_matmul_pack_workspace_bytes(ctx.handle, w.handle, False, T,
                                                           key.handle, N))
    rlwe.rlwe_workspace_reserve(ctx.handle, ws)
    kept, total = rlwe.rlwe_weights_digits(w.handle)
    stream = torch.cuda.current_stream()

    def step():
        if ks:
            rlwe.ct_matmul_pack(ctx.handle, w.handle, ct, T, key.handle, N, rlwe_out, False,
                                rlwe.RLWE_OUT_SWITCHED | in_flags, stream)
            if args.pack:
                rlwe.ct_pack_bits(ctx.handle, rlwe_out, G * 2, N, packed, stream)
            return
        rlwe.ct_matmul_clear(ctx.handle, w.handle, ct, T, out, False,
                             rlwe.RLWE_OUT_SWITCHED | in_flags, stream)
        if args.pack:
            rlwe.ct_pack_bits(ctx.handle, out, T * d_out, N + 1, packed, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.copy_calibration > 0:
        copy_calibration(torch, dev, args.copy_calibration)

    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    rlwe.rlwe_profile_begin(ctx.handle)
    torch.cuda.synchronize()  # one GPU: the barrier is this synchronisation
    t0 = time.perf_counter()
    for k in range(args.steps):
        marks[k].record(stream)
        step()
    marks[-1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = rlwe.rlwe_profile_end(ctx.handle)

    macs = d_in * d_out * T
    value = macs * args.steps / wall
    lat = np.array([marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps)])
    per_launch = {k: kt[k] / max(1, kt[k.replace("_ms", "_n")])
                  for k in ("prep_ms", "mask_ms", "ntt_ms", "body_ms", "persist_ms")}
    one = dict(kt, mask_ms=per_launch["mask_ms"], ntt_ms=per_launch["ntt_ms"],
               persist_ms=per_launch["persist_ms"])
    is_ntt = rlwe.rlwe_weights_method(w.handle) == rlwe.RLWE_METHOD_NTT
    n_o = rlwe.rlwe_weights_rows_per_product(w.handle)
    roof, _ = roofline([dict(T=T, M=d_out, K=d_in, kept=kept, ntt=is_ntt, n_o=n_o)], one, N,
                       len(primes), peaks,
                       traffic={"mfma": None if ks or not shape_default else kernel_traffic("mask"),
                                "alu": None if n_o != 1 or not shape_default else
                                kernel_traffic("ntt_ks" if ks else "ntt")})
    ks_roof = None
    if ks and kt["ksacc_n"]:
        ks_ms = {k: kt[f"ks{k}_ms"] / max(1, kt[f"ks{k}_n"]) * kt[f"ks{k}_n"] / args.steps
                 for k in ("dig", "acc", "fin")}  # per step (a step may hold several passes)
        ks_roof = keyswitch_roofline(T * d_out, N, P, args.ks_levels, ks_ms["acc"] * 1e-3, peaks)
        ks_roof["traffic"] = kernel_traffic("ksacc") if shape_default else None
        # the digit kernel reads the rounded masks (NTT method) or the raw residues
        read = 8 * N if is_ntt else P * 8 * (N + 1)
        ks_roof["digits_hbm_gbs"] = (T * d_out * (read + args.ks_levels * 8 * N)
                                     / (ks_ms["dig"] * 1e-3) / 1e9)
    pack_roof = None
    if args.pack and kt["pack_n"]:
        pack_ms = kt["pack_ms"] / kt["pack_n"]
        n_ct, ln = (G * 2, N) if ks else (T * d_out, N + 1)
        moved = n_ct * 4 * (ln + words)  # switched words read once, packed words written
        gbs = moved / (pack_ms * 1e-3) / 1e9
        pack_roof = {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                     "frac": gbs / 8000.0, "traffic": None, "ms": pack_ms,
                     "bytes_out_per_lwe": 4 * words}
        if ks:
            pack_roof["bytes_out_per_rlwe"] = pack_roof.pop("bytes_out_per_lwe") * 2
    switched = f"switched to 2^{qbits}" + (" and bit-packed" if args.pack else "")
    if ks:
        switched = (f"packed {N} per RLWE ciphertext (KeySwitch + Rotate), " + switched)
    result = {
        "metric": f"encrypted MACs/s (d_in*d_out*tokens/s), W.[x]_HE with outputs {switched}",
        "value": value,
        "unit": "MAC/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 (54-bit RNS residues)",
        "data": "synthetic (seeded uniform int8 weights, uniform ciphertext residues)",
        "config": {"workload": cfg["name"], "d_in": d_in, "d_out": d_out, "tokens": T, "N": N,
                   "primes": len(primes), "log2_t": log2_t, "q_out": f"2^{qbits}",
                   "packed": bool(args.pack), "seeded_input": bool(args.seeded),
                   "input_bytes": int(in_np.nbytes),
                   "method": "ntt" if is_ntt else "toeplitz", "rows_per_product": n_o,
                   "digits_on_matrix_cores": None if is_ntt else f"{kept}/{total}",
                   "keyswitch": ({"n_pack": N, "log2_base": args.ks_base_bits,
                                  "levels": args.ks_levels, "packed_ciphertexts": G}
                                 if ks else None)},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "kernels_ms": {"prep": per_launch["prep_ms"], "mask": per_launch["mask_ms"],
                       "ntt": per_launch["ntt_ms"], "persistent": per_launch["persist_ms"],
                       "body": per_launch["body_ms"]},
        "roofline": roof, "peaks": peaks, "tuner": tuner_info,
        "cpu_baseline": None,
    }
    if pack_roof:
        result["kernels_ms"]["pack"] = pack_roof.pop("ms")
        result["roofline_pack"] = pack_roof
    result["clear_gemm_context"] = clear_gemm_context(torch, dev, T, d_in, d_out, macs * args.steps / wall)
    if ks_roof:
        result["kernels_ms"].update({"ks_digits": ks_ms["dig"], "ks_accum": ks_ms["acc"],
                                     "ks_finish": ks_ms["fin"]})
        # the dominant kernel of the step carries the headline roofline
        if roof is None or ks_ms["acc"] > max(per_launch["ntt_ms"], per_launch["mask_ms"],
                                              per_launch["persist_ms"]):
            result["roofline"], result["roofline_product"] = ks_roof, roof
        else:
            result["roofline_keyswitch"] = ks_roof
        key.close()
    w.close()
    rlwe.rlwe_ctx_set_tuner(ctx.handle, None)
    tuner.close()
    ctx.close()
    if args.cpu_seconds > 0:
        result["cpu_baseline"] = cpu_baseline(W, ct_np, N, primes, T, d_out, d_in,
                                              args.cpu_seconds / 2 if ks else args.cpu_seconds, n_o)
        if ks:
            result["cpu_baseline"] = keyswitch_cpu_baseline(result["cpu_baseline"], N, primes, d_in,
                                                            args.ks_base_bits, args.ks_levels)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
