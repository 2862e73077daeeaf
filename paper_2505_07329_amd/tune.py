"""Autotuning of the launch shapes for the Llama-3.2-1B-shaped workloads.

    python -m paper_2505_07329_amd.tune [--buckets 1,4,16,64,512] [--out PATH]

Times, on device 0, every candidate launch shape (method, NTT token tile, block order,
grouped or persistent launch) of each projection of one layer (q, k, v, o, gate, up,
down), forward and transposed, N = 4096, two 54-bit primes, at the given token counts,
plus the launch of the layer's 14-product batch, through the library's
rlwe_autotune_product / rlwe_autotune_batch, and writes the choices to the device's
cache file (paper_2505_07329_amd/tuned/<arch>-<compute units>cu.json), which a context
loads with rlwe_tuner_load. The measurements are this device's; the file says which
device it was written for, and a tuner for another device skips its entries.
"""

from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

_HERE = os.path.dirname(os.path.abspath(__file__))


def cache_path(device: int = 0) -> str:
    """The cache file of a device: tuned/<gfx arch>-<compute units>cu.json."""
    from paper_2505_07329_amd import rlwe
    key = rlwe.rlwe_device_key(device)
    arch = re.sub(r"[^A-Za-z0-9]", "", key.split(":")[0].split("|")[0]) or "device"
    cus = key.rsplit("|", 1)[-1]
    return os.path.join(_HERE, "tuned", f"{arch}-{cus}cu.json")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--buckets", default="1,4,16,64,512",
                    help="token counts to tune each product for (a call uses the nearest)")
    ap.add_argument("--out", default=None, help="cache file (default: the device's)")
    ap.add_argument("--raw", action="store_true", help="also tune raw (mod q) outputs")
    args = ap.parse_args(argv)

    import numpy as np
    import torch

    from paper_2505_07329_amd import rlwe, synth

    N, primes, log2_t = 4096, synth.PRIMES_4096, 28
    path = args.out or cache_path(0)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = rlwe.Context(N, primes, log2_t, device=0)
    tuner = rlwe.Tuner(rlwe.rlwe_device_key(0))
    if os.path.exists(path):
        tuner.load(path)
    buckets = [int(x) for x in args.buckets.split(",") if x]
    t0 = time.perf_counter()
    oflags = [rlwe.RLWE_OUT_SWITCHED] + ([rlwe.RLWE_OUT_RAW_Q] if args.raw else [])
    for name, (d_in, d_out) in synth.LLAMA_1B_PROJ.items():
        for K, M in ((d_in, d_out), (d_out, d_in)):  # forward, transposed
            for T in buckets:
                for wflags in (0, rlwe.RLWE_W_ROWPACK):
                    if wflags and 2 * K > N:
                        continue  # packed rows need K <= N/2
                    for of in oflags:
                        best = rlwe.rlwe_autotune_product(ctx.handle, tuner.handle, K, M, T, wflags, of)
                        print(json.dumps({"progress": "product", "proj": name, "K": K, "M": M, "T": T,
                                          "rowpack": bool(wflags), "raw": of == rlwe.RLWE_OUT_RAW_Q,
                                          **best}), flush=True)
    # the layer batch: 14 products with the tuned per-product choices, at small and
    # large token counts
    rlwe.rlwe_ctx_set_tuner(ctx.handle, tuner.handle)
    for rowpack in (0, rlwe.RLWE_W_ROWPACK):
        for tmax in (16, 512):
            g = np.random.default_rng(tmax + rowpack)
            ws, items = [], []
            for pi, (name, (d_in, d_out)) in enumerate(synth.LLAMA_1B_PROJ.items()):
                W = torch.randint(-127, 128, (d_out, d_in), dtype=torch.int8, device=dev)
                w = rlwe.Weights(ctx, W, rlwe.RLWE_W_FWD | rlwe.RLWE_W_TRANSPOSE | rowpack)
                ws.append(w)
                for tr in (False, True):
                    K, M = (d_out, d_in) if tr else (d_in, d_out)
                    T = tmax if pi == 0 and not tr else int(g.integers(1, tmax + 1))
                    ct = torch.from_numpy(synth.uniform_mod_primes(g, primes, (T, (K + N - 1) // N, 2), N)
                                          .view(np.int64)).to(dev)
                    out = torch.empty((T, M, N + 1), dtype=torch.int32, device=dev)
                    items.append((w.handle, tr, ct, T, out))
            rlwe.rlwe_workspace_reserve(ctx.handle, rlwe.rlwe_batch_workspace_bytes(ctx.handle, items))
            best = rlwe.rlwe_autotune_batch(ctx.handle, tuner.handle, items)
            print(json.dumps({"progress": "layer batch", "rowpack": bool(rowpack), "T_max": tmax,
                              **best}), flush=True)
            del items
            for w in ws:
                w.close()
    rlwe.rlwe_ctx_set_tuner(ctx.handle, None)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tuner.save(path)
    print(json.dumps({"saved": os.path.relpath(path), "entries": len(tuner),
                      "seconds": time.perf_counter() - t0}), flush=True)
    tuner.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
