"""Autotuner for the library's launch knobs: grid search on the GPU, a JSON
cache, and the built-in defaults as the deterministic fallback.

    python -m paper_2310_03568_amd.tune [--out PATH] [--quick]

Knobs (see ``pcad_knob_*`` in include/pcad.h) never change results, only
speed.  Each group is searched on the shapes of the workloads it serves:

* ``scan.fwd.threads.<op>`` / ``scan.vjp.threads.<op>`` in {256, 512, 1024}:
  block size of the scan kernels over the same 8192-element tiles, timed on a
  forward (or adjoint) scan of n = 2^24 elements (2^22 for MAT2) with the
  value distributions of the workloads;
* ``rbi.lds_max_bins_f32`` / ``rbi.lds_max_bins_u64``: the bin count up to
  which reduce-by-index keeps a private LDS histogram per block rather than
  using global atomics -- the largest tested m at which the LDS strategy wins
  under both uniform and Zipf(1.1) keys (the skew buckets);
* ``rbi.elems_per_block``: elements per histogram block, timed at m = 256;
* ``rbi.sort_min_bins``: the smallest tested bin count beyond the LDS
  capacity from which sorting by bin (then a segmented scan) beats the LDS
  hash table under both key distributions; 2^26 (never, below that) if it
  wins at none.

The cache records the device it was measured on; ``load`` applies it only on
the same device name and architecture, otherwise the built-in defaults stay.
"""
from __future__ import annotations

import argparse
import json
import os
import time
from typing import Optional

DEFAULT_PATH = os.environ.get("PCAD_TUNE_CACHE",
                              os.path.join(os.path.expanduser("~"), ".cache", "pcad", "tune.json"))
THREADS = (256, 512, 1024)
SCAN_OPS = ("add", "mul", "min", "max", "linrec", "mat2")


def _device_id():
    import torch
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", "")}


def _time(fn, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def _scan_inputs(op: str, n: int):
    import torch
    g = torch.Generator(device="cuda").manual_seed(231003568)
    dev = "cuda"
    if op == "linrec":
        a = torch.rand(n, device=dev, generator=g) * 0.1 + 0.9
        b = torch.randn(n, device=dev, generator=g)
        return a, b, torch.randn(n, device=dev, generator=g)
    if op == "mat2":
        M = torch.randn(n, 4, device=dev, generator=g) * 0.5 ** 0.5
        return M, None, torch.randn(n, 4, device=dev, generator=g)
    x = torch.rand(n, device=dev, generator=g) * 1.5 + 0.5
    return x, None, torch.randn(n, device=dev, generator=g)


def tune_scan(pcad, timings: dict, quick: bool) -> dict:
    best = {}
    ops = ("add", "linrec", "mat2") if quick else SCAN_OPS
    for op in ops:
        n = (1 << 22) if op == "mat2" else (1 << 24)
        if quick:
            n >>= 2
        x0, x1, yb = _scan_inputs(op, n)
        for direction in ("fwd", "vjp"):
            name = f"scan.{direction}.threads.{op}"
            res = {}
            for th in THREADS:
                pcad.set_knob(name, th)
                _, _, saved = pcad.scan_fwd(op, x0, x1)
                if direction == "fwd":
                    res[th] = _time(lambda: pcad.scan_fwd(op, x0, x1), 5 if quick else 10)
                else:
                    res[th] = _time(lambda: pcad.scan_vjp(op, x0, x1, saved, yb), 5 if quick else 10)
            pcad.reset_knobs()
            best[name] = min(res, key=res.get)
            timings[name] = {str(k): v for k, v in res.items()}
    return best


def _rbi_inputs(n: int, m: int, zipf: bool):
    import numpy as np
    import torch
    rng = np.random.default_rng(231003568 + m)
    if zipf:
        # P(bin r-1) proportional to r^-1.1, by inverse CDF
        cdf = np.cumsum(np.arange(1, m + 1, dtype=np.float64) ** -1.1)
        idx = np.minimum(np.searchsorted(cdf / cdf[-1], rng.random(n), side="right"),
                         m - 1).astype(np.int32)
    else:
        idx = rng.integers(0, m, n).astype(np.int32)
    v = rng.standard_normal(n).astype(np.float32)
    return torch.from_numpy(idx).cuda(), torch.from_numpy(v).cuda()


def tune_rbi(pcad, timings: dict, quick: bool) -> dict:
    best = {}
    n = (1 << 22) if quick else (1 << 24)
    for kind, ops, knob in (("f32", ("add",), "rbi.lds_max_bins_f32"),
                            ("u64", ("min",), "rbi.lds_max_bins_u64")):
        hi = 8192 if kind == "f32" else 4096
        threshold = 0
        for m in (256, 1024, 4096, 8192):
            if m > hi:
                break
            lds_wins = True
            for zipf in (False, True):
                idx, v = _rbi_inputs(n, m, zipf)
                t = {}
                for strat, val in (("lds", hi), ("global", 0)):
                    pcad.set_knob(knob, val)
                    t[strat] = _time(lambda: pcad.rbi_fwd(ops[0], idx, v, m), 5)
                timings[f"{knob}@m={m},{'zipf' if zipf else 'uniform'}"] = t
                lds_wins = lds_wins and t["lds"] <= t["global"]
            pcad.reset_knobs()
            if lds_wins:
                threshold = m
            else:
                break
        best[knob] = threshold
    idx, v = _rbi_inputs(n, 256, False)
    res = {}
    for epb in (4096, 8192, 16384, 32768, 65536):
        pcad.set_knob("rbi.elems_per_block", epb)
        res[epb] = _time(lambda: pcad.rbi_fwd("add", idx, v, 256), 5)
    pcad.reset_knobs()
    best["rbi.elems_per_block"] = min(res, key=res.get)
    timings["rbi.elems_per_block"] = {str(k): t for k, t in res.items()}
    never = 1 << 26
    threshold = never
    for m in ((1 << 16, 1 << 20) if quick else (1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22)):
        sort_wins = True
        for zipf in (False, True):
            idx, v = _rbi_inputs(n, m, zipf)
            t = {}
            for strat, val in (("hash", never), ("sorted", 0)):
                pcad.set_knob("rbi.sort_min_bins", val)
                t[strat] = _time(lambda: pcad.rbi_fwd("add", idx, v, m), 5)
            timings[f"rbi.sort_min_bins@m={m},{'zipf' if zipf else 'uniform'}"] = t
            sort_wins = sort_wins and t["sorted"] <= t["hash"]
        pcad.reset_knobs()
        if sort_wins:
            threshold = m
            break
    best["rbi.sort_min_bins"] = threshold
    return best


def tune(out: Optional[str] = DEFAULT_PATH, quick: bool = False) -> dict:
    """Runs the search on cuda:0, writes the cache (if ``out``) and returns
    it.  The knobs are left at their built-in defaults afterwards; ``load``
    applies a cache."""
    import paper_2310_03568_amd as pcad
    pcad.lib()
    t0 = time.time()
    timings: dict = {}
    best = {}
    best.update(tune_scan(pcad, timings, quick))
    best.update(tune_rbi(pcad, timings, quick))
    cache = {"version": 1, "device": _device_id(), "knobs": best, "timings_s": timings,
             "quick": quick, "seconds": time.time() - t0}
    if out:
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        with open(out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return cache


def load(path: str = DEFAULT_PATH, device: Optional[dict] = None) -> bool:
    """Applies a tuning cache; returns False (built-in defaults kept) when it
    is missing, unreadable, or was measured on another device."""
    import paper_2310_03568_amd as pcad
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        return False
    if cache.get("version") != 1 or not isinstance(cache.get("knobs"), dict):
        return False
    if device is None:
        device = _device_id()
    if cache.get("device") != device:
        return False
    pcad.reset_knobs()
    for name, value in cache["knobs"].items():
        pcad.set_knob(name, int(value))
    return True


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_PATH)
    ap.add_argument("--quick", action="store_true", help="smaller shapes, fewer operators")
    args = ap.parse_args()
    cache = tune(args.out, args.quick)
    print(json.dumps({"knobs": cache["knobs"], "seconds": round(cache["seconds"], 1)}), flush=True)


if __name__ == "__main__":
    main()
