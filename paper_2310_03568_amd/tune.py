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
  wins at none;
* ``seg.tile`` in {4096, 8192} and ``seg.fwd.threads`` / ``seg.vjp.threads``
  in {256, 512, 1024}: the batched plan's item size and block sizes, timed
  on the segmented workload (4096 instances of lognormal length, median
  4096; 1024 instances with ``quick``): per item size the fastest forward
  and adjoint block sizes, then the item size with the smaller sum.

Cache entries are keyed by (combinator, op, n-bucket, m-bucket, skew): the
buckets are round(log2 n) and round(log2 m) of the shape the entry was
searched on and the key distribution ("uniform", "zipf", "uniform+zipf" for
thresholds searched under both, "lognormal" for the batched instance
lengths).  The cache records the device it was measured on; ``load``
applies it only on the same device name and architecture, otherwise the
built-in defaults stay.  ``load(path, key=...)`` applies the entry that
matches the key's combinator and op (and skew, when both give one) with the
nearest buckets; without a key every entry is applied.
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


def bucket(x: Optional[int]) -> Optional[int]:
    """round(log2 x): the n- and m-buckets of cache keys (None stays None)"""
    import math
    return None if not x else int(round(math.log2(x)))


def key(combinator: str, op: str, n: Optional[int] = None, m: Optional[int] = None,
        skew: Optional[str] = None) -> dict:
    return {"combinator": combinator, "op": op, "n_bucket": bucket(n), "m_bucket": bucket(m),
            "skew": skew}


def tune_scan(pcad, timings: dict, quick: bool, entries: list) -> dict:
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
        entries.append({"key": key("scan", op, n),
                        "knobs": {f"scan.{d}.threads.{op}": best[f"scan.{d}.threads.{op}"]
                                  for d in ("fwd", "vjp")}})
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


def tune_rbi(pcad, timings: dict, quick: bool, entries: list) -> dict:
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
    # thresholds over m were searched under both key distributions
    entries.append({"key": key("rbi", "add", n, None, "uniform+zipf"),
                    "knobs": {k: best[k] for k in ("rbi.lds_max_bins_f32", "rbi.sort_min_bins")}})
    entries.append({"key": key("rbi", "min", n, None, "uniform+zipf"),
                    "knobs": {"rbi.lds_max_bins_u64": best["rbi.lds_max_bins_u64"]}})
    entries.append({"key": key("rbi", "add", n, 256, "uniform"),
                    "knobs": {"rbi.elems_per_block": best["rbi.elems_per_block"]}})
    return best


def tune_segmented(pcad, timings: dict, quick: bool, entries: list) -> dict:
    """Item size and block sizes of the batched plan on the segmented
    workload: per item size the fastest forward and adjoint block sizes, then
    the item size whose forward + adjoint is smaller."""
    import numpy as np
    from workloads import segmented
    w = segmented(S=1024 if quick else 4096)
    per_tile = {}
    for tile in (4096, 8192):
        tf, tb = {}, {}
        for th in THREADS:
            pcad.reset_knobs()
            pcad.set_knob("seg.tile", tile)
            pcad.set_knob("seg.fwd.threads", th)
            pcad.set_knob("seg.vjp.threads", th)
            plan = pcad.BatchedPlan(w["offsets"], w["m"])
            plan.load(a=w["a"], b=w["b"], idx=w["idx"], ybar=w["ybar"], hbar=w["hbar"])
            tf[th] = _time(lambda: plan.run(pcad.PHASE_FWD), 5 if quick else 10)
            tb[th] = _time(lambda: plan.run(pcad.PHASE_BWD), 5 if quick else 10)
            plan.close()
            timings[f"seg@tile={tile},threads={th}"] = {"fwd": tf[th], "vjp": tb[th]}
        f, b = min(tf, key=tf.get), min(tb, key=tb.get)
        per_tile[tile] = (tf[f] + tb[b], f, b)
    pcad.reset_knobs()
    tile = min(per_tile, key=lambda t: per_tile[t][0])
    best = {"seg.tile": tile, "seg.fwd.threads": per_tile[tile][1],
            "seg.vjp.threads": per_tile[tile][2]}
    entries.append({"key": key("batched", "linrec+min", int(w["n_total"]), w["m"], "lognormal"),
                    "knobs": dict(best)})
    return best


def tune(out: Optional[str] = DEFAULT_PATH, quick: bool = False) -> dict:
    """Runs the search on cuda:0, writes the cache (if ``out``) and returns
    it.  The knobs are left at their built-in defaults afterwards; ``load``
    applies a cache."""
    import paper_2310_03568_amd as pcad
    pcad.lib()
    t0 = time.time()
    timings: dict = {}
    entries: list = []
    best = {}
    best.update(tune_scan(pcad, timings, quick, entries))
    best.update(tune_rbi(pcad, timings, quick, entries))
    best.update(tune_segmented(pcad, timings, quick, entries))
    cache = {"version": 2, "device": _device_id(), "entries": entries, "knobs": best,
             "timings_s": timings, "quick": quick, "seconds": time.time() - t0}
    if out:
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        with open(out, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return cache


def _match(entries: list, want: dict) -> Optional[dict]:
    """The entry for combinator/op (and skew, when both name one) whose
    buckets are nearest to the wanted ones; None if no entry qualifies."""
    def dist(a, b):
        return 0 if a is None or b is None else abs(a - b)
    best, best_d = None, None
    for e in entries:
        k = e.get("key", {})
        if k.get("combinator") != want.get("combinator") or k.get("op") != want.get("op"):
            continue
        ks, ws = k.get("skew"), want.get("skew")
        if ks is not None and ws is not None and ws not in ks.split("+"):
            continue
        d = dist(k.get("n_bucket"), want.get("n_bucket")) + dist(k.get("m_bucket"), want.get("m_bucket"))
        if best_d is None or d < best_d:
            best, best_d = e, d
    return best


def load(path: str = DEFAULT_PATH, device: Optional[dict] = None,
         key: Optional[dict] = None) -> bool:
    """Applies a tuning cache; returns False (built-in defaults kept) when it
    is missing, unreadable, was measured on another device, or (with
    ``key``) holds no entry for that combinator and op."""
    import paper_2310_03568_amd as pcad
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        return False
    if cache.get("version") != 2 or not isinstance(cache.get("entries"), list):
        return False
    if device is None:
        device = _device_id()
    if cache.get("device") != device:
        return False
    if key is None:
        chosen = cache["entries"]
    else:
        e = _match(cache["entries"], key)
        if e is None:
            return False
        chosen = [e]
    pcad.reset_knobs()
    for e in chosen:
        for name, value in e.get("knobs", {}).items():
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
