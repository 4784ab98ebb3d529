"""Benchmark: forward + reverse-mode adjoint on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pass of the hot path over one batch of synthetic input that is
already resident in HBM: the forward and the adjoint.  Prints one JSON line.

Workloads:
  segmented -- 4096 instances (lognormal lengths, median 4096, total about
             2^26): linear-recurrence scan -> min-by-index into 512 bins,
             forward + adjoint, each phase one hipGraph launch (default).
  linrec  -- linear-recurrence scan y_i = a_i y_{i-1} + b_i, n = 2^26, fp32,
             forward + adjoint w.r.t. a and b.
  mat2    -- 2x2 matrix-product scan, n = 2^24, entries ~ N(0, 0.5).
  rbi     -- reduce-by-index, n = 2^26 values into --bins bins (uniform or
             Zipf(1.1) keys), operator --op; extras: a sweep over
             m in {256, 65536, 2^22} x both key distributions x + * min max.
  vec     -- vectorised scan (map2 --op) over 2^20 rows of 64 floats, with
             vectorised reduce and reduce-by-index timings as extras.
  autograd -- 64 x 2^16 loss forward + backward through torch.autograd.
  matd    -- scan of --d x --d matrix products (3 or 5), n = 10^7
             (the evaluation's smaller dataset), Haar-orthogonal factors.

`value` is backward elements/s: n / (mean duration of the adjoint kernel,
HIP events on the stream the kernel runs on).  `roofline` prices that kernel
against the 8 TB/s HBM peak with the algorithmic bytes of the adjoint.
`roofline.copy_GBs` is the faster of two device copies measured in the same
run (torch's copy kernel, `copy_plain_GBs`, and the library's streaming copy
with nontemporal loads and stores, `copy_stream_GBs`) and `frac_of_copy` the
adjoint's rate over it.  Times are means over the
timed steps (30 by default), with 95% confidence half-widths and medians.
`cpu_baseline` is the CPU FP64 oracle timed on the host (1 thread) on the
same inputs; its outputs also gate the GPU results (`parity`).
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

HBM_PEAK_GBS = 8000.0
METRIC = "backward elems/s + % HBM peak, batched vs per-segment, at 1e-5 rel err"


# the source files each timed kernel is built from (its own file and the
# headers it includes): the traffic counters stay valid while these do
KERNEL_SOURCES = {
    "k_seg_bwd": ("batched.hip", "device.hpp", "adjoint.hpp"),
    "k_scan_vjp": ("scan.hip", "device.hpp", "adjoint.hpp"),
    "k_scan_vjp_d": ("scan.hip", "device.hpp", "adjoint.hpp"),
    "k_scan_vjp_m2d": ("scan.hip", "device.hpp", "adjoint.hpp"),
    "k_rbi_vjp": ("rbi.hip", "device.hpp"),
    "k_part_scatter": ("rbi_part.hip", "device.hpp"),
    "k_md_vapply": ("matd.hip", "device.hpp"),
}


def sources_digest(kernel: str) -> str:
    import hashlib
    src = os.path.join(ROOT, "paper_2310_03568_amd", "csrc")
    h = hashlib.sha1()
    for f in KERNEL_SOURCES[kernel.split("<")[0]]:
        h.update(open(os.path.join(src, f), "rb").read())
    return h.hexdigest()[:12]


def _traffic(kernel: str, workload: str):
    """HBM bytes per launch measured with rocprofv3 FETCH_SIZE/WRITE_SIZE,
    scaled by a plain copy kernel; None when the kernel's sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    digest = sources_digest(kernel)
    for line in open(path):
        parts = line.split()
        if len(parts) >= 4 and parts[0] == kernel and parts[1] == workload and parts[2] == digest:
            return float(parts[3])
    return None


def bench_linrec(args, pcad, torch, np):
    from workloads import linrec
    n = args.n or (1 << 26)
    w = linrec(n=n)
    dev = torch.device("cuda:0")
    A = torch.from_numpy(w["a"]).to(dev)
    B = torch.from_numpy(w["b"]).to(dev)
    YB = torch.from_numpy(w["ybar"]).to(dev)
    y = torch.empty_like(A)
    ab = torch.empty_like(A)
    bb = torch.empty_like(A)

    def fwd():
        return pcad.scan_fwd("linrec", A, B)

    def bwd(saved):
        pcad.scan_vjp("linrec", A, B, saved, YB, out=(ab, bb))

    # algorithmic bytes: fwd reads a, b and writes y; adjoint reads a, b,
    # ybar and writes a_bar, b_bar (the forward prefixes are recomputed)
    return dict(n=n, fwd=fwd, bwd=bwd, bytes_fwd=12 * n, bytes_bwd=20 * n,
                kernel="k_scan_vjp_d<LINREC>", inputs=w,
                out=lambda: (ab, bb), cfg={"workload": "linrec scan, n=2^26, fp32 (a~U[0.9,1), b~N(0,1))",
                                           "n": n, "op": "linrec", "combinator": "scan"})


def bench_mat2(args, pcad, torch, np):
    from workloads import mat2
    n = args.n or (1 << 24)
    w = mat2(n=n)
    dev = torch.device("cuda:0")
    M = torch.from_numpy(w["M"]).to(dev)
    PB = torch.from_numpy(w["Pbar"]).to(dev)
    mb = torch.empty_like(M)

    def fwd():
        return pcad.scan_fwd("mat2", M)

    def bwd(saved):
        pcad.scan_vjp("mat2", M, None, saved, PB, out=(mb,))

    return dict(n=n, fwd=fwd, bwd=bwd, bytes_fwd=32 * n, bytes_bwd=48 * n,
                kernel="k_scan_vjp_m2d<MAT2>", inputs=w, out=lambda: (mb,),
                cfg={"workload": "2x2 matrix-product scan, n=2^24, fp32 (entries ~N(0,0.5))",
                     "n": n, "op": "mat2", "combinator": "scan"})


def bench_matd(args, pcad, torch, np):
    from workloads import matd
    d = args.d
    n = args.n or 10_000_000
    w = matd(d, n)
    dev = torch.device("cuda:0")
    M = torch.from_numpy(w["M"][0]).to(dev)
    PB = torch.from_numpy(w["Pbar"][0]).to(dev)
    mb = torch.empty_like(M)

    def fwd():
        P, saved = pcad.matd_scan_fwd(M)
        return P, None, saved

    def bwd(saved):
        pcad.matd_scan_vjp(M, saved, PB, out=mb)

    e = 4 * d * d
    return dict(n=n, fwd=fwd, bwd=bwd, bytes_fwd=2 * e * n, bytes_bwd=3 * e * n,
                kernel=f"k_md_vapply<{d}>", inputs=w, out=lambda: (mb,), dev=(M, PB),
                cfg={"workload": f"{d}x{d} matrix-product scan, n={n}, fp32 (Haar-orthogonal factors)",
                     "n": n, "op": f"mat{d}", "combinator": "scan"})


def matd_extras(b, torch, np, reps=5):
    """Reduce of the same matrices: forward and adjoint times."""
    import paper_2310_03568_amd as pcad
    M, _ = b["dev"]
    d = M.shape[-1]
    yb = torch.randn(d, d, device=M.device)
    out = torch.empty_like(M)
    Y, saved = pcad.matd_reduce_fwd(M)
    pcad.matd_reduce_vjp(M, saved, yb, out=out)
    torch.cuda.synchronize()
    tf, tb = [], []
    s = torch.cuda.current_stream()
    for _ in range(reps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(s)
        Y, saved = pcad.matd_reduce_fwd(M)
        e[1].record(s)
        pcad.matd_reduce_vjp(M, saved, yb, out=out)
        e[2].record(s)
        torch.cuda.synchronize()
        tf.append(e[0].elapsed_time(e[1]))
        tb.append(e[1].elapsed_time(e[2]))
    n = b["n"]
    return {"reduce_fwd_ms": float(np.mean(tf)), "reduce_bwd_ms": float(np.mean(tb)),
            "reduce_fwd_GBs": 4 * d * d * n / (np.mean(tf) * 1e-3) / 1e9}


def matd_parity(b, torch, np, sample: int = 1 << 14):
    """Forward: the timed run's first `sample` outputs against the oracle on
    that prefix (a scan prefix depends on nothing after it).  Adjoint: the
    library on the prefix alone against the oracle.  The oracle's adjoint
    time on the prefix is the cpu_baseline."""
    import oracle
    import paper_2310_03568_amd as pcad
    from oracle.gate import RTOL, gate
    M, PB = b["dev"]
    w = b["inputs"]
    Mh, Pbh = w["M"][0][:sample], w["Pbar"][0][:sample]
    P, _, _ = b["fwd"]()
    P = P[:sample].cpu().numpy()
    Ms = M[:sample].contiguous()
    _, saved = pcad.matd_scan_fwd(Ms)
    g = pcad.matd_scan_vjp(Ms, saved, PB[:sample].contiguous()).cpu().numpy()
    rs, c = oracle.matd_scan(Mh)
    t0 = time.perf_counter()
    xb, cx = oracle.matd_scan_vjp(Mh, Pbh)
    dt = time.perf_counter() - t0
    d2 = Mh.shape[-1] ** 2
    r1 = gate(P, rs, np.repeat(c, d2).reshape(rs.shape), RTOL["mat2"])
    r2 = gate(g, xb, np.repeat(cx, d2).reshape(xb.shape), RTOL["mat2"])
    cpu = {"value": sample / dt, "unit": "elem/s", "cores": 1, "kind": "oracle",
           "sample": f"first {sample} elements of the row: oracle adjoint incl. its forward, fp64, {dt:.2f} s"}
    par = dict(ok=r1["ok"] and r2["ok"] and r1["n_range_exceeded"] == 0 and r2["n_range_exceeded"] == 0,
               max_rel_fwd=r1["max_rel"], max_rel_bwd=r2["max_rel"], sample=sample)
    return cpu, par


def bench_segmented(args, pcad, torch, np):
    """4096 instances of lognormal length (median 4096, total about 2^26):
    linear-recurrence scan -> min-by-index into 512 bins, forward and
    adjoint, each phase one hipGraph launch."""
    from workloads import segmented
    w = segmented(S=args.segments)
    plan = pcad.BatchedPlan(w["offsets"], w["m"], per_segment=True)
    plan.load(a=w["a"], b=w["b"], idx=w["idx"], ybar=w["ybar"], hbar=w["hbar"])
    N, S, m = plan.n, plan.nseg, plan.m

    def fwd():
        plan.run(pcad.PHASE_FWD)
        return None, None, None

    def bwd(_saved):
        plan.run(pcad.PHASE_BWD)

    return dict(n=N, fwd=fwd, bwd=bwd, plan=plan, inputs=w,
                # forward reads a, b, idx and writes y (+ h, argk per bin);
                # adjoint reads a, y, y_bar, idx and writes a_bar, b_bar (+ argk,
                # h_bar per bin): the prefixes y_{i-1} come from the forward's y
                bytes_fwd=16 * N + 8 * S * m, bytes_bwd=24 * N + 8 * S * m,
                kernel="k_seg_bwd", out=lambda: (plan.abar[:N], plan.bbar[:N]),
                cfg={"workload": f"segmented: {S} instances, lognormal lengths (median 4096, cap 2^20), "
                                 f"linrec scan -> min-by-index into {m} bins, fwd+adjoint, fp32",
                     "instances": S, "elements": N, "bins": m, "work_items": plan.n_items,
                     "combinator": "scan+reduce_by_index", "op": "linrec+min"})


def bench_rbi(args, pcad, torch, np):
    """Reduce-by-index of n = 2^26 values into m bins (uniform or Zipf(1.1)
    keys, values ~ N(0,1)): the histogram forward and its adjoint."""
    from workloads import rbi
    n = args.n or (1 << 26)
    m, op = args.bins, args.op
    w = rbi(op, n=n, m=m, dist=args.dist)
    dev = torch.device("cuda:0")
    I = torch.from_numpy(w["idx"]).to(dev)
    V = torch.from_numpy(w["v"]).to(dev)
    HB = torch.from_numpy(w["hbar"]).to(dev)
    vb = torch.empty_like(V)
    state = {}

    def fwd():
        h, saved = pcad.rbi_fwd(op, I, V, m)
        state["h"] = h
        return None, None, saved

    def bwd(saved):
        pcad.rbi_vjp(op, I, V, m, saved, HB, out=vb)

    # compulsory bytes.  Forward: reads idx, v; writes the bins (+ saved per
    # bin: n0 and y_pos for *, argk for min/max).  Adjoint: reads idx (+ v
    # for *), writes v_bar, and reads each bin's hbar (+ saved) once; min/max
    # need no keys (v_bar is zero except at each bin's arg-extremum)
    per_bin = {"add": 4, "mul": 12, "min": 8, "max": 8, "sumprod": 8}[op]
    per_elem_bwd = {"add": 8, "mul": 12, "min": 4, "max": 4, "sumprod": 12}[op]
    return dict(n=n, fwd=fwd, bwd=bwd, inputs=w, bytes_fwd=8 * n + per_bin * m,
                bytes_bwd=per_elem_bwd * n + per_bin * m, kernel=f"k_rbi_vjp<{op.upper()}>",
                out=lambda: (state["h"], vb),
                cfg={"workload": f"reduce_by_index {op}, n=2^{n.bit_length() - 1}, m={m}, "
                                 f"{args.dist} keys, values ~N(0,1), fwd+adjoint, fp32",
                     "n": n, "bins": m, "keys": args.dist, "op": op, "combinator": "reduce_by_index"})


def rbi_sweep(torch, reps=3):
    """Forward and adjoint times of reduce-by-index at n = 2^26 over the bin
    counts {256, 65536, 2^22}, uniform and Zipf(1.1) keys, + * min max.
    Inputs are drawn on the device (torch generator, seeded): timing only."""
    import paper_2310_03568_amd as pcad
    n = 1 << 26
    g = torch.Generator(device="cuda:0").manual_seed(231003568)
    v = torch.randn(n, device="cuda:0", generator=g)
    out = {}
    for m in (256, 65536, 1 << 22):
        cdf = torch.cumsum(torch.arange(1, m + 1, device="cuda:0", dtype=torch.float64) ** -1.1, 0)
        cdf /= cdf[-1].clone()
        for dist in ("uniform", "zipf"):
            if dist == "uniform":
                idx = torch.randint(0, m, (n,), device="cuda:0", generator=g, dtype=torch.int32)
            else:
                u = torch.rand(n, device="cuda:0", generator=g, dtype=torch.float64)
                idx = torch.searchsorted(cdf, u, right=True).clamp_(max=m - 1).to(torch.int32)
            hb = torch.randn(m, device="cuda:0", generator=g)
            for op in ("add", "mul", "min", "max", "sumprod"):
                h, saved = pcad.rbi_fwd(op, idx, v, m)
                vb = pcad.rbi_vjp(op, idx, v, m, saved, hb)
                times = []
                for fn in (lambda: pcad.rbi_fwd(op, idx, v, m),
                           lambda: pcad.rbi_vjp(op, idx, v, m, saved, hb, out=vb)):
                    fn()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):
                        fn()
                    e1.record()
                    torch.cuda.synchronize()
                    times.append(e0.elapsed_time(e1) / reps)
                out[f"{op} m={m} {dist}"] = {"fwd_ms": round(times[0], 4), "vjp_ms": round(times[1], 4),
                                             "fwd_GBs": round(8 * n / times[0] * 1e-6, 1)}
            del idx, hb
    # reduce with the invertible operator sumOfProd (Section 3.3), same n
    y, saved = pcad.reduce_fwd("sumprod", v)
    yb = torch.ones(1, device="cuda:0")
    g = pcad.reduce_vjp("sumprod", v, None, saved, yb)
    times = []
    for fn in (lambda: pcad.reduce_fwd("sumprod", v),
               lambda: pcad.reduce_vjp("sumprod", v, None, saved, yb, out=(g,))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / reps)
    out["reduce sumprod"] = {"fwd_ms": round(times[0], 4), "vjp_ms": round(times[1], 4),
                             "fwd_GBs": round(4 * n / times[0] * 1e-6, 1),
                             "vjp_GBs": round(8 * n / times[1] * 1e-6, 1)}
    return {"rbi_sweep_n2e26": out}


def rbi_parity(b, np):
    """Oracle (fp64, one thread) forward and adjoint on the whole workload:
    its time is the cpu_baseline, its outputs gate the GPU's."""
    import oracle
    from oracle.gate import RTOL, gate
    w = b["inputs"]
    n, op, m = b["n"], b["cfg"]["op"], b["cfg"]["bins"]
    h, vb = (t.cpu().numpy() for t in b["out"]())
    if op != "sumprod":
        t0 = time.perf_counter()
        o = oracle.rbi_fwd(op, w["idx"], m, w["v"])
        xb, cx = oracle.rbi_vjp(op, w["idx"], m, w["hbar"], w["v"])
        dt = time.perf_counter() - t0
    if op == "sumprod":
        t0 = time.perf_counter()
        o = oracle.sumprod_rbi_fwd(w["idx"], m, w["v"])
        xb, cx = oracle.sumprod_rbi_vjp(w["idx"], m, w["hbar"], w["v"])
        dt = time.perf_counter() - t0
        rh = gate(h, o["hist"], o["c"], RTOL[op])
        rv = gate(vb, xb, cx, RTOL[op])
        par = dict(ok=rh["ok"] and rv["ok"], hist_max_rel=rh["max_rel"], vbar_max_rel=rv["max_rel"],
                   range_exceeded=rh["n_range_exceeded"] + rv["n_range_exceeded"])
    elif op in ("min", "max"):
        ok = bool(np.array_equal(h, o["hist"][:, 0].astype(np.float32)))
        ok = ok and bool(np.array_equal(vb, xb[:, 0].astype(np.float32)))
        par = dict(ok=ok, exact=True)
    else:
        rh = gate(h, o["hist"][:, 0], o["c"][:, 0], RTOL[op])
        rv = gate(vb, xb[:, 0], cx[:, 0], RTOL[op])
        par = dict(ok=rh["ok"] and rv["ok"], hist_max_rel=rh["max_rel"], vbar_max_rel=rv["max_rel"],
                   range_exceeded=rh["n_range_exceeded"] + rv["n_range_exceeded"])
    cpu = {"value": n / dt, "unit": "elem/s", "cores": 1, "kind": "oracle",
           "sample": f"whole workload (n={n}, m={m}): oracle forward + adjoint, fp64, {dt:.2f} s"}
    return cpu, par


def bench_vec(args, pcad, torch, np):
    """Vectorised scan (map2 op over vectors of d = 64 floats, n = 2^20 rows,
    2^26 values; N(0,1), or U[0.5, 2) for *): forward and adjoint through
    the transposed scalar form (the ISWIM rule)."""
    n, d = (args.n or (1 << 20)), 64
    op = args.op
    g = np.random.default_rng(231003568 + 7)
    x = g.standard_normal((n, d)).astype(np.float32) if op != "mul" else \
        g.uniform(0.5, 2.0, (n, d)).astype(np.float32)
    yb = g.standard_normal((n, d)).astype(np.float32)
    dev = torch.device("cuda:0")
    X, YB = torch.from_numpy(x).to(dev), torch.from_numpy(yb).to(dev)
    xb = torch.empty_like(X)
    state = {}

    def fwd():
        y, saved = pcad.vscan_fwd(op, X)
        state["y"] = y
        return None, None, saved

    def bwd(saved):
        pcad.vscan_vjp(op, X, saved, YB, out=xb)

    N = n * d
    # the scalar scan's algorithmic bytes; the rule's transposes add
    # 2 x 8 B (forward) and 3 x 8 B (adjoint) per value on top
    per_bwd = 8 if op == "add" else 12
    return dict(n=N, fwd=fwd, bwd=bwd, bytes_fwd=8 * N, bytes_bwd=per_bwd * N,
                kernel="k_scan_vjp_d<vec>", inputs={"x": x, "ybar": yb, "n": n, "d": d},
                out=lambda: (state["y"], xb),
                cfg={"workload": f"vectorised scan ({op} over vectors of {d}), {n} rows, fp32",
                     "rows": n, "d": d, "op": op, "combinator": "scan (map2)"})


def vec_extras(b, torch, np, reps=5):
    """Vectorised reduce and reduce-by-index (1024 bins) on the same values."""
    import paper_2310_03568_amd as pcad
    x = torch.from_numpy(b["inputs"]["x"]).cuda()
    n, d = b["inputs"]["n"], b["inputs"]["d"]
    op = b["cfg"]["op"]
    idx = torch.randint(0, 1024, (n,), device="cuda", dtype=torch.int32,
                        generator=torch.Generator(device="cuda").manual_seed(5))
    hb = torch.randn(1024, d, device="cuda")
    yb = torch.randn(d, device="cuda")
    out = {}
    y, sv = pcad.vreduce_fwd(op, x)
    h, sh = pcad.vrbi_fwd(op, idx, x, 1024)
    gx = torch.empty_like(x)
    for name, fn in (("vreduce_fwd", lambda: pcad.vreduce_fwd(op, x)),
                     ("vreduce_vjp", lambda: pcad.vreduce_vjp(op, x, sv, yb, out=gx)),
                     ("vrbi_fwd", lambda: pcad.vrbi_fwd(op, idx, x, 1024)),
                     ("vrbi_vjp", lambda: pcad.vrbi_vjp(op, idx, x, 1024, sh, hb, out=gx))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_ms"] = e0.elapsed_time(e1) / reps
    return out


def vec_parity(b, np):
    """Oracle (fp64, one thread) on the whole workload: the vectorised scan
    and its adjoint, column by column."""
    import oracle
    from oracle.gate import RTOL, gate
    w = b["inputs"]
    op = b["cfg"]["op"]
    y, xb = (t.cpu().numpy() for t in b["out"]())
    t0 = time.perf_counter()
    Y, CY = oracle.vscan_fwd(op, w["x"])
    XB, CX = oracle.vscan_vjp(op, w["ybar"], w["x"])
    dt = time.perf_counter() - t0
    r1 = gate(y, Y, CY, RTOL[op])
    r2 = gate(xb, XB, CX, RTOL[op])
    par = dict(ok=r1["ok"] and r2["ok"], y_max_rel=r1["max_rel"], xbar_max_rel=r2["max_rel"],
               range_exceeded=r1["n_range_exceeded"] + r2["n_range_exceeded"])
    cpu = {"value": b["n"] / dt, "unit": "elem/s", "cores": 1, "kind": "oracle",
           "sample": f"whole workload ({b['n']} values): oracle scan + adjoint per column, fp64, {dt:.2f} s"}
    return cpu, par


def bench_autograd(args, pcad, torch, np):
    """64 sequences of 2^16: loss = sum log|linrec scan| + sum over non-empty
    bins of max-by-index (65536 bins); a step is the loss forward and its
    backward through the autograd Functions."""
    import paper_2310_03568_amd.autograd as ag
    from workloads import autograd
    w = autograd()
    dev = torch.device("cuda:0")
    a = torch.from_numpy(w["a"]).to(dev).requires_grad_(True)
    bb = torch.from_numpy(w["b"]).to(dev).requires_grad_(True)
    v = torch.from_numpy(w["v"]).to(dev).requires_grad_(True)
    idx = torch.from_numpy(w["idx"]).to(dev)
    B, T, m = a.shape[0], a.shape[1], w["m"]
    state = {}

    def fwd():
        for t in (a, bb, v):
            t.grad = None
        y = ag.scan_linrec(a, bb, mode=args.mode)
        h = ag.reduce_by_index("max", idx, v, m)
        state["loss"] = torch.log(torch.abs(y)).sum() + torch.where(torch.isfinite(h), h, 0).sum()
        return None, None, None

    def bwd(_saved):
        state.pop("loss").backward()

    n = B * T
    return dict(n=n, fwd=fwd, bwd=bwd, inputs=w, autograd=(a, bb, v, idx, m),
                # forward: scan reads a, b, writes y; log|y| and its sum read y;
                # histogram reads v, idx (+ 12 B per bin); backward: scan
                # adjoint reads a, b, y_bar, writes a_bar, b_bar; v_bar one-hot
                bytes_fwd=(12 + 8 + 8) * n, bytes_bwd=(20 + 8) * n,
                kernel="k_scan_vjp_d<LINREC>", out=lambda: (a.grad, bb.grad, v.grad),
                cfg={"workload": f"autograd: {B} sequences x {T}, loss = sum log|linrec scan| + "
                                 f"sum of non-empty max-by-index ({m} bins), fwd+bwd, fp32, "
                                 f"saved state: {args.mode}",
                     "batch": B, "seq_len": T, "bins": m, "mode": args.mode})


def autograd_extras(b, torch, np):
    """Peak device memory of one loss forward + backward in each saved-state
    form (allocations above what is resident before the step)."""
    import paper_2310_03568_amd.autograd as ag
    a, bb, v, idx, m = b["autograd"]
    out = {}
    for mode in ("recompute", "checkpoint"):
        for t in (a, bb, v):
            t.grad = None
        torch.cuda.synchronize()
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        y = ag.scan_linrec(a, bb, mode=mode)
        h = ag.reduce_by_index("max", idx, v, m)
        loss = torch.log(torch.abs(y)).sum() + torch.where(torch.isfinite(h), h, 0).sum()
        del y, h
        loss.backward()
        torch.cuda.synchronize()
        out[f"peak_extra_bytes_{mode}"] = int(torch.cuda.max_memory_allocated() - base)
    return out


def segmented_extras(b, torch, np, reps=3):
    """Single-launch (forward+adjoint) graph time and the per-instance
    plain-call baseline on the same buffers."""
    import paper_2310_03568_amd as pcad
    plan = b["plan"]
    out = {}
    for name, fn in (("both_graph", lambda: plan.run(pcad.PHASE_BOTH)),
                     ("per_segment_fwd", lambda: plan.run_per_segment(pcad.PHASE_FWD)),
                     ("per_segment_bwd", lambda: plan.run_per_segment(pcad.PHASE_BWD))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_ms"] = e0.elapsed_time(e1) / reps
    return out


def segmented_parity(b, torch, np):
    """Oracle (fp64, one thread) on the whole workload: times the adjoint
    (cpu_baseline) and gates the GPU forward and adjoint.  The min-by-index
    decisions are taken on the plan's own float32 y: every bin's argk must
    be the lowest index of that y's minimum in the bin and h must be y at
    argk, bit for bit (Section 4.2, Min/Max); the adjoint runs on the plan's
    own argk and is gated against the oracle's adjoint for those decisions."""
    import oracle
    import paper_2310_03568_amd as pcad
    from oracle.gate import gate, segmented_decisions
    w, plan = b["inputs"], b["plan"]
    N, S, m = plan.n, plan.nseg, plan.m
    plan.run(pcad.PHASE_FWD)
    torch.cuda.synchronize()
    y = plan.y[:N].cpu().numpy()
    h = plan.h.cpu().numpy()
    argk = plan.argk.cpu().numpy().reshape(S, m)
    t0 = time.perf_counter()
    f = oracle.segmented_fwd(w["offsets"], w["a"], w["b"], w["idx"], m)
    tf = time.perf_counter() - t0
    ry = gate(y, f["y"], f["cy"], 1e-4)
    dec = segmented_decisions(w["offsets"], w["idx"], m, y, h, argk, f)
    plan.run(pcad.PHASE_BWD)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ab, bb, cab, cbb = oracle.segmented_vjp(w["offsets"], w["a"], w["b"], w["idx"], m,
                                            w["ybar"], w["hbar"], argk)
    tb = time.perf_counter() - t0
    ra = gate(plan.abar[:N].cpu().numpy(), ab, cab, 1e-4)
    rb = gate(plan.bbar[:N].cpu().numpy(), bb, cbb, 1e-4)
    rx = ry["n_range_exceeded"] + ra["n_range_exceeded"] + rb["n_range_exceeded"]
    ok = (ry["ok"] and ra["ok"] and rb["ok"] and rx == 0
          and dec["argk_ok"] and dec["h_ok"] and dec["diff_ok"])
    par = dict(ok=ok, y_max_rel=ry["max_rel"], a_max_rel=ra["max_rel"], b_max_rel=rb["max_rel"],
               normwise_a=ra["normwise"], normwise_b=rb["normwise"],
               argk_lowest_min_of_own_y=dec["argk_ok"], argk_bad_bins=dec["argk_bad_bins"],
               h_is_y_at_argk=dec["h_ok"], argk_differs_from_fp64_oracle_bins=dec["n_diff_oracle"],
               argk_differences_are_ties=dec["diff_ok"], range_exceeded=rx)
    cpu = {"value": N / tb, "unit": "elem/s", "cores": 1, "kind": "oracle",
           "sample": f"whole workload ({S} instances, {N} elements): oracle adjoint incl. its "
                     f"forward re-execution {tb:.2f} s (forward alone {tf:.2f} s), fp64"}
    return cpu, par


def cpu_baseline_and_parity(name, b, np):
    """Times the oracle (fp64, one thread) on the same inputs and gates the
    GPU outputs against it."""
    import oracle
    from oracle.gate import RTOL, gate
    w = b["inputs"]
    n = b["n"]
    outs = [t.cpu().numpy() for t in b["out"]()]
    if name == "linrec":
        t0 = time.perf_counter()
        yt = np.zeros((n, 2))
        yt[:, 1] = w["ybar"]
        xb, cx = oracle.scan_vjp("linrec", yt, w["a"], w["b"])
        dt = time.perf_counter() - t0
        r1 = gate(outs[0], xb[:, 0], cx[:, 0], RTOL["linrec"])
        r2 = gate(outs[1], xb[:, 1], cx[:, 1], RTOL["linrec"])
        par = dict(ok=r1["ok"] and r2["ok"] and r1["n_range_exceeded"] == 0 and r2["n_range_exceeded"] == 0,
                   max_rel_a=r1["max_rel"], max_rel_b=r2["max_rel"],
                   normwise_a=r1["normwise"], normwise_b=r2["normwise"],
                   range_exceeded=r1["n_range_exceeded"] + r2["n_range_exceeded"])
    else:
        t0 = time.perf_counter()
        xb, cx = oracle.scan_vjp("mat2", w["Pbar"], w["M"])
        dt = time.perf_counter() - t0
        r = gate(outs[0], xb, cx, RTOL["mat2"])
        par = dict(ok=r["ok"], max_rel=r["max_rel"], normwise=r["normwise"],
                   range_exceeded=r["n_range_exceeded"])
    cpu = {"value": n / dt, "unit": "elem/s", "cores": 1, "kind": "oracle",
           "sample": f"whole workload (n={n}): oracle adjoint incl. its forward re-execution, fp64, {dt:.2f} s"}
    return cpu, par


def autograd_parity(b, torch, np):
    """Oracle gradient of every sequence (seeded with the float32 1/y that the
    last step fed the scan adjoint, recomputed here from the GPU's y) against
    the autograd gradients; the oracle's time is the cpu_baseline."""
    import oracle
    import paper_2310_03568_amd.autograd as ag
    from oracle.gate import gate
    w = b["inputs"]
    a, bb, v, idx, m = b["autograd"]
    for t in (a, bb, v):
        t.grad = None
    y = ag.scan_linrec(a, bb, mode="recompute")
    seed = {}
    y.register_hook(lambda g: seed.setdefault("g", g.detach().clone()))
    h = ag.reduce_by_index("max", idx, v, m)
    (torch.log(torch.abs(y)).sum() + torch.where(torch.isfinite(h), h, 0).sum()).backward()
    torch.cuda.synchronize()
    ga, gb, gv = (t.grad.cpu().numpy() for t in (a, bb, v))
    yb = seed["g"].cpu().numpy()
    B = ga.shape[0]
    ok, worst, rx = True, 0.0, 0
    t0 = time.perf_counter()
    for s in range(B):
        ab, bbar, vb, ca, cb, cv = oracle.autograd_grad(w["a"][s], w["b"][s], w["v"][s], w["idx"][s],
                                                        m, ybar=yb[s])
        for g, r, c in ((ga[s], ab, ca), (gb[s], bbar, cb)):
            res = gate(g, r, c, 1e-4)
            ok = ok and res["ok"]
            worst = max(worst, res["max_rel"])
            rx += res["n_range_exceeded"]
        ok = ok and bool(np.array_equal(gv[s], vb.astype(np.float32)))
    dt = time.perf_counter() - t0
    n = b["n"]
    cpu = {"value": n / dt, "unit": "elem/s", "cores": 1, "kind": "oracle",
           "sample": f"whole workload ({B} sequences): oracle forward + gradient, fp64, {dt:.2f} s"}
    return cpu, dict(ok=ok and rx == 0, max_rel=worst, range_exceeded=rx)


def _tune_key(tune, args):
    """The tuning-cache bucket of the workload (None: apply every entry)."""
    n = args.n or None
    if args.workload == "segmented":
        return tune.key("batched", "linrec+min", n or args.segments * 16384, 512, "lognormal")
    if args.workload == "linrec":
        return tune.key("scan", "linrec", n or (1 << 26))
    if args.workload == "mat2":
        return tune.key("scan", "mat2", n or (1 << 24))
    if args.workload == "rbi":
        return tune.key("rbi", args.op, n or (1 << 26), args.bins, args.dist)
    return None


def _knobs_used(pcad, args):
    """The knobs that the timed workload reads, as set for the run."""
    k = pcad.knobs()
    prefix = {"segmented": ("seg.",), "linrec": ("scan.",), "mat2": ("scan.",),
              "rbi": ("rbi.",), "vec": ("scan.", "rbi."), "autograd": ("scan.", "rbi."),
              "matd": ()}[args.workload]
    return {n: v for n, v in sorted(k.items()) if n.startswith(prefix)}


def copy_bandwidth(torch, np, pcad=None, reps=9):
    """HBM rate of a device-to-device copy of 512 MiB into 512 MiB, in GB/s
    of bytes read + written, median of `reps` timed launches: torch's copy
    kernel (plain loads and stores), and with `pcad` also the library's
    streaming copy (nontemporal loads and stores).  Returns (plain,
    streaming or None)."""
    src = torch.empty(1 << 27, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)

    def rate(copy):
        copy()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            copy()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return 2 * (1 << 27) * 4 / float(np.median(ts)) / 1e9

    plain = rate(lambda: dst.copy_(src))
    streaming = rate(lambda: pcad.stream_copy(dst, src)) if pcad is not None else None
    del src, dst
    return plain, streaming


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="segmented",
                    choices=["segmented", "linrec", "mat2", "rbi", "vec", "autograd", "matd"])
    ap.add_argument("--op", default="add", choices=["add", "mul", "min", "max", "sumprod"],
                    help="operator of the rbi workload")
    ap.add_argument("--d", type=int, default=3, choices=[3, 5], help="matrix size of the matd workload")
    ap.add_argument("--bins", type=int, default=65536, help="bins of the rbi workload")
    ap.add_argument("--dist", default="uniform", choices=["uniform", "zipf"],
                    help="key distribution of the rbi workload")
    ap.add_argument("--mode", default="recompute", choices=["recompute", "checkpoint"],
                    help="saved-state form of the autograd workload's scan")
    ap.add_argument("--segments", type=int, default=4096, help="instances of the segmented workload")
    ap.add_argument("--n", type=int, default=0, help="override the element count")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the single-graph and per-instance comparison runs (profiling)")
    ap.add_argument("--knob", action="append", default=[], metavar="NAME=VALUE",
                    help="set a tuning knob before the workload is built (repeatable); "
                         "applied after the tuning cache")
    ap.add_argument("--tune-cache", default=None,
                    help="tuning cache to apply (default: the tuner's default path, if present)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the timed region, run a plain 256 MiB device copy 3 times "
                         "(reference for scaling the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2310_03568_amd as pcad

    pcad.lib()
    from paper_2310_03568_amd import tune
    tuned = tune.load(args.tune_cache or tune.DEFAULT_PATH, key=_tune_key(tune, args))
    for kv in args.knob:
        name, _, val = kv.partition("=")
        pcad.set_knob(name, int(val))
    b = {"linrec": bench_linrec, "mat2": bench_mat2, "segmented": bench_segmented,
         "rbi": bench_rbi, "vec": bench_vec, "autograd": bench_autograd,
         "matd": bench_matd}[args.workload](args, pcad, torch, np)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        _, _, saved = b["fwd"]()
        b["bwd"](saved)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        e0, e1, e2 = ev[k]
        e0.record(stream)
        _, _, saved = b["fwd"]()
        e1.record(stream)
        b["bwd"](saved)
        e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_fwd = np.array([e[0].elapsed_time(e[1]) for e in ev]) * 1e-3
    t_bwd = np.array([e[1].elapsed_time(e[2]) for e in ev]) * 1e-3
    n = b["n"]
    tb = float(t_bwd.mean())
    tf = float(t_fwd.mean())
    achieved = b["bytes_bwd"] / tb / 1e9
    copy_plain_gbs, copy_stream_gbs = copy_bandwidth(torch, np, pcad)
    copy_gbs = max(copy_plain_gbs, copy_stream_gbs or 0.0)

    if args.calib_copy:
        src = torch.empty(1 << 26, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    extras = {}
    if args.workload == "segmented" and not args.no_extras:
        extras = segmented_extras(b, torch, np)
    if args.workload == "autograd" and not args.no_extras:
        extras = autograd_extras(b, torch, np)
    if args.workload == "rbi" and not args.no_extras:
        extras = rbi_sweep(torch)
    if args.workload == "vec" and not args.no_extras:
        extras = vec_extras(b, torch, np)
    if args.workload == "matd" and not args.no_extras:
        extras = matd_extras(b, torch, np)
    cpu, par = (None, None)
    if not args.no_cpu:
        if args.workload == "segmented":
            cpu, par = segmented_parity(b, torch, np)
        elif args.workload == "autograd":
            cpu, par = autograd_parity(b, torch, np)
        elif args.workload == "rbi":
            cpu, par = rbi_parity(b, np)
        elif args.workload == "vec":
            cpu, par = vec_parity(b, np)
        elif args.workload == "matd":
            cpu, par = matd_parity(b, torch, np)
        else:
            cpu, par = cpu_baseline_and_parity(args.workload, b, np)

    wl_key = args.workload
    if args.workload == "rbi":
        wl_key = f"rbi-{args.op}-m{args.bins}-{args.dist}"
    if args.workload == "matd":
        wl_key = f"matd{args.d}-n{n}"
    out = {
        "metric": METRIC,
        "value": n / tb,
        "unit": "elem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {**b["cfg"], "tuning": {"cache_applied": tuned, "knobs": _knobs_used(pcad, args)}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _traffic(b["kernel"], wl_key),
                     "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "copy_plain_GBs": copy_plain_gbs, "copy_stream_GBs": copy_stream_gbs},
        "cpu_baseline": cpu,
        "bwd_ms": tb * 1e3,
        "fwd_ms": tf * 1e3,
        "bwd_over_fwd": tb / tf,
        "fwd_GBs": b["bytes_fwd"] / tf / 1e9,
        "bwd_ci95_ms": 1.96 * float(t_bwd.std(ddof=1)) / np.sqrt(len(t_bwd)) * 1e3 if len(t_bwd) > 1 else 0.0,
        "bwd_median_ms": float(np.median(t_bwd)) * 1e3,
        "fwd_median_ms": float(np.median(t_fwd)) * 1e3,
        "fwd_ci95_ms": 1.96 * float(t_fwd.std(ddof=1)) / np.sqrt(len(t_fwd)) * 1e3 if len(t_fwd) > 1 else 0.0,
        "parity": par,
        **extras,
    }
    if "per_segment_bwd_ms" in extras:
        out["per_segment_bwd_elem_s"] = n / (extras["per_segment_bwd_ms"] * 1e-3)
        out["batched_over_per_segment_bwd"] = extras["per_segment_bwd_ms"] / (tb * 1e3)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
