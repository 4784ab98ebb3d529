"""Every value of every tuning knob gives oracle-exact results (each scan
block size is its own kernel instantiation), and the quick tuner run
produces a cache of valid knob values."""
from __future__ import annotations

import json

import numpy as np
import pytest
import torch

import oracle
from oracle.gate import RTOL, assert_gate

pytestmark = pytest.mark.gpu


@pytest.fixture()
def pcad():
    import paper_2310_03568_amd as p
    p.lib()
    p.reset_knobs()
    yield p
    p.reset_knobs()


@pytest.mark.parametrize("threads", [256, 512, 1024])
@pytest.mark.parametrize("op", ["add", "mul", "min", "max", "linrec", "mat2"])
def test_scan_block_sizes(pcad, op, threads):
    from test_gpu_parity import check_scan
    pcad.set_knob(f"scan.fwd.threads.{op}", threads)
    pcad.set_knob(f"scan.vjp.threads.{op}", threads)
    print(f"scan {op} threads {threads}", flush=True)
    check_scan(pcad, op, 1, 30_011, seed=threads + len(op))
    check_scan(pcad, op, 2, 9_000, seed=threads + 7, ckpt=op != "add")


@pytest.mark.parametrize("strategy", ["lds", "global", "parts", "parts4", "partition", "hash_large",
                                      "sorted"])
@pytest.mark.parametrize("op", ["add", "mul", "min", "max"])
def test_rbi_strategies(pcad, op, strategy):
    """lds: private LDS histograms; global: the hash path forced at a small
    bin count; parts / parts4: beyond the LDS capacity, bins split into one
    to four 128 KB LDS tables (default up to four tables; * takes the
    partition there); partition /
    hash_large / sorted: the partition by bin range, the hash table, or the
    sort by bin with a segmented scan"""
    m = 300
    if strategy == "global":
        pcad.set_knob("rbi.lds_max_bins_f32", 0)
        pcad.set_knob("rbi.lds_max_bins_u64", 0)
    if strategy in ("parts", "partition", "hash_large", "sorted"):
        m = 20_011
    if strategy == "parts4":
        m = 131_072 if op == "add" else 65_536
    if strategy in ("partition", "hash_large", "sorted"):
        pcad.set_knob("rbi.parts", 0)
    if strategy == "hash_large":
        pcad.set_knob("rbi.partition", 0)
    if strategy == "sorted":
        pcad.set_knob("rbi.sort_min_bins", 0)
    pcad.set_knob("rbi.elems_per_block", 4096)
    print(f"rbi {op} {strategy} m={m}", flush=True)
    rng = np.random.default_rng(5)
    n = 70_001
    v = rng.uniform(0.5, 2.0, n).astype(np.float32)
    if op in ("min", "max"):
        v = np.floor(v * 8) / 8
    if op == "mul":
        v[rng.choice(n, 70, replace=False)] = 0.0
    idx = rng.integers(-2, m + 2, n).astype(np.int32)
    h, saved = pcad.rbi_fwd(op, torch.from_numpy(idx).cuda(), torch.from_numpy(v).cuda(), m)
    torch.cuda.synchronize()
    r = oracle.rbi_fwd(op, idx, m, v)
    if op in ("min", "max"):
        np.testing.assert_array_equal(h.cpu().numpy(), r["hist"][:, 0].astype(np.float32))
        np.testing.assert_array_equal(pcad.saved_argk(saved, 1, m).cpu().numpy()[0], r["argk"])
    else:
        assert_gate(h.cpu().numpy(), r["hist"][:, 0], r["c"][:, 0], RTOL[op],
                    max_range_exceeded=m if op == "mul" else 0, what=f"rbi {op} {strategy}")


def test_quick_tune_writes_valid_cache(pcad, tmp_path):
    from paper_2310_03568_amd import tune
    out = tmp_path / "tune.json"
    cache = tune.tune(str(out), quick=True)
    assert json.loads(out.read_text())["entries"] == cache["entries"]
    assert tune.load(str(out))
    k = pcad.knobs()
    for name, v in cache["knobs"].items():
        assert k[name] == v
    seg = tune.key("batched", "linrec+min", 1 << 26, 512, "lognormal")
    assert tune.load(str(out), key=seg)
    for name in ("seg.tile", "seg.fwd.threads", "seg.vjp.threads"):
        assert pcad.knobs()[name] == cache["knobs"][name]
    print(json.dumps(cache["knobs"]), flush=True)


@pytest.mark.parametrize("threads", [256, 512, 1024])
@pytest.mark.parametrize("tile", [4096, 8192])
def test_segmented_plan_shapes(pcad, tile, threads):
    """Every item size and block size of the batched plan (each its own
    kernel instantiation, chosen when the plan is created) against the
    oracle, forward and adjoint, on ragged instances."""
    from test_gpu_batched import check_backward, check_forward, ragged_lengths, workload
    pcad.set_knob("seg.tile", tile)
    pcad.set_knob("seg.fwd.threads", threads)
    pcad.set_knob("seg.vjp.threads", 1024 if threads == 256 else threads // 2)
    print(f"segmented tile {tile} threads {threads}", flush=True)
    w = workload(ragged_lengths(3), 512, seed=tile + threads)
    plan = pcad.BatchedPlan(w["offsets"], 512)
    plan.load(a=w["a"], b=w["b"], idx=w["idx"], ybar=w["ybar"], hbar=w["hbar"])
    N = plan.n
    plan.run(pcad.PHASE_BOTH)
    torch.cuda.synchronize()
    check_forward(pcad, w, plan.y[:N].cpu().numpy(), plan.h.cpu().numpy(),
                  plan.argk.cpu().numpy(), f"tile {tile} threads {threads}")
    check_backward(w, plan.argk.cpu().numpy(), plan.abar[:N].cpu().numpy(),
                   plan.bbar[:N].cpu().numpy(), f"tile {tile} threads {threads}")
    assert plan.ws_error() == 0
    plan.close()
