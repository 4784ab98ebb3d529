"""Tuning knobs and the tuner's cache on the host (no GPU): validation of
knob values, and that a cache applies only on the device it was measured on,
the built-in defaults staying otherwise."""
from __future__ import annotations

import json

import pytest


@pytest.fixture()
def pcad():
    import paper_2310_03568_amd as p
    p.lib()
    p.reset_knobs()
    yield p
    p.reset_knobs()


def test_knob_validation(pcad):
    k = pcad.knobs()
    assert k["scan.fwd.threads.add"] == 1024 and k["scan.vjp.threads.linrec"] == 512
    assert len(k) == pcad.lib().pcad_knob_count()
    for v in (256, 512, 1024):
        pcad.set_knob("scan.vjp.threads.mat2", v)
        assert pcad.knobs()["scan.vjp.threads.mat2"] == v
    for bad in (0, 128, 300, 2048):
        with pytest.raises(pcad.PcadError):
            pcad.set_knob("scan.vjp.threads.mat2", bad)
    with pytest.raises(pcad.PcadError):
        pcad.set_knob("no.such.knob", 1)
    with pytest.raises(pcad.PcadError):
        pcad.set_knob("rbi.lds_max_bins_u64", 4097)
    pcad.set_knob("rbi.lds_max_bins_u64", 0)  # always global atomics
    assert pcad.lib().pcad_knob_name(-1) is None
    pcad.reset_knobs()
    assert pcad.knobs() == k


def test_cache_applies_on_its_device_only(pcad, tmp_path):
    from paper_2310_03568_amd import tune
    dev = {"name": "AMD Instinct MI355X", "arch": "gfx950:sramecc+:xnack-"}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"version": 2, "device": dev, "entries": [
        {"key": tune.key("scan", "add", 1 << 24), "knobs": {"scan.fwd.threads.add": 256}},
        {"key": tune.key("rbi", "add", 1 << 24, 256, "uniform"), "knobs": {"rbi.elems_per_block": 8192}},
    ]}))
    assert not tune.load(str(path), device={"name": "other", "arch": "gfx942"})
    assert pcad.knobs()["scan.fwd.threads.add"] == 1024
    assert tune.load(str(path), device=dev)
    k = pcad.knobs()
    assert k["scan.fwd.threads.add"] == 256 and k["rbi.elems_per_block"] == 8192
    assert not tune.load(str(tmp_path / "missing.json"), device=dev)
    (tmp_path / "bad.json").write_text("{not json")
    assert not tune.load(str(tmp_path / "bad.json"), device=dev)
    # the first cache format (a flat knob table, no buckets) is not applied
    (tmp_path / "v1.json").write_text(json.dumps({"version": 1, "device": dev,
                                                  "knobs": {"scan.fwd.threads.add": 256}}))
    pcad.reset_knobs()
    assert not tune.load(str(tmp_path / "v1.json"), device=dev)
    assert pcad.knobs()["scan.fwd.threads.add"] == 1024


def test_cache_entry_by_bucket(pcad, tmp_path):
    """With a key, only the entry of that combinator and op (and skew) with
    the nearest n/m buckets is applied."""
    from paper_2310_03568_amd import tune
    dev = {"name": "AMD Instinct MI355X", "arch": "gfx950:sramecc+:xnack-"}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"version": 2, "device": dev, "entries": [
        {"key": tune.key("scan", "linrec", 1 << 20), "knobs": {"scan.vjp.threads.linrec": 256}},
        {"key": tune.key("scan", "linrec", 1 << 26), "knobs": {"scan.vjp.threads.linrec": 1024}},
        {"key": tune.key("batched", "linrec+min", 61_772_580, 512, "lognormal"),
         "knobs": {"seg.tile": 4096, "seg.vjp.threads": 256}},
        {"key": tune.key("rbi", "min", 1 << 24, None, "uniform+zipf"),
         "knobs": {"rbi.lds_max_bins_u64": 1024}},
    ]}))
    assert tune.key("scan", "add", 1 << 24)["n_bucket"] == 24
    assert tune.load(str(path), device=dev, key=tune.key("scan", "linrec", 1 << 25))
    assert pcad.knobs()["scan.vjp.threads.linrec"] == 1024
    assert tune.load(str(path), device=dev, key=tune.key("scan", "linrec", 1 << 21))
    k = pcad.knobs()
    assert k["scan.vjp.threads.linrec"] == 256 and k["seg.tile"] == 8192
    assert tune.load(str(path), device=dev,
                     key=tune.key("batched", "linrec+min", 1 << 26, 512, "lognormal"))
    k = pcad.knobs()
    assert k["seg.tile"] == 4096 and k["seg.vjp.threads"] == 256
    assert k["scan.vjp.threads.linrec"] == 512  # defaults outside the entry
    assert tune.load(str(path), device=dev, key=tune.key("rbi", "min", 1 << 26, 1 << 16, "zipf"))
    assert pcad.knobs()["rbi.lds_max_bins_u64"] == 1024
    assert not tune.load(str(path), device=dev, key=tune.key("rbi", "mul", 1 << 26, 256, "zipf"))
    assert not tune.load(str(path), device=dev, key=tune.key("scan", "mat2", 1 << 24))
