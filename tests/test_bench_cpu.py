"""Host-side checks of bench.py's measurement bookkeeping (no GPU): the byte
models and the lookup of committed HBM counters."""
import hashlib
import json
import os

import pytest

import bench


def test_check_share_enters_the_byte_models():
    """A check sweep adds per-node bytes (previous mean, and S once settled);
    with one check in c sweeps the model charges 1/c of them per sweep."""
    n, E = 1000, 8000
    assert bench.pair_bytes_per_sweep(n, E, 2) - bench.pair_bytes_per_sweep(n, E, 4) == pytest.approx(
        8.0 * n * (1 / 2 - 1 / 4))
    assert bench.grid_bytes_per_sweep(n, E, True, False, 8) == pytest.approx(12.0 * E + 4.0 * n + 1.5 * n)
    assert bench.grid_bytes_per_sweep(n, E, False, True, 2) == pytest.approx(24.0 * E + 4.0 * n + 4.0 * n)


def _traffic(tmp_path, entries, src_text=b"kernel source"):
    root = tmp_path
    (root / "profiles").mkdir()
    (root / "paper_0810_1119_amd" / "csrc").mkdir(parents=True)
    (root / "paper_0810_1119_amd" / "csrc" / "k.hip").write_bytes(src_text)
    sha = hashlib.sha256(b"kernel source").hexdigest()
    kernels = {name: {"workload": "w", "bytes_per_launch": v, "source": "k.hip", "source_sha256": sha}
               for name, v in entries.items()}
    (root / "profiles" / "traffic.json").write_text(json.dumps({"kernels": kernels}))
    return str(root)


def test_measured_traffic_weights_plain_and_check_launches(tmp_path, monkeypatch):
    """Only the named instantiation counts: records of the same kernel with
    other template arguments (other modes, the coarse levels' variants) are
    not mixed in."""
    root = _traffic(tmp_path, {"gabp::k<float, 0, false>": 100.0, "gabp::k<float, 1, false>": 200.0,
                               "gabp::k<float, 2, false>": 7.0, "gabp::k<float, 0, true>": 9.0})
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.measured_traffic("gabp::k<float, {m}, false>", "w", 0.25) == pytest.approx(125.0)
    assert bench.measured_traffic("gabp::k<float, {m}, false>", "w") == pytest.approx(150.0)
    assert bench.measured_traffic("gabp::k<float, {m}, true>", "w") == pytest.approx(9.0)
    assert bench.measured_traffic("gabp::k<float, 2, false>", "w") == pytest.approx(7.0)
    assert bench.measured_traffic("gabp::k<float, {m}, false>", "other") is None


def test_measured_traffic_is_dropped_when_the_source_changed(tmp_path, monkeypatch):
    root = _traffic(tmp_path, {"gabp::k<float, 0, false>": 100.0}, src_text=b"edited source")
    monkeypatch.setattr(bench, "ROOT", root)
    assert bench.measured_traffic("gabp::k<float, {m}, false>", "w", 0.5) is None


def test_grid_traffic_keys_name_the_template_arguments():
    assert bench.grid_tkey("k_rb_sweep", False, True, True) == \
        "gabp::k_rb_sweep<float, {m}, false, true, true>"
    assert bench.grid_tkey("k_rb_frozen", False, True, True) == "gabp::k_rb_frozen<float, {m}, false, true>"
    assert bench.grid_tkey("k_grid_sweep", True, False, False) == \
        "gabp::k_grid_sweep<float, {m}, true, false>"
    assert bench.grid_tkey("k_grid_frozen", True, False, False) == \
        "gabp::k_grid_frozen<float, {m}, true, false>"


def test_committed_traffic_matches_the_sources():
    """Every committed counter record names a kernel source that exists."""
    path = os.path.join(bench.ROOT, "profiles", "traffic.json")
    t = json.load(open(path))
    for name, rec in t["kernels"].items():
        src = os.path.join(bench.ROOT, "paper_0810_1119_amd", "csrc", rec["source"])
        assert os.path.exists(src), name
        assert rec["bytes_per_launch"] > 0


def test_headline_bytes_follow_the_measurement_unit():
    """The C4 full sweep is priced at 18 B per directed edge + 8 B per node:
    about 1.92 GB per sweep of the 64 grids of 64^3 (99,090,432 directed
    edges, 16,777,216 nodes)."""
    n, count = 64, 64
    E = 2 * 3 * (n - 1) * n * n * count
    N = n ** 3 * count
    assert E == 99_090_432
    assert bench.c4_full_bytes_per_sweep(N, E) == pytest.approx(1.9179e9, rel=1e-4)
