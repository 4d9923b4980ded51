"""CPU checks of the tooling around the library: the benchmark's argument
contract, the autotuned table and its loader, the autotuner's search space,
and the traffic figure's staleness check."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_committed_tuning_table_loads():
    from paper_1702_07961_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    with open(_lib.TUNING_PATH) as f:
        table = json.load(f)
    entries = table["entries"]
    pentries = table.get("pairs_entries", [])
    for es in (entries, pentries):
        assert [e["max_log2_n"] for e in es] == sorted(e["max_log2_n"] for e in es)
    lib = _lib.lib()
    assert _lib.load_tuning(lib) == len(entries) + len(pentries)
    t = _lib.MmsTuning()
    for e in entries:
        assert lib.mms_get_tuning(1 << e["max_log2_n"], 0, t) == 0
        assert (t.fanout, t.merge_tile, t.variant, t.base) == (e["fanout"], e["merge_tile"], e["variant"],
                                                               e.get("base", 0))
    for e in pentries:
        assert lib.mms_get_tuning(1 << e["max_log2_n"], _lib.MMS_PAIRS, t) == 0
        assert (t.fanout, t.base, t.flags) == (e["fanout"], e["base"], _lib.MMS_PAIRS)
    # pairs keep the key-value merge tile whatever the table says
    assert lib.mms_get_tuning(1 << 27, _lib.MMS_PAIRS, t) == 0 and t.merge_tile == 3840


def test_autotune_candidates():
    from paper_1702_07961_amd import autotune
    assert list(autotune.candidates(11)) == [(16, 8192, 0)]
    big = set(autotune.candidates(27))
    assert len(big) == len(autotune.FANOUTS) * len(autotune.TILES) * len(autotune.VARIANTS)
    assert {v for _, _, v in big} == {0, 1, 2, 3, 4}
    assert autotune.BASES == [0, 1, 2, 3, 4, 5, 6]
    assert autotune.PAIR_BASES == [0, 3]


def test_traffic_is_null_when_sources_change(monkeypatch, tmp_path):
    import bench
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"source_hash": "0" * 16, "bytes_per_launch": 123}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic() is None
    f.write_text(json.dumps({"source_hash": bench.kernel_source_hash(), "bytes_per_launch": 123}))
    assert bench.measured_traffic() == 123
