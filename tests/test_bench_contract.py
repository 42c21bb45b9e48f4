"""bench.py's command-line contract, on the CPU: more than one GPU is refused with a
message (the moments of one volume need no collective; the bench measures one GPU), and the
traffic counters are tied to the projection kernel's own sources."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_traffic_hash_covers_the_projection_sources():
    csrc = os.path.join(ROOT, "paper_2012_08099_amd", "csrc")
    for f in bench.PROJECTION_SOURCES:
        assert os.path.exists(os.path.join(csrc, f)), f
    h = bench.source_hash()
    assert len(h) == 16 and h == bench.source_hash()


def test_stored_traffic_is_used_only_for_its_sources(tmp_path, monkeypatch):
    import json
    p = os.path.join(ROOT, "profiles", "traffic_ct512_k6.json")
    t = json.load(open(p))
    assert bench.read_traffic("ct512_k6", t["source_hash"]) == t["bytes_per_launch"]
    assert bench.read_traffic("ct512_k6", "0" * 16) is None
    assert bench.read_traffic("no_such_workload", t["source_hash"]) is None
