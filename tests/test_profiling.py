"""Host-side checks of the measurement helpers (no GPU): the aggregation
source hash that ties a stored traffic record to the code it measured."""
import json
import os

from paper_1807_06271_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_code_only_ignores_comments_and_spacing():
    a = b"int f(int x) {  // the argument\n  return x + 1; /* one more */\n}\n"
    b = b"int f(int x) {\n\n    return x + 1;\n}"
    assert profiling._code_only(a) == profiling._code_only(b)
    c = b"int f(int x) { return x + 2; }"
    assert profiling._code_only(a) != profiling._code_only(c)


def test_source_hash_shape():
    h = profiling.source_hash()
    assert len(h) == 16 and int(h, 16) >= 0


def test_traffic_records_name_their_sources():
    names = [n for n in os.listdir(os.path.join(ROOT, "profiles")) if n.startswith("traffic_")]
    assert "traffic_agg_1920x1080_d256_batch8.json" in names
    for name in names:
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
        assert len(rec["source_hash"]) == 16
        assert rec["calibration"]["bytes"] > 0
        assert rec["calibration"]["fetch_factor"] > 0 and rec["calibration"]["write_factor"] > 0
        assert rec["fetch_command"].startswith("rocprofv3 --pmc FETCH_SIZE")
        assert rec["write_command"].startswith("rocprofv3 --pmc WRITE_SIZE")
