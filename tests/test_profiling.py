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


def test_stats_selects_the_last_dispatches_of_the_largest_grid(tmp_path):
    # kernel A: 3 small-grid dispatches then 4 large ones (durations 10, 20,
    # 30, 40 us); the last 2 large ones average 35 us
    stats_csv = tmp_path / "s.csv"
    stats_csv.write_text("Name,Calls,AverageNs,MinNs,MaxNs,Percentage\nvoid A(x),7,1000,500,40000,100\n")
    trace_csv = tmp_path / "t.csv"
    rows = ["Kernel_Name,Grid_Size_X,Start_Timestamp,End_Timestamp"]
    t = 0
    for g, us in [(64, 1), (64, 1), (64, 1), (256, 10), (256, 20), (256, 30), (256, 40)]:
        rows.append("void A(x),%d,%d,%d" % (g, t, t + us * 1000))
        t += 100000
    trace_csv.write_text("\n".join(rows) + "\n")
    out = tmp_path / "o.txt"
    profiling.stats(str(stats_csv), str(out), "cmd", str(trace_csv), [("A(", 2, -1, True), ("A(", 3, 0, False)])
    text = out.read_text()
    assert "# dispatches 2..3 (in start order) (grid 256 only) of A(: avg 35.0 us, min 30.0, max 40.0" in text
    assert "# dispatches 0..2 (in start order) of A(: avg 1.0 us" in text
