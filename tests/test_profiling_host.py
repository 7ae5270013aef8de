"""Host-side summaries of rocprofv3 output (paper_1501_02946_amd.profiling) and
the benchmark's keys for measured traffic: parsed from small CSV files written
here in rocprofv3's column layout."""
import importlib.util
import os

from paper_1501_02946_amd import profiling as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_short_and_base_names():
    n = "void nedner::k_spread<12, 4, float, float, float, true, true>(nedner::KP, int const*, float*)"
    assert P.short_name(n) == "k_spread<12, 4, float, float, float, true, true>"
    assert P.base_name(n) == "k_spread"
    assert P.base_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_kernel_stats_table(tmp_path):
    f = tmp_path / "x_kernel_stats.csv"
    f.write_text('"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"\n'
                 '"void nedner::k_lat_a<float, true>(nedner::KP)",4,4000,1000,20.0,900,1100,50\n'
                 '"void nedner::k_spread<12, 4>(nedner::KP)",4,16000,4000,80.0,3900,4100,80\n')
    rows = P.kernel_stats(str(f))
    assert [r["name"] for r in rows] == ["k_spread<12, 4>", "k_lat_a<float, true>"]
    assert rows[0]["avg_us"] == 4.0 and rows[0]["calls"] == 4
    md = P.stats_markdown(rows)
    assert "| `k_spread<12, 4>` | 4 | 4.0 | 3.9 | 4.1 | 80.0 |" in md


def test_counter_means_sum_instances_then_average(tmp_path):
    f = tmp_path / "x_counter_collection.csv"
    rows = ["Correlation_Id,Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value"]
    # two dispatches, each with two hardware-instance rows of one counter
    for d, vals in ((1, (10, 20)), (2, (30, 40))):
        for v in vals:
            rows.append(f'{d},{d},"void nedner::k_column<float>(nedner::KP)",SQ_WAVES,{v}')
    rows.append('3,3,"__amd_rocclr_copyBuffer",SQ_WAVES,7')
    f.write_text("\n".join(rows) + "\n")
    m = P.counter_means(str(f))
    assert m["k_column"]["SQ_WAVES"] == (50.0, 2)
    assert m["__amd_rocclr_copyBuffer"]["SQ_WAVES"] == (7.0, 1)
    assert "| `k_column` | 2 | 50 |" in P.counters_markdown(m)


def test_traffic_key_uses_only_the_stage_shape():
    b = _bench()
    t = dict(rows_per_wave=96, time_per_lane=4, spread_depth=1, pass_lines=8, pass_threads=512,
             pass_inplace=1)
    assert b.traffic_key("c3", "fp32c", "spread", t) == \
        "c3:fp32c:spread:rows_per_wave=96,time_per_lane=4,spread_depth=1"
    t2 = dict(t, pass_lines=32)
    assert b.traffic_key("c3", "fp32c", "spread", t2) == b.traffic_key("c3", "fp32c", "spread", t)
    assert b.traffic_key("c3", "fp32c", "lat_a", t2) != b.traffic_key("c3", "fp32c", "lat_a", t)
    assert b.traffic_key("c3", "fp32c", "column", t) == "c3:fp32c:column"
