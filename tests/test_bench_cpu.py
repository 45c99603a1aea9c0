"""Host logic of bench.py (no GPU): the counter-traffic lookup honours the
workload, the kernel class and the source hash recorded with the counters,
and the launch-tuner report is parsed into the bench line's `tune` object."""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench   # noqa: E402


def _profile(tmp, name, cls, workload, src, digest, traffic):
    (tmp / "profiles").mkdir(exist_ok=True)
    (tmp / "profiles" / name).write_text(
        "# title\n\n| a | b |\n|---|---|\n\nkernel_class: %s\nworkload: %s\n"
        "traffic_bytes_per_launch: %s\nsource: %s sha256 %s\n" % (cls, workload, traffic, src, digest))


def test_counter_traffic_lookup(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel source\n")
    digest = hashlib.sha256(src.read_bytes()).hexdigest()
    _profile(tmp_path, "x_traffic.md", "gs_update", "C4", "k.hip", digest, "1.2345e+10")
    _profile(tmp_path, "y_traffic.md", "dslash", "C4", "k.hip", "0" * 64, "9.9e+09")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("gs_update", "C4") == 1.2345e10
    assert bench.counter_traffic("gs_update", "C5") is None     # other workload
    assert bench.counter_traffic("combine", "C4") is None       # no summary for the class
    assert bench.counter_traffic("dslash", "C4") is None        # source changed since
    src.write_text("kernel source, edited\n")
    assert bench.counter_traffic("gs_update", "C4") is None


def test_tune_shapes_parsing():
    class FakeGdr:
        @staticmethod
        def gdr_tune_report():
            return ("dslash_r12|gfx950|24x24x24x48|12|0 -> 1 (594 us per unit)\n"
                    "blk_update|gfx950|7962624|1|4|2 -> 3 (0.343 us per unit)\n"
                    "malformed line\n")
    t = bench.tune_shapes(FakeGdr)
    assert t["chosen"] == {"dslash_r12|gfx950|24x24x24x48|12|0": {"form": 1, "us_per_unit": 594.0},
                           "blk_update|gfx950|7962624|1|4|2": {"form": 3, "us_per_unit": 0.343}}
    assert set(t["forms"]) >= {"dslash_r12", "vrecombine_mfma", "blk_update", "vcombine"}

    class Empty:
        @staticmethod
        def gdr_tune_report():
            return ""
    assert bench.tune_shapes(Empty) is None
