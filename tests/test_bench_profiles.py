"""bench.py takes the HBM traffic of its roofline objects from the committed
rocprofv3 summaries, and only while a summary describes the kernel source as
committed: a kernel edited after its counters were taken makes the bench report
the traffic as unknown (null), and this test then names the summary to refresh
(skipped, not failed).  CPU only."""
import glob
import hashlib
import os
import re

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _blocks():
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        text = open(path).read()
        if "source_sha256_16:" not in text:
            continue
        fields = dict(re.findall(r"^\s*(kernel|workload|traffic_bytes_per_launch|source|"
                                 r"source_sha256_16):\s*(.+?)\s*$", text, re.M))
        out.append((os.path.basename(path), fields))
    return out


BLOCKS = _blocks()


def test_machine_readable_summaries_exist():
    names = {n for n, _ in BLOCKS}
    # the headline scan and both walks feed bench.py's roofline objects
    assert {"scan16_pass_bf16_N2e27_m65536.md", "ann_walk_N1e9_m32768.md",
            "kmeans_walk_N1e9_m32768.md"} <= names


@pytest.mark.parametrize("name,fields", BLOCKS, ids=[n for n, _ in BLOCKS])
def test_summary_matches_committed_source(name, fields):
    for k in ("kernel", "workload", "traffic_bytes_per_launch", "source", "source_sha256_16"):
        assert k in fields, f"{name}: no '{k}' line"
    src = os.path.join(ROOT, fields["source"])
    assert os.path.exists(src), f"{name}: {fields['source']} does not exist"
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    traffic = float(fields["traffic_bytes_per_launch"])
    assert 1e8 < traffic < 1e13
    if digest != fields["source_sha256_16"]:
        # the kernel changed after its counters were taken: the bench must not use them
        assert bench.profile_traffic(name, fields["workload"]) is None
        pytest.skip(f"{name} was measured on another version of {fields['source']} "
                    f"({fields['source_sha256_16']}, now {digest}): profile it again")
    assert bench.profile_traffic(name, fields["workload"]) == traffic


def test_stale_or_foreign_summary_gives_no_traffic():
    name, fields = next((n, f) for n, f in BLOCKS if n == "ann_walk_N1e9_m32768.md")
    assert bench.profile_traffic(name, fields["workload"] + " other") is None
    assert bench.profile_traffic("no_such_summary.md", fields["workload"]) is None
    assert bench.measured_traffic("fp16", 2048, 1 << 27, 65536) is None
    scan = dict(BLOCKS)["scan16_pass_bf16_N2e27_m65536.md"]
    assert bench.measured_traffic("bf16", 2048, 1 << 27, 65536) == bench.profile_traffic(
        "scan16_pass_bf16_N2e27_m65536.md", scan["workload"])
    assert bench.measured_traffic("bf16", 1024, 1 << 27, 65536) is None
