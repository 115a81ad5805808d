"""The committed counter summaries feed the benchmark line only while they
describe the kernel source that runs: a stale summary (source changed since
the counters were taken) yields no traffic and no issue fraction."""
import json

import pytest

from paper_1503_02368_amd import profile_summary as ps


@pytest.fixture
def summaries(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hip"
    src.write_text("__global__ void k() {}\n")
    path = tmp_path / "traffic.json"
    monkeypatch.setattr(ps, "TRAFFIC_FILE", str(path))

    def write(entries):
        path.write_text(json.dumps(entries))

    return str(src), write


def test_current_summary_is_used(summaries):
    src, write = summaries
    # 614.4 M wave-instructions x 4 cycles fill 1024 SIMDs at 2.4 GHz for 1 ms
    write({"w": {"kernel_sha": ps.kernel_sha(src), "bytes_per_launch": 3.5e9,
                 "valu_insts_per_launch": 614.4e6}})
    assert ps.measured_traffic("w", src) == 3.5e9
    got = ps.valu_issue("w", 1.0, src)
    assert got["valu_insts_per_launch"] == 614.4e6
    assert got["valu_issue_frac"] == pytest.approx(1.0)
    assert ps.valu_issue("w", 2.0, src)["valu_issue_frac"] == pytest.approx(0.5)


def test_stale_or_missing_summary_is_not_used(summaries):
    src, write = summaries
    write({"w": {"kernel_sha": "0" * 16, "bytes_per_launch": 3.5e9,
                 "valu_insts_per_launch": 614.4e6},
           "no_valu": {"kernel_sha": ps.kernel_sha(src), "bytes_per_launch": 1.0}})
    assert ps.measured_traffic("w", src) is None
    assert ps.valu_issue("w", 1.0, src) == {"valu_insts_per_launch": None, "valu_issue_frac": None}
    assert ps.measured_traffic("absent", src) is None
    assert ps.valu_issue("no_valu", 1.0, src)["valu_issue_frac"] is None
    assert ps.measured_traffic("no_valu", src) == 1.0
