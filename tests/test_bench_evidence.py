"""Host logic behind bench.py's evidence (no GPU): the kernel-source hash that
ties the committed HBM counter summary to the sources, the summaries made
from rocprofv3 counter CSVs, and the traffic figure a bench line carries."""
import csv
import json
import os
import shutil

import pytest

import bench

SOURCES = ("kernels.hip", "wave.h", "ltrk_device.h", "sinpi_coeffs.h", "sinpi32_coeffs.h")


@pytest.fixture
def tree(tmp_path, monkeypatch):
    """A copy of the hashed sources and of profiles/ under a temporary root."""
    src = os.path.join(bench.ROOT, "paper_1610_05801_amd", "csrc")
    dst = tmp_path / "paper_1610_05801_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in SOURCES:
        shutil.copy(os.path.join(src, f), dst / f)
    shutil.copytree(os.path.join(bench.ROOT, "profiles"), tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def test_committed_traffic_summary_matches_the_sources():
    with open(os.path.join(bench.ROOT, "profiles", "fused_leapfrog_f64_1e6_traffic.json")) as f:
        d = json.load(f)
    assert d["kernel_hash"] == bench.kernel_source_hash()
    per = d["hbm_bytes_per_particle_turn"]
    assert bench.load_traffic("fused_leapfrog_f64_1e6_traffic.json", 1e9) == pytest.approx(per * 1e9)
    # the state once per 1024 turns (32 B / 1024) plus 40 B of partials per wave tile and turn
    assert 32 / 1024 < per < 0.2


def test_hash_ignores_comments_and_blank_space(tree):
    h0 = bench.kernel_source_hash()
    p = tree / "paper_1610_05801_amd" / "csrc" / "kernels.hip"
    text = p.read_text()
    p.write_text("// a new comment line\n/* and a block\n   comment */\n\n" +
                 text.replace("\n", "\n\n", 3))
    assert bench.kernel_source_hash() == h0


def test_hash_follows_code_and_drops_the_traffic(tree):
    h0 = bench.kernel_source_hash()
    assert bench.load_traffic("fused_leapfrog_f64_1e6_traffic.json", 1.0) is not None
    p = tree / "paper_1610_05801_amd" / "csrc" / "sinpi32_coeffs.h"
    p.write_text(p.read_text().replace("0x1.956f8c", "0x1.956f8d"))
    assert bench.kernel_source_hash() != h0
    assert bench.load_traffic("fused_leapfrog_f64_1e6_traffic.json", 1.0) is None
    assert bench.load_traffic("no_such_summary.json", 1.0) is None


FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value",
          "Start_Timestamp", "End_Timestamp"]


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summarize_counters_scales_by_the_calibration_kernel(tree, tmp_path):
    """FETCH_SIZE / WRITE_SIZE (KiB) of the fused launches (4) and the unfused
    ones (5) are scaled by what the copy kernel of known size reads: here the
    copy reads twice its bytes and writes them once, so fetches halve."""
    cal_kib = bench.COUNTER_CAL_BYTES / 1024.0

    def rows(counter, cal, fused, unfused):
        out, i = [], 0
        for name, vals in (("vectorized_elementwise_kernel<MulFunctor>", [cal] * 3),
                           ("ltrk::k_track_single<1, 0, 8>", fused),
                           ("ltrk::k_track_single<1, 0, 2>", unfused)):
            for v in vals:
                i += 1
                out.append({"Dispatch_Id": i, "Kernel_Name": name, "Grid_Size": 256,
                            "Counter_Name": counter, "Counter_Value": v,
                            "Start_Timestamp": 0, "End_Timestamp": 1000})
        return out

    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(fetch, rows("FETCH_SIZE", 2 * cal_kib, [4000.0] * 4, [3.2e6] * 5))
    write_csv(write, rows("WRITE_SIZE", cal_kib, [100000.0] * 4, [1.6e6] * 5))
    out = tmp_path / "t.json"
    bench.summarize_counters(str(fetch), str(write), str(out), 1024)
    d = json.load(open(out))
    assert d["kernel_hash"] == bench.kernel_source_hash()
    assert d["calibration"]["fetch_scale"] == pytest.approx(0.5)
    assert d["calibration"]["write_scale"] == pytest.approx(1.0)
    assert d["fused_leapfrog_1e6"]["fetch_bytes"] == pytest.approx(2000.0 * 1024)
    assert d["fused_leapfrog_1e6"]["write_bytes"] == pytest.approx(100000.0 * 1024)
    assert d["hbm_bytes_per_particle_turn"] == pytest.approx(102000.0 * 1024 / 1.024e9)
    assert d["unfused_hbm_bytes_per_particle_turn"] == pytest.approx(3.2e6 * 1024 / 1e8)


def test_summarize_valu_f32c_per_particle_turn(tmp_path):
    """Wave-level counts x 64 lanes / particle-turns; flops with FMA = 2;
    issue utilisation against 256 CUs at 4 cycles per wave instruction."""
    pt = 1e6 * 1024
    per = {"SQ_INSTS_VALU": 47.0, "SQ_INSTS_VALU_FMA_F32": 7.0, "SQ_INSTS_VALU_ADD_F32": 14.0,
           "SQ_INSTS_VALU_MUL_F32": 5.0, "SQ_INSTS_VALU_FMA_F64": 4.5,
           "SQ_INSTS_VALU_ADD_F64": 6.5, "SQ_INSTS_VALU_MUL_F64": 0.5}
    ns = 1_250_000
    cycles = 2.0e9 * ns * 1e-9            # 2 GHz
    rows = [{"Dispatch_Id": 1, "Kernel_Name": "ltrk::k_track_single<1, 1, 8>", "Grid_Size": 125184,
             "Counter_Name": k, "Counter_Value": v * pt / 64, "Start_Timestamp": 0,
             "End_Timestamp": ns} for k, v in per.items()]
    rows.append({"Dispatch_Id": 1, "Kernel_Name": "ltrk::k_track_single<1, 1, 8>",
                 "Grid_Size": 125184, "Counter_Name": "GRBM_GUI_ACTIVE",
                 "Counter_Value": cycles * 8, "Start_Timestamp": 0, "End_Timestamp": ns})
    src, out = tmp_path / "v.csv", tmp_path / "v.md"
    write_csv(src, rows)
    bench.summarize_valu_f32c(str(src), str(out), 1024)
    line = out.read_text().strip().split("\n")[-1]
    cells = [c.strip() for c in line.strip("|").split("|")]
    assert cells[0] == "0" and float(cells[1]) == pytest.approx(1250.0)
    assert float(cells[2]) == pytest.approx(47.0)
    assert cells[3] == "7.00 / 14.00 / 5.00" and cells[4] == "4.50 / 6.50 / 0.50"
    assert float(cells[5]) == pytest.approx((2 * 7 + 14 + 5) * pt / 1.25e-3 / 1e12, rel=1e-3)
    assert float(cells[6]) == pytest.approx((2 * 4.5 + 6.5 + 0.5) * pt / 1.25e-3 / 1e12, rel=1e-3)
    assert float(cells[7]) == pytest.approx(2.0)
    assert float(cells[8]) == pytest.approx(47.0 * pt / 64 / (256 * cycles), rel=1e-2)
