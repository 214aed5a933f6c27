"""Host logic of bench.py that needs no GPU: the conversion of two rocprofv3
counter runs (FETCH_SIZE, WRITE_SIZE) into HBM bytes per launch."""
import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _write(path, counter, rows):
    # rows: (dispatch, kernel, grid, values per block); each value is one row
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name, grid, vals in rows:
            for v in vals:
                w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                            "Counter_Value": v})


FUSED = "void pat::k_line_nufft2_pipe<float, 12>(pat::StageArgs)"
X2 = "void pat::k_tr_x2_pipe<float, 0>(pat::StageArgs)"


def test_traffic_scales_pairs_and_groups(tmp_path):
    b = _bench()
    copy_kib = 1 << 20  # 1 GiB calibration copy
    fetch = [
        (1, "__amd_rocclr_fillBufferAligned", 1024, [0.0]),
        (2, "__amd_rocclr_copyBuffer", 1024, [copy_kib / 4, copy_kib / 4]),  # reads half: scale 2
        (3, FUSED, 4096, [20000.0, 13000.0]),
        (4, FUSED, 4096, [33000.0]),
        (5, X2, 2048, [66000.0]),   # 512-sample lines
        (6, X2, 2048, [33000.0]),   # 256-sample lines, same persistent grid
    ]
    write = [
        (1, "__amd_rocclr_fillBufferAligned", 1024, [copy_kib / 2, copy_kib / 2]),
        (2, "__amd_rocclr_copyBuffer", 1024, [copy_kib]),
        (3, FUSED, 4096, [66048.0]),
        (4, FUSED, 4096, [66048.0]),
        (5, X2, 2048, [132096.0]),
        (6, X2, 2048, [66048.0]),
    ]
    f, w, o = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    _write(f, "FETCH_SIZE", fetch)
    _write(w, "WRITE_SIZE", write)
    out = b.traffic_from_counters(str(f), str(w), copy_kib * 1024, "wl", "f32", out_path=str(o))
    assert out["fetch_scale"] == pytest.approx(2.0)
    assert out["write_scale"] == pytest.approx(1.0)
    assert out["kernel_source"] == b.kernel_source_hash()
    # block rows of a dispatch are summed, dispatches of one group averaged
    assert out["bytes_per_launch"]["nufft_fused:wl:f32"] == pytest.approx(1024 * (33000 * 2 + 66048))
    x2 = {k: v for k, v in out["bytes_per_launch"].items() if k.startswith("dft_x2:")}
    assert len(x2) == 2   # the two line lengths are told apart despite one grid size
    assert sorted(x2.values()) == pytest.approx(sorted([1024 * (66000 * 2 + 132096), 1024 * (33000 * 2 + 66048)]))
    assert json.load(open(o)) == json.loads(json.dumps(out))


def test_counter_table_per_wave_and_busy(tmp_path):
    """`bench.py --counters-from`: block rows of a dispatch are summed,
    dispatches averaged, instructions divided by waves, VALU busy from the
    traced duration (4 cycles per wave instruction over 1024 SIMDs at
    2.4 GHz), LDS conflicts per active LDS cycle."""
    b = _bench()
    p1, p2, tr = tmp_path / "p1.csv", tmp_path / "p2.csv", tmp_path / "t.csv"
    rows1 = []
    for d in (7, 8):
        rows1 += [(d, FUSED, 4096, [2048.0, 2048.0])]
    _write(p1, "SQ_WAVES", rows1)
    with open(p1, "a", newline="") as fh:
        w = csv.writer(fh)
        for d in (7, 8):
            w.writerow([d, FUSED, 4096, "SQ_INSTS_VALU", 4096 * 1000.0])
            w.writerow([d, FUSED, 4096, "SQ_LDS_BANK_CONFLICT", 300.0])
            w.writerow([d, FUSED, 4096, "SQ_ACTIVE_INST_LDS", 200.0])
    _write(p2, "SQ_INSTS_VALU_FLOPS_FP32", [(7, FUSED, 4096, [1.0]), (8, FUSED, 4096, [1.0])])
    # 100 us per dispatch
    with open(tr, "w", newline="") as fh:
        w = csv.DictWriter(fh, ["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for t0 in (0, 10 ** 6):
            w.writerow({"Kernel_Name": FUSED, "Grid_Size": 4096, "Start_Timestamp": t0,
                        "End_Timestamp": t0 + 100000})
    text = b.counters_summary([str(p1), str(p2)], str(tr), "wl")
    row = [l for l in text.splitlines() if "k_line_nufft2_pipe<float, 12>" in l][0].split("|")
    cells = [c.strip() for c in row[1:-1]]
    assert cells[0] == "nufft_fused" and cells[3] == "2"       # stage, dispatches
    assert cells[4] == "100.0" and cells[5] == "4096"          # avg us, waves
    assert cells[6] == "1000"                                  # VALU per wave
    busy = 4 * 4096 * 1000.0 / (1024 * 2.4e9 * 100e-6)
    assert cells[11] == f"{busy:.2f}"
    assert cells[12] == "1.50"


def test_code_hash_ignores_comments_not_code():
    """The traffic table stays valid across comment edits of the kernels and
    is dropped by any change of their code."""
    b = _bench()
    base = "int f(int x) {  // twice\n  return 2 * x; /* doubled */\n}\n"
    assert b.code_of(base) == b.code_of("int f(int x) {\n  // other words\n  return 2 * x;\n}")
    assert b.code_of(base) != b.code_of("int f(int x) {\n  return 3 * x;\n}")

