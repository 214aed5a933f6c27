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
