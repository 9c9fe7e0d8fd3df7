"""Host-side summaries of profiler output (no GPU): the per-kernel traffic
table averages each kernel's counter over its dispatches (summing the
per-dispatch rows first) and scales by the copy-probe factors; the traffic
record of one template variant counts that variant only."""
import csv
import json

from paper_2311_04648_amd import profsum


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def _rows(spec):
    out = []
    for d, name, parts in spec:
        for v in parts:   # one row per counter instance of a dispatch
            out.append({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": "X", "Counter_Value": v})
    return out


A = "void (anonymous namespace)::k_step_fused<true, false>(int)"
B = "void (anonymous namespace)::k_step_fused<false, false>(int)"
C = "void k_b(float*)"


def test_kernels_table_averages_and_scales(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(f, _rows([(1, A, [100, 300]), (2, A, [200, 200]), (3, C, [50])]))
    _write(w, _rows([(1, A, [10]), (2, A, [30]), (3, C, [0])]))
    t = profsum.kernels_traffic(str(f), str(w), 2.0, 1.0)
    line = next(l for l in t.splitlines() if l.startswith("| k_step_fused<true, false>"))
    cells = [c.strip() for c in line.strip("|").split("|")]
    # fetch: dispatch sums 400 and 400 KiB, mean 400 KiB, x2 -> 0.8192 MB;
    # write: mean 20 KiB -> 0.02048 MB
    assert cells[1] == "2"
    assert cells[2] == f"{400 * 1024 * 2.0 / 1e6:.2f}"
    assert cells[3] == f"{20 * 1024 / 1e6:.2f}"


def test_traffic_record_counts_one_variant(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    cf, cw = tmp_path / "cf.csv", tmp_path / "cw.csv"
    _write(f, _rows([(1, A, [100]), (2, B, [900])]))
    _write(w, _rows([(1, A, [40]), (2, B, [400])]))
    copy = 1 << 20
    _write(cf, _rows([(9, C, [copy / 1024 / 2])]))   # a copy that reads half its bytes by this counter
    _write(cw, _rows([(9, C, [copy / 1024])]))
    rec = profsum.traffic(str(f), str(w), str(cf), str(cw), copy, "k_step_fused", "dem_dyn.hip", "test",
                          "k_step_fused<true, false>")
    k = rec["k_step_fused"]
    assert rec["copy_probe"]["fetch_scale"] == 2.0 and rec["copy_probe"]["write_scale"] == 1.0
    assert k["variant"] == "k_step_fused<true, false>"
    assert k["FETCH_SIZE_KiB"] == 100 and k["WRITE_SIZE_KiB"] == 40
    assert k["bytes_per_launch"] == 100 * 1024 * 2.0 + 40 * 1024
    # the record is tied to the kernel's current source text
    import bench
    import os
    src = os.path.join(os.path.dirname(profsum.__file__), "csrc", "dem_dyn.hip")
    assert k["kernel_sha"] == bench.kernel_sha(src, "k_step_fused")
    json.dumps(rec)
