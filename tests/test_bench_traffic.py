"""bench.py's HBM-traffic summary from rocprofv3 counter CSVs: the first
copy the program dispatches (the 256 MiB calibration copy) sets the
counter scale, later and larger copies do not, and the selected kernel's
dispatches are averaged."""
import csv
import os

import bench

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for d, name, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_summarize_traffic_calibrates_on_first_copy(tmp_path):
    kib = bench.COPY_BYTES / 1024.0
    kern = "void hicu::conv_kernel<1, 4, 4, 2, 2, 1, false, 2>(hicu::ConvArgs, long, int, int)"
    fetch = [
        (1, "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float> >", 17.5),
        (2, "__amd_rocclr_copyBuffer", kib / 2),          # calibration copy: counter reads half the bytes
        (3, kern, 1000.0),
        (4, kern, 3000.0),
        (5, "void hicu::conv_kernel<1, 8, 2, 1, 2, 2, false, 1>(hicu::ConvArgs, long, int, int)", 9e9),
        (6, "__amd_rocclr_copyBuffer", kib * 10),         # a later, larger copy must not calibrate
    ]
    write = [(d, n, v * (2 if "copyBuffer" in n and d == 2 else 1)) for d, n, v in fetch]
    fp, wp = os.path.join(tmp_path, "f.csv"), os.path.join(tmp_path, "w.csv")
    _write(fp, "FETCH_SIZE", fetch)
    _write(wp, "WRITE_SIZE", write)
    vals = bench.summarize_traffic([fp, wp], "void hicu::conv_kernel<1, 4, 4, 2, 2, 1, false, 2>")
    fb, fs, fn = vals["fetch"]
    wb, ws, wn = vals["write"]
    assert fn == 2 and wn == 2
    assert abs(fs - 2.0) < 1e-12 and abs(ws - 1.0) < 1e-12
    assert abs(fb - 2000.0 * 1024 * 2.0) < 1e-6
    assert abs(wb - 2000.0 * 1024 * 1.0) < 1e-6


def test_traffic_is_null_for_changed_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(os.path.join(tmp_path, "profiles"))
    for rel in bench.CONV_SOURCES:
        os.makedirs(os.path.dirname(os.path.join(tmp_path, rel)), exist_ok=True)
        with open(os.path.join(tmp_path, rel), "w") as f:
            f.write("v1 " + rel)
    rec = {"fetch_bytes_per_launch": 10.0, "write_bytes_per_launch": 5.0, "source_sha": bench._sha(bench.CONV_SOURCES)}
    import json
    with open(os.path.join(tmp_path, "profiles", "traffic.json"), "w") as f:
        json.dump({"w/bf16/tag": rec}, f)
    assert bench._traffic("tag", "w", "bf16") == 15.0
    with open(os.path.join(tmp_path, bench.CONV_SOURCES[0]), "w") as f:
        f.write("v2")
    assert bench._traffic("tag", "w", "bf16") is None
