"""Host logic of the counter summary: calibration scaling, kernel filter,
per-dispatch aggregation of split counter rows, and the source hash."""
import json

from paper_2312_02891_amd import pmc

HDR = ('"Correlation_Id","Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')


def _csv(path, rows):
    with open(path, "w") as fh:
        fh.write(HDR)
        for d, name, cnt, val in rows:
            fh.write(f'{d},{d},"{name}","{cnt}",{val}\n')


def test_summary_scales_by_the_copy_and_filters_kernels(tmp_path):
    cf, cw = tmp_path / "cf.csv", tmp_path / "cw.csv"
    kf, kw = tmp_path / "kf.csv", tmp_path / "kw.csv"
    # the copy of 4 MiB counts half of its reads and all of its writes
    _csv(cf, [(1, "fill", "FETCH_SIZE", 1.0), (2, "copyBuffer", "FETCH_SIZE", 2048.0),
              (3, "copyBuffer", "FETCH_SIZE", 2048.0)])
    _csv(cw, [(2, "copyBuffer", "WRITE_SIZE", 4096.0)])
    # dispatch 7 is reported in two rows (two hardware instances)
    _csv(kf, [(7, "k_gram_vu<double, 4>", "FETCH_SIZE", 100.0),
              (7, "k_gram_vu<double, 4>", "FETCH_SIZE", 50.0),
              (8, "k_gram_vu<double, 4>", "FETCH_SIZE", 250.0),
              (9, "k_update<double, 4>", "FETCH_SIZE", 9999.0)])
    _csv(kw, [(7, "k_gram_vu<double, 4>", "WRITE_SIZE", 10.0),
              (8, "k_gram_vu<double, 4>", "WRITE_SIZE", 30.0)])
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    out = tmp_path / "t.json"
    pmc.main(["summarize", "--fetch", str(kf), "--write", str(kw), "--calib-fetch", str(cf),
              "--calib-write", str(cw), "--kernel", r"k_gram_vu<double, 4>",
              "--calib-kernel", "copyBuffer", "--mib", "4", "--source", str(src),
              "--json", str(out)])
    t = json.loads(out.read_text())
    assert t["scale"] == {"fetch": 2.0, "write": 1.0}
    assert t["dispatches"]["fetch"] == 2
    # mean fetch (150 + 250) / 2 KiB, doubled; mean write 20 KiB
    assert t["fetch_bytes_per_dispatch"] == 400 * 1024
    assert t["write_bytes_per_dispatch"] == 20 * 1024
    assert t["traffic_bytes_per_dispatch"] == 420 * 1024
    assert t["source_sha256"] == pmc.source_digest([str(src)])
    src.write_text("kernel source, changed")
    assert t["source_sha256"] != pmc.source_digest([str(src)])
