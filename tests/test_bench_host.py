"""Host-side logic of bench.py (CPU): the DRAM-traffic summary reads only the
benchmark call's own kernel instantiations from the rocprofv3 counter files
and scales each counter by what it reads for the 1 GiB copy kernel."""
import csv
import os

import pytest

import bench
from paper_2605_20353_amd import _lib as G


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_summary_reads_the_exact_kernels(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    lg0 = "void gcp::k_loss_grad<float, 3, 8, 4, 0>(gcp::LGParams<float>)"
    lg2 = "void gcp::k_loss_grad<float, 3, 8, 4, 2>(gcp::LGParams<float>)"      # another call's kernel
    lg16 = "void gcp::k_loss_grad<float, 3, 16, 2, 0>(gcp::LGParams<float>)"    # another lane shape
    ba = "void gcp::k_bucket_accum<float, 3, 8, 4>(gcp::LGParams<float>)"
    ad = "void gcp::k_adam<float>(gcp::AdamArgs<float>)"
    d = [str(tmp_path / n) for n in ("f", "w", "cf", "cw")]
    _write_counters(d[0], "FETCH_SIZE", [(lg0, 100), (lg0, 110), (lg0, 90)] + [(lg2, 999)] * 5 + [(lg16, 777)] * 5
                    + [(ba, 50), (ba, 50), (ad, 7)])
    _write_counters(d[1], "WRITE_SIZE", [(lg0, 30)] * 3 + [(lg2, 888)] * 5 + [(ba, 20), (ad, 9)])
    _write_counters(d[2], "FETCH_SIZE", [("void gcp::k_ceil_copy(float4 const*, float4*, long)", 524288)])
    _write_counters(d[3], "WRITE_SIZE", [("void gcp::k_ceil_copy(float4 const*, float4*, long)", 1048576)])
    out = bench.traffic_summary(d, G.Tile(lanes=8, vec=4, block=1024, bucket_modes=-1))
    cal = out["copy_calibration"]
    assert cal["fetch_factor"] == pytest.approx(2.0) and cal["write_factor"] == pytest.approx(1.0)
    per = out["per_kernel"]
    assert per["k_loss_grad"]["fetch_size_kib"] == 100 and per["k_loss_grad"]["dispatches"] == 3
    assert per["k_loss_grad"]["write_size_kib"] == 30
    assert per["k_bucket_accum"]["fetch_size_kib"] == 50
    # the call's bytes: the two kernels, Adam not included
    assert out["read_bytes_per_launch"] == (100 + 50) * 1024 * 2
    assert out["write_bytes_per_launch"] == (30 + 20) * 1024
    assert os.path.exists(bench.TRAFFIC_FILE)


def test_traffic_summary_needs_the_tile(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    with pytest.raises(SystemExit):
        bench.traffic_summary([str(tmp_path)] * 4, G.Tile())
