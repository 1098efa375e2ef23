"""Host-side summaries of rocprofv3 counter runs (paper_2508_20735_amd.profiling):
HBM bytes per launch, scaled by a calibration copy, and the grouping step's
dispatches folded into one launch under the library's timing name."""
import csv
import os

from paper_2508_20735_amd import profiling as P


def _write(run_dir, counter, rows):
    os.makedirs(run_dir, exist_ok=True)
    with open(os.path.join(run_dir, "x_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": kib})


def test_traffic_scales_and_groups(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    ins2 = "void dfamin::(anonymous namespace)::k_insert_lds2<4>(dfamin::InsParams)"
    ins = "void dfamin::(anonymous namespace)::k_insert(dfamin::InsParams)"
    sig = "void dfamin::(anonymous namespace)::k_signature<4>(dfamin::SigParams)"
    # a 1 MiB copy reads as 512 KiB fetched (scale 2) and 1024 KiB written
    fetch = [(copy, 512), (ins2, 100), (ins, 1), (ins2, 300), (ins, 3), (sig, 50)]
    write = [(copy, 1024), (ins2, 10), (ins, 0), (ins2, 30), (ins, 0), (sig, 5)]
    _write(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write(str(tmp_path / "w"), "WRITE_SIZE", write)
    out = P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), 1 << 20)
    assert out["fetch_scale"] == 2.0 and out["write_scale"] == 1.0
    k = out["kernels"]
    assert k["k_insert_lds2"]["launches"] == 2
    assert k["k_insert_lds2"]["fetch_bytes_per_launch"] == 200 * 1024 * 2
    assert k["k_signature"]["hbm_bytes_per_launch"] == (50 * 2 + 5) * 1024
    lib = out["library_kernels"]
    # one library launch = one k_insert_lds2 and one k_insert dispatch
    assert lib["k_insert"]["launches"] == 2
    assert lib["k_insert"]["fetch_bytes_per_launch"] == (100 + 1 + 300 + 3) * 1024 * 2 / 2
    assert lib["k_insert"]["write_bytes_per_launch"] == (10 + 30) * 1024 / 2
    assert lib["k_signature"] == k["k_signature"]
    assert "k_insert_lds2" not in lib


def test_short_and_base_names():
    n = "void dfamin::(anonymous namespace)::k_pb_scatter<16>(unsigned int const*, ...)"
    assert P.short_name(n) == "k_pb_scatter<16>"
    assert P.base_name(n) == "k_pb_scatter"


def test_packed_slice_round_is_one_library_launch(tmp_path):
    """The packed label round through slices is three dispatches (byte
    gather, round, label count) under one timing name, k_packed_pb."""
    copy = "__amd_rocclr_copyBuffer"
    g8 = "void dfamin::(anonymous namespace)::k_pb_gather8(dfamin::(anonymous namespace)::SigParams)"
    pk = "void dfamin::(anonymous namespace)::k_packed_pb<4>(dfamin::(anonymous namespace)::SigParams)"
    cnt = "void dfamin::(anonymous namespace)::k_count_labels(dfamin::(anonymous namespace)::SigParams)"
    fetch = [(copy, 512), (g8, 40), (pk, 200), (cnt, 16384), (g8, 60), (pk, 300), (cnt, 16384)]
    write = [(copy, 1024), (g8, 10), (pk, 20), (cnt, 0), (g8, 30), (pk, 40), (cnt, 0)]
    _write(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write(str(tmp_path / "w"), "WRITE_SIZE", write)
    out = P.traffic(str(tmp_path / "f"), str(tmp_path / "w"), 1 << 20)
    lib = out["library_kernels"]
    assert set(lib) == {"k_packed_pb"}
    e = lib["k_packed_pb"]
    assert e["launches"] == 2
    assert e["dispatches"] == {"k_pb_gather8": 2, "k_packed_pb": 2, "k_count_labels": 2}
    assert e["fetch_bytes_per_launch"] == (40 + 200 + 16384 + 60 + 300 + 16384) * 1024 * 2 / 2
    assert e["write_bytes_per_launch"] == (10 + 20 + 30 + 40) * 1024 / 2
