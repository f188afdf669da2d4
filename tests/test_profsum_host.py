"""Host tests of the rocprofv3 summary code on small hand-made counter files.

The counter values below are chosen so every figure is known by hand: a
256 MiB device copy whose FETCH_SIZE reads half its bytes (128-byte requests
counted as 64 bytes), and kernels whose read requests are all 32, 64 or 128
bytes wide.
"""
import csv
import json
import os

from paper_1707_05354_amd import profsum

HEADER = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]
COPY = 1 << 28


def write_csv(path, rows):
    """rows: (dispatch id, kernel name, counter name, value)."""
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEADER)
        for d, name, counter, value in rows:
            w.writerow([d, d, "Agent 1", 1, 1, 1, 64, 1, name, 64, 0, 0, 8, 0, 16, counter, value,
                        0, 1])


def make_traffic(tmp_path):
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    cf = tmp_path / "copy_fetch.csv"
    cw = tmp_path / "copy_write.csv"
    k_stream = "void lsm::(anonymous namespace)::k_merge<8>(lsm::MergeArgs)"
    k_rand = "void lsm::(anonymous namespace)::k_lookup(lsm::QueryArgs)"
    write_csv(fetch, [(1, k_stream, "FETCH_SIZE", 1024.0), (2, k_stream, "FETCH_SIZE", 3072.0),
                      (3, k_rand, "FETCH_SIZE", 64.0)])
    write_csv(write, [(1, k_stream, "WRITE_SIZE", 4096.0), (2, k_stream, "WRITE_SIZE", 4096.0),
                      (3, k_rand, "WRITE_SIZE", 8.0)])
    write_csv(cf, [(1, "fill", "FETCH_SIZE", 1.0),
                   (2, "__amd_rocclr_copyBuffer", "FETCH_SIZE", COPY / 2048.0)])
    write_csv(cw, [(1, "fill", "WRITE_SIZE", 1.0),
                   (2, "__amd_rocclr_copyBuffer", "WRITE_SIZE", COPY / 1024.0)])
    md = tmp_path / "traffic.md"
    doc = profsum.counters(str(fetch), str(write), str(cf), str(cw), COPY, str(md), ["cmd"])
    return doc, md


def test_copy_scaled_traffic(tmp_path):
    doc, md = make_traffic(tmp_path)
    assert abs(doc["fetch_scale"] - 2.0) < 1e-12 and abs(doc["write_scale"] - 1.0) < 1e-12
    k = doc["kernels"]["k_merge<8>"]
    assert k["dispatches"] == 2
    assert k["fetch_bytes_per_launch"] == 2048 * 1024 * 2.0
    assert k["write_bytes_per_launch"] == 4096 * 1024
    assert profsum.load_traffic(str(md))["kernels"] == json.loads(json.dumps(doc["kernels"]))


def test_stale_traffic_is_dropped(tmp_path):
    _, md = make_traffic(tmp_path)
    text = md.read_text().replace(profsum.kernel_source_sha256(), "0" * 64)
    md.write_text(text)
    assert profsum.load_traffic(str(md)) is None
    assert profsum.load_traffic(str(tmp_path / "missing.md")) is None


def test_read_bytes_from_request_sizes(tmp_path):
    _, md = make_traffic(tmp_path)
    sizes = tmp_path / "sizes.csv"
    csizes = tmp_path / "copy_sizes.csv"
    k_stream = "void lsm::(anonymous namespace)::k_merge<8>(lsm::MergeArgs)"
    k_rand = "void lsm::(anonymous namespace)::k_lookup(lsm::QueryArgs)"
    rows = []
    # k_merge: 4 MiB of 128-byte requests per launch (what its scaled FETCH_SIZE says).
    for d in (1, 2):
        rows += [(d, k_stream, "TCC_EA0_RDREQ_32B_sum", 0.0),
                 (d, k_stream, "TCC_EA0_RDREQ_64B_sum", 0.0),
                 (d, k_stream, "TCC_EA0_RDREQ_128B_sum", 4 * 1024 * 1024 / 128.0)]
    # k_lookup: 64 KiB read as 64-byte requests; the copy scale doubles it.
    rows += [(3, k_rand, "TCC_EA0_RDREQ_32B_sum", 0.0),
             (3, k_rand, "TCC_EA0_RDREQ_64B_sum", 1024.0),
             (3, k_rand, "TCC_EA0_RDREQ_128B_sum", 0.0)]
    write_csv(sizes, rows)
    write_csv(csizes, [(1, "fill", "TCC_EA0_RDREQ_32B_sum", 2.0),
                       (2, "__amd_rocclr_copyBuffer", "TCC_EA0_RDREQ_32B_sum", 0.0),
                       (2, "__amd_rocclr_copyBuffer", "TCC_EA0_RDREQ_64B_sum", 0.0),
                       (2, "__amd_rocclr_copyBuffer", "TCC_EA0_RDREQ_128B_sum", COPY / 128.0)])
    out = tmp_path / "sizes.md"
    doc = profsum.readsizes(str(sizes), str(csizes), COPY, str(md), str(out), ["cmd"])
    assert doc["copy_read_bytes_from_sizes"] == COPY
    m = doc["kernels"]["k_merge<8>"]
    assert m["dispatches"] == 2 and m["read_bytes_per_launch"] == 4 * 1024 * 1024
    assert abs(m["scaled_over_sized"] - 1.0) < 1e-12
    q = doc["kernels"]["k_lookup"]
    assert q["read_bytes_per_launch"] == 64 * 1024
    assert abs(q["scaled_over_sized"] - 2.0) < 1e-12
    text = out.read_text()
    assert "| k_lookup | 1 | 0 | 1024 | 0 | 65536 | 131072 | 2.000 |" in text
    assert os.path.getsize(out) < 8192
