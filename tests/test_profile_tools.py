"""The counter and trace summarizers on small synthetic rocprofv3 CSVs: the
copy probe found by position and summed over its dispatches, the scale
factors, the request-size cross-check, and the alone / overlapped split."""
import csv
import json

from paper_1707_05647_amd import trace_summary, traffic


def _counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for d, name, counter, value in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


FILL = "void at::native::vectorized_elementwise_kernel<16, at::native::FillFunctor<unsigned char>>"
COPY = "__amd_rocclr_copyBuffer"
STAR = "void oss::star_batch_kernel<oss::TabPS<3, 1>, 16, false, true>(void const*)"
LIST = "oss::compact_list_kernel(unsigned char const*)"


def test_traffic_probe_split_copy_and_sizes(tmp_path):
    # 1 MiB probe copied in two dispatches; FETCH_SIZE reads half the bytes
    mib = 1
    kib = 1024 * mib
    fetch = [(1, FILL, "FETCH_SIZE", 0.0), (2, COPY, "FETCH_SIZE", kib / 4),
             (3, COPY, "FETCH_SIZE", kib / 4), (4, STAR, "FETCH_SIZE", 100.0),
             (5, COPY, "FETCH_SIZE", 999.0),  # a later copy: not the probe
             (6, STAR, "FETCH_SIZE", 300.0), (7, LIST, "FETCH_SIZE", 10.0)]
    write = [(1, FILL, "WRITE_SIZE", kib), (2, COPY, "WRITE_SIZE", kib / 2),
             (3, COPY, "WRITE_SIZE", kib / 2), (4, STAR, "WRITE_SIZE", 8.0),
             (6, STAR, "WRITE_SIZE", 24.0), (7, LIST, "WRITE_SIZE", 4.0)]
    sizes = []
    for c, n in (("TCC_EA0_RDREQ_32B_sum", 0), ("TCC_EA0_RDREQ_64B_sum", 0),
                 ("TCC_EA0_RDREQ_128B_sum", (1 << 20) // 256)):
        sizes += [(1, FILL, c, 0.0), (2, COPY, c, n), (3, COPY, c, n)]
    sizes += [(4, STAR, "TCC_EA0_RDREQ_32B_sum", 2), (4, STAR, "TCC_EA0_RDREQ_64B_sum", 1),
              (4, STAR, "TCC_EA0_RDREQ_128B_sum", 3)]
    _counters(tmp_path / "f.csv", fetch)
    _counters(tmp_path / "w.csv", write)
    _counters(tmp_path / "s.csv", sizes)
    out = tmp_path / "t.json"
    traffic.main(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), mib, str(out),
                 str(tmp_path / "s.csv"))
    d = json.loads(out.read_text())
    assert d["probe"]["copy_dispatches"] == [2, 2]
    assert d["fetch_bytes_per_unit"] == 2048.0
    assert d["write_bytes_per_unit"] == 1024.0
    assert d["probe"]["read_bytes_by_request_size"] == float(1 << 20)
    st = d["kernels"]["star_batch"]
    assert st["dispatches"] == 2
    assert st["read_bytes_per_launch"] == 2048.0 * 200.0
    assert st["write_bytes_per_launch"] == 1024.0 * 16.0
    assert st["read_bytes_by_request_size"] == 32 * 2 + 64 * 1 + 128 * 3
    assert st["source_sha"] == traffic.kernel_sha("star_batch")
    assert "compact_list" in d["kernels"] and "copy" not in d["kernels"]


def test_trace_overlap_split(tmp_path):
    path = tmp_path / "k.csv"
    cols = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X",
            "Workgroup_Size_X", "Queue_Id"]
    runs = [(STAR, 0, 10_000_000), (STAR, 20_000_000, 30_000_000),  # alone
            (STAR, 40_000_000, 60_000_000), (LIST, 50_000_000, 51_000_000),  # overlapped
            (STAR, 70_000_000, 75_000_000), ("void other_kernel()", 72_000_000, 73_000_000)]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for name, s, e in runs:
            w.writerow({"Kernel_Name": name, "Start_Timestamp": s, "End_Timestamp": e,
                        "Grid_Size_X": 768 * 512, "Workgroup_Size_X": 512, "Queue_Id": 1})
    rows = trace_summary.load(str(path))
    assert len(rows) == 5  # the non-library kernel is dropped
    assert trace_summary.overlapped(rows) == [False, False, True, True, False]
    text = trace_summary.summarize(rows)
    assert "| star_batch | 768 x 512 | 3 | alone | 8.333 | 10.000 | 5.000 | 10.000 |" in text
    assert "| star_batch | 768 x 512 | 1 | overlapped | 20.000 | 20.000 |" in text
    # only the list pass listed; its overlap with the star pass still counts
    only = trace_summary.summarize(rows, only=["compact_list"])
    assert "star_batch" not in only
    assert "| compact_list | 768 x 512 | 1 | overlapped | 1.000 |" in only
