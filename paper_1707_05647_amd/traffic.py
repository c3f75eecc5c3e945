"""Per-kernel HBM traffic from rocprofv3 counter runs.

    python -m paper_1707_05647_amd.traffic FETCH_CSV WRITE_CSV COPY_MIB OUT_JSON [SIZES_CSV]

FETCH_CSV / WRITE_CSV are rocprofv3 ``counter_collection.csv`` files of two
runs of ``bench.py --copy-probe-mb COPY_MIB`` with ``--pmc FETCH_SIZE`` and
``--pmc WRITE_SIZE`` (KiB per dispatch).  The probe is the run's first GPU
work: a fill of a COPY_MIB MiB byte tensor, then one device-to-device copy of
it, which the runtime may split into several copy dispatches.  The copy
dispatches that directly follow that first fill are the probe; their summed
readings against the COPY_MIB MiB each way give the scale factor (bytes per
counted KiB) applied to every kernel.

SIZES_CSV (optional) is a third run with ``--pmc TCC_EA0_RDREQ_sum
TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum TCC_EA0_RDREQ_128B_sum``: the
L2's read requests to memory by size, which give each kernel's read bytes
without a scale factor (a cross-check of the calibrated figure).

Writes OUT_JSON with, per library kernel, the mean scaled read and write
bytes per launch and a hash of the sources the kernel was built from.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

KERNELS = {
    # short name: (substring of the mangled / demangled name, source file)
    "row_base": ("row_base_kernel", "paper_1707_05647_amd/csrc/builder.hip"),
    "band_agg": ("band_agg_kernel", "paper_1707_05647_amd/csrc/builder.hip"),
    "carry": ("carry_kernel", "paper_1707_05647_amd/csrc/builder.hip"),
    "band_final": ("band_final_kernel", "paper_1707_05647_amd/csrc/builder.hip"),
    "star_plain": ("star_plain_kernel", "paper_1707_05647_amd/csrc/star.hip"),
    "star_batch": ("star_batch_kernel", "paper_1707_05647_amd/csrc/batched_kernel.h"),
    "star_moments": ("star_moments_kernel", "paper_1707_05647_amd/csrc/moments.hip"),
    "compact_sum": ("compact_sum_kernel", "paper_1707_05647_amd/csrc/compact.hip"),
    "compact_scan": ("compact_scan_kernel", "paper_1707_05647_amd/csrc/compact.hip"),
    "compact_add": ("compact_add_kernel", "paper_1707_05647_amd/csrc/compact.hip"),
    "compact_list": ("compact_list_kernel", "paper_1707_05647_amd/csrc/compact.hip"),
}

PROBE_FILL = "FillFunctor<unsigned char>"
PROBE_COPY = "copyBuffer"

# headers every kernel source includes (a change there can change the kernel)
SHARED = ("paper_1707_05647_amd/csrc/oss_internal.h", "paper_1707_05647_amd/csrc/star_common.h")

SIZE_COUNTERS = ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")


def kernel_sha(short: str) -> str:
    """Hash of the source file a kernel is built from and the shared headers."""
    h = hashlib.sha256()
    for path in (KERNELS[short][1], *SHARED):
        with open(os.path.join(ROOT, path), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(kernel_name: str):
    for short, (needle, _) in KERNELS.items():
        if needle in kernel_name:
            return short
    return None


def read_rows(path):
    """[(dispatch id, kernel name, {counter: value})] in dispatch order."""
    by_id = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            d = int(row["Dispatch_Id"])
            ent = by_id.setdefault(d, (row.get("Kernel_Name", ""), {}))
            ent[1][row["Counter_Name"]] = float(row["Counter_Value"])
    return [(d, by_id[d][0], by_id[d][1]) for d in sorted(by_id)]


def probe_sum(rows, counter):
    """Summed `counter` over the copy dispatches that directly follow the
    first byte fill (the probe's copy, however the runtime split it)."""
    i = next((k for k, r in enumerate(rows) if PROBE_FILL in r[1]), None)
    if i is None:
        raise SystemExit("no probe fill (a byte fill as the first GPU work) in the counter run")
    total, n = 0.0, 0
    for _, name, vals in rows[i + 1:]:
        if PROBE_COPY not in name:
            break
        total += vals.get(counter, 0.0)
        n += 1
    if n == 0:
        raise SystemExit("no copy dispatch right after the probe fill")
    return total, n


def per_kernel(rows, counter):
    """{short kernel name: [values per dispatch]} for one counter."""
    out = defaultdict(list)
    for _, name, vals in rows:
        short = short_name(name)
        if short and counter in vals:
            out[short].append(vals[counter])
    return out


def main(fetch_csv, write_csv, copy_mib, out_json, sizes_csv=None):
    frows, wrows = read_rows(fetch_csv), read_rows(write_csv)
    copy_bytes = float(copy_mib) * (1 << 20)
    f_probe, f_n = probe_sum(frows, "FETCH_SIZE")
    w_probe, w_n = probe_sum(wrows, "WRITE_SIZE")
    f_scale = copy_bytes / f_probe  # bytes per counted KiB
    w_scale = copy_bytes / w_probe
    res = {"copy_mib": copy_mib,
           "probe": {"copy_dispatches": [f_n, w_n], "fetch_kib": f_probe, "write_kib": w_probe},
           "fetch_bytes_per_unit": f_scale, "write_bytes_per_unit": w_scale, "kernels": {}}
    fetch = per_kernel(frows, "FETCH_SIZE")
    write = per_kernel(wrows, "WRITE_SIZE")
    sizes = {}
    if sizes_csv:
        srows = read_rows(sizes_csv)
        parts = {c: per_kernel(srows, c) for c in SIZE_COUNTERS}
        for short in parts[SIZE_COUNTERS[0]]:
            n = len(parts[SIZE_COUNTERS[0]][short])
            b = sum(w * sum(parts[c][short]) for w, c in zip((32, 64, 128), SIZE_COUNTERS))
            sizes[short] = b / n
        s_probe = sum(w * probe_sum(srows, c)[0] for w, c in zip((32, 64, 128), SIZE_COUNTERS))
        res["probe"]["read_bytes_by_request_size"] = s_probe
    for short in KERNELS:
        if short not in fetch:
            continue
        fv, wv = fetch[short], write.get(short, [0.0])
        rd = f_scale * sum(fv) / len(fv)
        wr = w_scale * sum(wv) / len(wv)
        ent = {"read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
               "hbm_bytes_per_launch": rd + wr, "dispatches": len(fv),
               "fetch_kib_per_launch": sum(fv) / len(fv),
               "write_kib_per_launch": sum(wv) / len(wv),
               "source_sha": kernel_sha(short)}
        if short in sizes:
            ent["read_bytes_by_request_size"] = sizes[short]
        res["kernels"][short] = ent
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    if len(sys.argv) not in (5, 6):
        raise SystemExit(__doc__)
    main(sys.argv[1], sys.argv[2], int(sys.argv[3]), sys.argv[4],
         sys.argv[5] if len(sys.argv) == 6 else None)
