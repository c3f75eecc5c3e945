"""Per-kernel HBM traffic from rocprofv3 counter runs.

    python -m paper_1707_05647_amd.traffic FETCH_CSV WRITE_CSV COPY_MIB OUT_JSON

FETCH_CSV / WRITE_CSV are rocprofv3 ``counter_collection.csv`` files of two
runs of ``bench.py --copy-probe-mb COPY_MIB`` with ``--pmc FETCH_SIZE`` and
``--pmc WRITE_SIZE`` (KiB per dispatch).  The plain copy kernel in the same
run moves COPY_MIB MiB each way; its counter readings give the scale factor
(bytes per counted KiB) applied to every kernel.  Writes OUT_JSON with, per
library kernel, the mean scaled read and write bytes per launch and a
hash of the sources the kernel was built from.
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
    "compact_scan": ("compact_scan_kernel", "paper_1707_05647_amd/csrc/compact.hip"),
    "compact_list": ("compact_list_kernel", "paper_1707_05647_amd/csrc/compact.hip"),
    "copy": ("copy", None),
}


# headers every kernel source includes (a change there can change the kernel)
SHARED = ("paper_1707_05647_amd/csrc/oss_internal.h", "paper_1707_05647_amd/csrc/star_common.h")


def kernel_sha(short: str) -> str:
    """Hash of the source file a kernel is built from and the shared headers."""
    h = hashlib.sha256()
    for path in (KERNELS[short][1], *SHARED):
        with open(os.path.join(ROOT, path), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counter(path, counter):
    """{short kernel name: [values per dispatch]} for one counter."""
    out = defaultdict(list)
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = row.get("Kernel_Name", "")
            for short, (needle, _) in KERNELS.items():
                if needle in name:
                    out[short].append(float(row["Counter_Value"]))
                    break
    return out


def main(fetch_csv, write_csv, copy_mib, out_json):
    fetch = read_counter(fetch_csv, "FETCH_SIZE")
    write = read_counter(write_csv, "WRITE_SIZE")
    copy_bytes = float(copy_mib) * (1 << 20)
    if not fetch.get("copy") or not write.get("copy"):
        raise SystemExit("no copy kernel in the counter runs")
    f_scale = copy_bytes / max(fetch["copy"])   # bytes per counted unit
    w_scale = copy_bytes / max(write["copy"])
    res = {"copy_mib": copy_mib, "fetch_bytes_per_unit": f_scale,
           "write_bytes_per_unit": w_scale, "kernels": {}}
    for short in KERNELS:
        if short == "copy" or short not in fetch:
            continue
        fv, wv = fetch[short], write.get(short, [0.0])
        rd = f_scale * sum(fv) / len(fv)
        wr = w_scale * sum(wv) / len(wv)
        res["kernels"][short] = {"read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
                                 "hbm_bytes_per_launch": rd + wr, "dispatches": len(fv),
                                 "source_sha": kernel_sha(short)}
    with open(out_json, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


if __name__ == "__main__":
    if len(sys.argv) != 5:
        raise SystemExit(__doc__)
    main(sys.argv[1], sys.argv[2], int(sys.argv[3]), sys.argv[4])
