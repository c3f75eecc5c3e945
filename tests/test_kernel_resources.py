"""Resources of the built kernels, read on the CPU from the gfx950 code
objects inside liboss.so (the AMDGPU metadata note of each): no kernel uses
scratch memory or spills vector registers, and the batched star kernels keep
the occupancy the sweep relies on (64-template groups within 168 VGPRs,
3 waves per SIMD, and within 128, 4 waves, for the mixed and planar
split-square layouts; the 16-template planar staged kernel of the large
workload within 72: 7 waves)."""
import os
import re
import struct
import subprocess
import tempfile

import pytest
import yaml

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1707_05647_amd", "liboss.so")
READELF = "/opt/rocm/llvm/bin/llvm-readelf"


def _code_objects(path):
    """The gfx950 code objects of every offload bundle in the library."""
    data = open(path, "rb").read()
    out = []
    for m in re.finditer(b"__CLANG_OFFLOAD_BUNDLE__", data):
        off = m.start()
        n = struct.unpack_from("<Q", data, off + 24)[0]
        p = off + 32
        for _ in range(n):
            eo, es, ts = struct.unpack_from("<QQQ", data, p)
            p += 24
            triple = data[p:p + ts].decode()
            p += ts
            if "gfx950" in triple:
                out.append(data[off + eo:off + eo + es])
    return out


def _kernels():
    ks = {}
    for co in _code_objects(LIB):
        with tempfile.NamedTemporaryFile(suffix=".co", delete=False) as f:
            f.write(co)
            name = f.name
        try:
            txt = subprocess.run([READELF, "--notes", name], capture_output=True, text=True,
                                 check=True).stdout
        finally:
            os.unlink(name)
        body = txt[txt.index("---"):]
        body = body[:body.index("\n...") + 4] if "\n..." in body else body
        meta = yaml.safe_load(body)
        for k in meta["amdhsa.kernels"]:
            ks[k[".name"]] = k
    return ks


@pytest.mark.skipif(not (os.path.exists(LIB) and os.path.exists(READELF)),
                    reason="library not built or llvm-readelf missing")
def test_no_scratch_and_batched_occupancy():
    ks = _kernels()
    lib = {n: k for n, k in ks.items() if "oss" in n}
    assert len(lib) > 100
    scratch = [n for n, k in lib.items() if k.get(".private_segment_fixed_size", 0) != 0]
    assert not scratch, f"kernels using scratch memory: {scratch[:5]}"
    spills = [n for n, k in lib.items() if k.get(".vgpr_spill_count", 0) != 0]
    assert not spills, f"kernels spilling VGPRs: {spills[:5]}"
    big = {n: k[".vgpr_count"] for n, k in lib.items()
           if "star_batch_kernel" in n and re.search(r"EEELi64ELb0", n)}
    # every 64-template kernel keeps 3 waves per SIMD, those of the mixed
    # and planar split-square layouts (the 8192^2 and 16384^2 workloads) 4
    assert big and max(big.values()) <= 168, big
    mixed = {n: v for n, v in big.items() if "TabMix" in n or "TabPS" in n}
    assert mixed and max(mixed.values()) <= 128, mixed
    head = [k[".vgpr_count"] for n, k in lib.items()
            if "star_batch_kernel" in n and "TabPSILi3ELi1EEELi16ELb0ELb1" in n]
    assert head and head[0] <= 72, head
