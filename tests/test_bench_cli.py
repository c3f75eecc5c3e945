"""Host-side contract of bench.py (no GPU): a multi-GPU request is refused
with a message, and the algorithmic byte counts of the roofline follow
their definitions."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_algorithmic_bytes():
    H, W, T = 64, 80, 3
    a = bench.algorithmic_bytes(H, W, T, 1, 12, n_cand=7)
    # the star pass reads the tables once (three tables of (H+1)(W+1)
    # entries) and writes the uint8 mask; the builder reads the image once
    # and writes the tables; the list is 16 bytes per candidate.  The
    # implementation's own scratch (scale-bit words, staged candidates) is
    # not counted.
    assert a["star_plain"] == 3 * (H + 1) * (W + 1) * 12 + T * H * W
    assert a["star_batch"] == a["star_plain"]
    assert a["band_final"] == 3 * (H + 1) * (W + 1) * 12 + H * W
    assert a["compact_list"] == 16 * 7


def test_batch_group_matches_header():
    """The lookup count of a batched launch uses the library's group size."""
    import re
    src = open(os.path.join(ROOT, "paper_1707_05647_amd", "csrc", "oss_internal.h")).read()
    assert int(re.search(r"BATCH_GROUP = (\d+);", src).group(1)) == bench.BATCH_GROUP
    assert int(re.search(r"BATCH_GROUP_RINGS = (\d+);", src).group(1)) == bench.BATCH_GROUP_RINGS


def test_default_line_is_the_headline_workload():
    a = bench.parse_args([])
    assert a.workload == 0 and a.gpus == 1


def test_pixel_scales_count_valid_positions():
    # a radius-r star fits at (H - 2r)(W - 2r) positions; none when 2r >= H
    assert bench.pixel_scales(10, 12, [(0, 0, 2), (0, 1, 5)]) == 6 * 8 + 0


def test_lanes_copy_every_option():
    """The lanes of a two-lane run are contexts that copy the main context's
    options: every option the header defines must be in that list."""
    import re
    hdr = open(os.path.join(ROOT, "include", "oss.h")).read()
    defined = set(re.findall(r"#define (OSS_OPT_\w+) \d+", hdr))
    assert defined and set(bench.OPTIONS) == defined


def test_binding_option_ids_match_header():
    import re
    from paper_1707_05647_amd import _lib as L
    hdr = open(os.path.join(ROOT, "include", "oss.h")).read()
    for name, val in re.findall(r"#define (OSS_OPT_\w+) (\d+)", hdr):
        assert getattr(L, name) == int(val), name


def test_screen_gate_orders_screens():
    """The serial-screens gate: the first screen waits for nothing, each
    later screen waits for the event recorded after the previous one."""
    class Ev:
        def __init__(self):
            self.on = None

        def record(self, st):
            self.on = st

    class FakeTorch:
        class cuda:
            Event = Ev

    class St:
        def __init__(self, name):
            self.name, self.waited = name, []

        def wait_event(self, ev):
            self.waited.append(ev.on.name)

    g = bench.ScreenGate(FakeTorch)
    a, b = St("a"), St("b")
    g.wait(a)
    g.record(a)
    g.wait(b)
    g.record(b)
    g.wait(a)
    assert a.waited == ["b"] and b.waited == ["a"]
