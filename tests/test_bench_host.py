"""Host logic of bench.py, no GPU needed: the one-GPU contract, the algorithmic byte counts of
the streaming and emitter kernels (their differences between forms), and the measured traffic
figure, which is reported only while the kernel sources are the ones it was measured on."""
import os
import re
import subprocess
import sys

import bench
from paper_2301_07684_amd import build


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and r.stdout == ""
    assert "one GPU" in r.stderr


def test_byte_counts_differ_between_forms_by_what_each_form_moves():
    n, live, em, conv = 10_000, 9_000, 700, 50
    plain = bench.stream_kernel_bytes(n, live, em, conv)
    # every slot's alive flag, 80 B read per live particle, the depth of every live
    # non-acting particle written
    assert plain == n + 80 * live + 8 * (live - em - conv)
    # plane-wave tiles: amplitude and phase (16 B) instead of E and B (48 B) per live particle
    assert plain - bench.wave_stream_kernel_bytes(n, live, em, conv) == 32 * live
    # the fused push: 24 B of momentum written for each live lepton that does not emit
    leptons = 4_000
    assert (bench.pushed_stream_kernel_bytes(n, live, em, conv, leptons) - plain
            == 24 * (leptons - em))
    # nobody acting: one read and one write of the depth, no emitter traffic
    assert bench.stream_kernel_bytes(n, n, 0, 0) == 89 * n
    assert bench.emit_kernel_bytes(0, 0) == 0
    # the emitter kernel grows linearly with emissions and conversions
    assert bench.emit_kernel_bytes(2 * em, 2 * conv) == 2 * bench.emit_kernel_bytes(em, conv)
    # a uniform-field tile reads p and tau only, and writes them back for non-emitters
    assert bench.constant_field_kernel_bytes(n, 0) == 64 * n
    assert bench.constant_field_kernel_bytes(n, n) == 32 * n
    # the served form's step: 170 B per beyond-LCFA electron (97 read, 73 written: pushed p,
    # F_perp, dF, flag), every photon slot's flag and 48 B per live photon; no optical depths
    assert bench.served_stream_kernel_bytes(leptons, n - leptons, live - leptons) == \
        170 * leptons + (n - leptons) + 48 * (live - leptons)
    # the whole step's yardstick: 96 B per update, 80 B per emission, 104 B per conversion
    assert bench.survey_step_bytes(live, 0, 0) == 96 * live
    assert bench.survey_step_bytes(live, em, conv) - bench.survey_step_bytes(live, 0, 0) == \
        80 * em + 104 * conv


def test_traffic_is_reported_only_for_the_measured_sources(monkeypatch):
    txt = open(bench.TRAFFIC_FILE).read()
    recorded = re.search(r"^source_hash:\s*(\S+)\s*$", txt, re.M).group(1)
    t = bench.measured_traffic()
    if recorded == build.kernel_source_hash():
        fetch = float(re.search(r"^fetch_bytes_per_launch:\s*(\S+)", txt, re.M).group(1))
        write = float(re.search(r"^write_bytes_per_launch:\s*(\S+)", txt, re.M).group(1))
        assert t == fetch + write and t > 0
    else:
        assert t is None
    monkeypatch.setattr(build, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic() is None


def test_memory_probe_library_rejects_bad_arguments_before_any_device_call():
    # the benchmark's memory-only reference (csrc/mem_probe.hip, built beside libsfq.so):
    # argument checks come first, so these calls touch no GPU
    import ctypes

    if not os.path.exists(build.PROBE_LIB):
        build.build_probe(verbose=False)
    fn = ctypes.CDLL(build.PROBE_LIB).sfq_probe_stream
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                   ctypes.POINTER(ctypes.c_float)]
    ms = ctypes.c_float(0.0)
    good = (2, 2, 1 << 20, 2048, 5)
    for bad in ((0, 2, 1 << 20, 2048, 5), (17, 2, 1 << 20, 2048, 5), (2, 3, 1 << 20, 2048, 5),
                (2, 4, 1 << 20, 1536, 5), (2, 2, 1000, 2048, 5), (2, 2, 1 << 20, 2048, 2),
                (2, 2, 0, 2048, 5)):
        assert bad != good and fn(*bad, ctypes.byref(ms)) == -1
    assert fn(*good, None) == -1
