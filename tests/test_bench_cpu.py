"""Host logic of bench.py: the HBM traffic it reports is read from a committed
counter summary only while that summary's recorded kernel SHA-256 is the
current source's, and each committed summary's figure lies between the bytes
the kernel must read and that plus every output it may write."""
import hashlib
import importlib.util
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_traffic_needs_the_current_kernel_source(tmp_path):
    b = _bench()
    src = hashlib.sha256(open(b.JACOBI_SRC, "rb").read()).hexdigest()
    good = tmp_path / "good.md"
    good.write_text("x\ntraffic_bytes_per_launch: 12345\nkernel_source_sha256: %s\n" % src)
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch: 12345\nkernel_source_sha256: %s\n" % ("0" * 64))
    assert b.measured_traffic(str(good)) == 12345
    assert b.measured_traffic(str(stale)) is None
    assert b.measured_traffic(str(tmp_path / "missing.md")) is None


def _committed(path):
    text = open(path).read()
    m = re.search(r"traffic_bytes_per_launch:\s*(\d+)", text)
    return int(m.group(1)) if m else None


def test_committed_figures_are_within_the_algorithmic_bytes():
    b = _bench()
    f = 4   # FP32
    # warm real kernel, 150 slices: M and Z read (144 x 144 each), Z written,
    # at most all 144 kept columns of 144 rows written
    t = _committed(b.TRAFFIC_PROFILE)
    lo = 150 * (2 * 144 * 144 + 144 * 144) * f
    assert lo <= t <= lo + 150 * 144 * 144 * f
    # complex kernel, 76 representatives: the 288 x 144 interleaved factor
    # read; each kept column written with its twin (at most 288 columns of 288)
    t = _committed(b.TRAFFIC_PROFILE_DFT)
    lo = 76 * 288 * 144 * f
    assert lo <= t <= lo + 76 * 288 * 288 * f
