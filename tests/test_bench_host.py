"""Host-side checks of the benchmark's bookkeeping (no GPU): the kernel
names it looks up in the committed rocprofv3 traffic summary exist there,
and the figures it takes from it are plausible."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import pytest  # noqa: E402


def test_traffic_summary_names_the_bench_kernels():
    """Every window of the bench step maps to a kernel name with a
    traffic-per-launch line in the summary (a renamed or re-templated kernel
    would silently drop the traffic figure from the bench line)."""
    path = os.path.join(ROOT, bench.TRAFFIC_FILE)
    names = set()
    for line in open(path):
        if line.startswith("traffic-per-launch:"):
            names.add(line.split(":", 1)[1].rsplit("=", 1)[0].strip())
    for w in (16, 256, 4096, 65536):
        k = bench.kernel_name("tile" if w <= 8192 else "chunk", w)
        assert k in names, (w, k, sorted(names))


def test_traffic_summary_is_plausible():
    """While the summary belongs to the current kernel sources (else the
    bench reports null traffic, by design), the dominant kernel's measured
    HBM bytes lie between the algorithmic bytes and 10% above them."""
    v, src = bench.measured_traffic(bench.kernel_name("tile", 16), 1 << 28)
    if v is None:
        pytest.skip("traffic summary: %s" % src)
    alg = bench.alg_bytes(1 << 28, 16, 4)
    assert 1.0 <= v / alg < 1.1, v / alg
