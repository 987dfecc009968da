"""Host-side checks of bench.py: the one-GPU contract, and the HBM traffic
table that feeds ``roofline.traffic`` (no GPU needed)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_contract_probe", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("n", [2, 8])
def test_multi_gpu_request_exits_with_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_table_entries_are_well_formed():
    b = _bench_module()
    for name, t in b.TRAFFIC.items():
        assert t["bytes_per_dispatch"] > 0
        # the digest is taken over existing source sections: a marker that no
        # longer matches raises instead of silently nulling the figure
        d = b.kernel_digest(t["sources"])
        assert len(d) == 16
        got = b.traffic_for(name)
        assert got is None or got == int(round(t["bytes_per_dispatch"]))
    assert b.traffic_for("no_such_kernel") is None


def test_traffic_at_least_algorithmic():
    # measured HBM bytes per dispatch can exceed the algorithmic bytes (re-reads)
    # but never undercut them: 16384^2 x 8 B per Jacobi sweep, and one 1 GiB A
    # panel, one 1 GiB B panel and a 64 MiB C tile per GEMM dispatch
    b = _bench_module()
    assert b.TRAFFIC["k_jacobi2d_stack"]["bytes_per_dispatch"] >= 16384 * 16384 * 8
    assert b.TRAFFIC["k_gemm"]["bytes_per_dispatch"] >= 2 * 4096 * 65536 * 4 + 4096 * 4096 * 4
    # k-means: 64 B per point and its 4 B label for 2^26 points per assignment
    # dispatch and 2^22 per update dispatch (plus the partial slots)
    assert b.TRAFFIC["k_kmeans"]["bytes_per_dispatch"] >= (1 << 26) * 68
    # 512 partial slots per 2^22-point superblock at d = 16
    assert b.TRAFFIC["k_kmeans_update"]["bytes_per_dispatch"] >= (1 << 22) * 68 + 512 * (64 * 16 * 8 + 64 * 4)


def test_copy_overlap_measures_copy_time_under_kernels():
    import numpy as np

    b = _bench_module()
    dt = [("name", "S32"), ("stream", np.int32), ("start_ms", np.float64), ("end_ms", np.float64)]
    # H2D copies [0, 10] and [12, 20] (18 ms in flight), kernels [5, 15] and
    # [14, 16] (merged: [5, 16]); D2H [14, 18]
    sp = np.array([(b"copy_h2d", 4, 0.0, 10.0), (b"copy_h2d", 4, 12.0, 20.0), (b"k", 0, 5.0, 15.0),
                   (b"k", 1, 14.0, 16.0), (b"copy_d2h", 5, 14.0, 18.0)], dtype=dt)
    o = b.copy_overlap(sp)
    assert o["kernel_busy_ms"] == 11.0
    assert o["h2d"]["copies"] == 2 and o["h2d"]["busy_ms"] == 18.0
    assert abs(o["h2d"]["overlap_frac"] - 9.0 / 18.0) < 1e-12   # [5, 10] and [12, 16]
    assert abs(o["d2h"]["overlap_frac"] - 2.0 / 4.0) < 1e-12    # [14, 16]
    # kernels [5, 16] under copies [0, 10] U [12, 20]: [5, 10] and [12, 16]
    assert abs(o["kernel_under_copy_frac"] - 9.0 / 11.0) < 1e-4   # rounded to 4 places
    # overlapping copies of one direction count once
    sp2 = np.array([(b"copy_h2d", 4, 0.0, 4.0), (b"copy_h2d", 4, 2.0, 6.0), (b"k", 0, 0.0, 6.0)], dtype=dt)
    o2 = b.copy_overlap(sp2)
    assert o2["h2d"]["busy_ms"] == 6.0 and o2["h2d"]["overlap_frac"] == 1.0
    assert o2["d2h"]["overlap_frac"] is None
