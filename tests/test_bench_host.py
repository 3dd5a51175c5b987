"""Host logic of bench.py (no GPU): the flop bases behind `value` and the roofline,
and the gate that reports the rocprofv3 traffic record only while the GEMM sources
hash to the value it was measured with."""
import hashlib
import json
import os

import pytest

import bench


@pytest.mark.parametrize("order", [2, 3, 4])
@pytest.mark.parametrize("n", [1, 7, 256, 4096])
def test_flop_bases_count_the_products(n, order):
    """A residual evaluation is S Z (2 N^3) and the symmetric Z^T (S Z); an update of
    order m is m - 1 symmetric delta products and the full Z Q.  The irreducible basis
    counts a symmetric product as N^3 (its N^2 (N + 1) per-launch count, less the
    diagonal), the paper's basis every product as dense (2 N^3)."""
    f = bench.kernel_alg_flops
    x3 = lambda c: f(c, n) / 3.0  # one product of the three
    ev = x3("gemm_x3") + x3("gemm_x3_sym")
    up = (order - 1) * x3("gemm_x3_sym") + x3("gemm_x3")
    for evals, updates in [(1, 0), (1, 1), (7, 6), (9, 7)]:
        exact = evals * ev + updates * up
        got = bench.alg_flops(n, order, evals, updates)
        # the irreducible basis drops the diagonal's N^2 per symmetric product
        assert abs(got - exact) <= (evals + (order - 1) * updates) * n * n
        assert got == n ** 3 * (3 * evals + (order + 1) * updates)
        assert bench.paper_flops(n, order, evals, updates) == n ** 3 * (4 * evals + 2 * order * updates)
    # order 2: 6 N^3 per sweep, 8 N^3 on the dense count
    assert bench.alg_flops(n, 2, 1, 1) == 6 * n ** 3
    assert bench.paper_flops(n, 2, 1, 1) == 8 * n ** 3
    # the emulated FP64 products stand for the FP64 flops they replace
    assert f("gemm_crt", n) == f("gemm_f64", n) and f("gemm_crt_sym", n) == f("gemm_f64_sym", n)


def _tree(tmp_path, record):
    for i, rel in enumerate(bench.GEMM_SOURCES):
        p = tmp_path / rel
        p.parent.mkdir(parents=True, exist_ok=True)
        p.write_bytes(f"// source {i}\n".encode())
    h = hashlib.sha256()
    for rel in bench.GEMM_SOURCES:
        h.update((tmp_path / rel).read_bytes())
    rec = dict(record, sources_sha256=h.hexdigest())
    prof = tmp_path / bench.TRAFFIC_PROFILE
    prof.parent.mkdir(parents=True, exist_ok=True)
    prof.write_text("# summary\n\n```json\n" + json.dumps(rec) + "\n```\n")
    return prof


def test_traffic_record_gated_by_the_sources(tmp_path, monkeypatch):
    rec = {"kernel": "gemm_x3", "n": 4096, "traffic_bytes_per_dispatch": 123456789,
           "alg_bytes_per_dispatch": 98765}
    _tree(tmp_path, rec)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("gemm_x3", 4096) == (123456789, 98765)
    # another kernel or order: no record
    assert bench.measured_traffic("gemm_x3_sym", 4096) == (None, None)
    assert bench.measured_traffic("gemm_x3", 2048) == (None, None)
    # one changed byte in any GEMM source invalidates it
    for rel in bench.GEMM_SOURCES:
        p = tmp_path / rel
        old = p.read_bytes()
        p.write_bytes(old + b" ")
        assert bench.measured_traffic("gemm_x3", 4096) == (None, None)
        p.write_bytes(old)
    assert bench.measured_traffic("gemm_x3", 4096) == (123456789, 98765)
    # a missing source or profile: no record, no exception
    os.remove(tmp_path / bench.GEMM_SOURCES[0])
    assert bench.measured_traffic("gemm_x3", 4096) == (None, None)


def test_committed_traffic_record_is_well_formed():
    """The committed record parses and names the dominant kernel at N = 4096; its
    traffic is at least the algorithmic bytes (operands read once, outputs written
    once), and the fetch / write factors are the copy calibration's."""
    import re
    text = open(os.path.join(bench.ROOT, bench.TRAFFIC_PROFILE)).read()
    rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
    assert rec["kernel"] == "gemm_x3" and rec["n"] == 4096
    assert rec["traffic_bytes_per_dispatch"] >= rec["alg_bytes_per_dispatch"] > 0
    assert 1.9 <= rec["fetch_factor"] <= 2.1 and 0.9 <= rec["write_factor"] <= 1.1
    calib = 1024 * (rec["fetch_kib"] * rec["fetch_factor"] + rec["write_kib"] * rec["write_factor"])
    assert abs(calib - rec["traffic_bytes_per_dispatch"]) <= 1e-4 * calib
