"""bench.py's host-side bookkeeping (no GPU): the committed traffic records are taken only for the
kernel source and launch shape they were measured on, and the algorithmic byte counts follow the
per-unit figures of the kernels' roofline table."""
import hashlib
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SHAPE = dict(scan_blocks=1024, relax_blocks=2048, chunk=256, use_graph=0, queue=2, single=0)


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def source_sha():
    h = hashlib.sha256()
    for f in ("paper_1903_12085_amd/csrc/phased.hip", "paper_1903_12085_amd/csrc/common.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


@pytest.mark.parametrize("record", ["er22", "er23", "rmat22"])
def test_traffic_record_taken_only_for_its_kernel_source(bench, record):
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_identify_%s.json" % record)))
    shapes = {r["launch"] for r in rec["by_launch"]}
    got = bench.measured_traffic("k_identify_queue", record, SHAPE)
    if rec["source_sha256"] != source_sha():
        assert got is None  # counters of another kernel version are never reported
    elif "1024,2048,256,0,2" in shapes:
        assert isinstance(got, int) and got > 0
    for r in rec["by_launch"]:  # calibrated FETCH + WRITE, as the record says
        assert r["traffic_bytes_per_launch"] == pytest.approx(
            1024 * (r["fetch_kib_per_dispatch"] * r["fetch_scale"] + r["write_kib_per_dispatch"] * r["write_scale"]),
            rel=1e-3)


def test_traffic_record_refused_for_other_shape_or_kernel(bench):
    assert bench.measured_traffic("k_identify_queue", "er22", dict(SHAPE, scan_blocks=512)) is None
    assert bench.measured_traffic("k_identify_queue", "er22", dict(SHAPE, queue=1)) is None
    assert bench.measured_traffic("k_relax", "er22", SHAPE) is None
    assert bench.measured_traffic("k_identify_queue", "no_such_graph", SHAPE) is None


def test_algorithmic_bytes(bench):
    st = {"sum_f": 1000, "n_reach": 100, "m_reach": 1600, "improving": 50}
    assert bench.alg_bytes("identify", st, 10) == 24 * 1000 / 10
    assert bench.alg_bytes("relax", st, 10) == (16 * (100 + 1600) + 8 * 50) / 10


def test_more_than_one_gpu_is_refused():
    """bench.py measures one device; asked for several it says so and exits non-zero before it
    touches a GPU (so this runs on a machine without one)."""
    import subprocess
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr and p.stdout == ""
