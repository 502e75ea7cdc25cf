"""Host logic of bench.py (no GPU): the code hash that ties a traffic record to its kernel source,
the traffic figure's scaling and its null rule, the algorithmic work behind each roofline figure,
and the refusal of more than one GPU."""
import importlib.util
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)            # defines functions only; main() runs under __main__
    return mod


def test_code_hash_ignores_comments_only(bench, tmp_path):
    a = tmp_path / "k.hip"
    a.write_text("__global__ void k(float* x) {\n  x[0] = 1.0f;   // store\n}\n")
    h0 = bench.code_hash(str(a))
    a.write_text("// a kernel\n__global__ void k(float* x) {\n\n  x[0] = 1.0f;   // one store   \n}\n")
    assert bench.code_hash(str(a)) == h0
    a.write_text("__global__ void k(float* x) {\n  x[0] = 2.0f;\n}\n")
    assert bench.code_hash(str(a)) != h0


def test_code_hash_of_one_kernel(bench, tmp_path):
    """With a kernel name the hash covers that kernel's definition only: editing another kernel of
    the same file keeps it, editing this one changes it."""
    a = tmp_path / "k.hip"
    a.write_text("__global__ void k(float* x) {\n  x[0] = 1.0f;\n}\n\n__global__ void k2(float* x) {\n  x[1] = 0;\n}\n")
    h0 = bench.code_hash(str(a), "k")
    a.write_text("__global__ void k(float* x) {\n  x[0] = 1.0f;   // store\n}\n\n__global__ void k2(float* x) {\n"
                 "  x[1] = 5;\n}\n")
    assert bench.code_hash(str(a), "k") == h0
    a.write_text("__global__ void k(float* x) {\n  x[0] = 3.0f;\n}\n\n__global__ void k2(float* x) {\n  x[1] = 5;\n}\n")
    assert bench.code_hash(str(a), "k") != h0


def test_traffic_scaling_and_null_rule(bench, tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("__global__ void k() {}\n")
    rel = os.path.relpath(str(src), bench.ROOT)
    rec = {"src": rel, "sha": bench.code_hash(str(src)), "kib": [("k", 100.0, 50.0), ("k2", 10.0, 0.0)]}
    monkeypatch.setitem(bench.TRAFFIC, "phase_x", rec)
    want = ((100.0 + 10.0) * bench.FETCH_SCALE + 50.0 * bench.WRITE_SCALE) * 1024.0
    assert bench.traffic_bytes("phase_x", 1, 16) == pytest.approx(want)
    assert bench.traffic_bytes("phase_x", 2, 16) is None          # measured for one right-hand side
    assert bench.traffic_bytes("no_such_phase", 1, 16) is None
    src.write_text("__global__ void k() { }\n__global__ void k2() {}\n")   # the kernel source changed
    assert bench.traffic_bytes("phase_x", 1, 16) is None


def test_algorithmic_work(bench):
    st = SimpleNamespace(near_pairs=1000, fmm_m2l_pairs=43488, fmm_boxes=977, fmm_p2p_pairs=494612056)
    N, q, p = 153600, 10, 6
    v, unit, bound, peak = bench.algorithmic_work("fmm_m2l", st, N, q, 1, p)
    assert (unit, bound, peak) == ("TFLOP/s", "mfma", 157.3)
    assert v == pytest.approx(2 * 9 * 6 ** 6 * 43488 / 1e12)       # 3.65e10 flop per launch
    v, unit, bound, _ = bench.algorithmic_work("fmm_p2p", st, N, q, 1, p)
    assert (unit, bound) == ("TFLOP/s", "alu") and v == pytest.approx(494612056 * 26 / 1e12)
    v, unit, bound, peak = bench.algorithmic_work("direct64", st, N, q, 16, p)
    assert (bound, peak) == ("alu", 78.6) and v == pytest.approx(N * N * (24 + 32) / 1e12)
    v, unit, bound, peak = bench.algorithmic_work("near", st, N, q, 1, p, path="mixed")
    assert (unit, bound, peak) == ("GB/s", "hbm", 8000.0)
    assert v == pytest.approx((8.0 * 1000 * q * q + 8.0 * N * 2 + 8.0 * (N + 1) + 4.0 * 1000) / 1e9)
    v64, *_ = bench.algorithmic_work("near", st, N, q, 1, p, path="fp64")
    assert v64 == pytest.approx(v + 8.0 * N / 1e9)                 # the FP64 path's far partials
    assert bench.algorithmic_work("fmm_l2l", st, N, q, 1, p) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
