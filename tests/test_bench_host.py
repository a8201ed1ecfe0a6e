"""Host-side pieces of bench.py, no GPU: the one-GPU guard and the algorithmic byte counts behind
the operator roofline (per pass: complex128 input and output vectors, compute-precision
intermediates, 4-byte packed material ids in the CrossDoF stencil pass, and the complex128 K.x
per point that the first x-pass hands to the last)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and r.stdout == ""
    assert "single MI355X" in r.stderr


def test_pass_bytes_of_one_application():
    b = _bench()
    N, nvec = 128, 16
    n3 = N ** 3
    for cross, npass in ((True, 6), (False, 5)):
        for s in (8, 16):  # FP32 / FP64 intermediates
            names, by = b.pass_bytes(N, nvec, cross, s)
            assert len(names) == len(by) == npass
            # every intermediate is written by one pass and read by the next; x is read once by
            # the first pass, y written once by the last, K.x written by the first and read by
            # the last, the ids read once by the pass that applies the permittivity
            inter = (npass - 1) * 2 * s * 3 * n3 * nvec
            expect = inter + 2 * 16 * 3 * n3 * nvec + 2 * 16 * n3 * nvec + 4 * n3 * nvec
            assert sum(by) == expect, (cross, s, sum(by), expect)
    # the bench's FP32 CrossDoF figure on 16 vectors at 128^3, and the boundary's own bytes per
    # band (read x, write y, read the ids): 210 MB
    assert sum(b.pass_bytes(128, 16, True, 8)[1]) == 12482248704
    assert 2 * 16 * 3 * n3 + 4 * n3 == 209715200
