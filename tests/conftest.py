import os
import sys

# Small dense LAPACK calls in the oracle pins are slowed down badly by spinning BLAS threads
# when the host is shared; a handful of threads is plenty for the matrix sizes used here.
os.environ.setdefault("OPENBLAS_NUM_THREADS", "4")
os.environ.setdefault("OMP_NUM_THREADS", "4")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

try:
    from threadpoolctl import threadpool_limits

    threadpool_limits(limits=4)
except Exception:  # pragma: no cover - threadpoolctl is optional
    pass


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~10 s")
