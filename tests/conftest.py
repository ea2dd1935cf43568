import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Under pytest-xdist each worker process loads its own copy of the OpenMP
# oracle; with every worker using all cores, the oracle's many short parallel
# loops (threads spin at each barrier) slow down by orders of magnitude.  Give
# each worker its share of the cores.  Read by the OpenMP runtime when the
# oracle library is first loaded, which happens after this module runs.
_workers = os.environ.get("PYTEST_XDIST_WORKER_COUNT")
if _workers:
    os.environ["OMP_NUM_THREADS"] = str(max(1, (os.cpu_count() or 1) // int(_workers)))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
