import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    oracle.build(force=False)
    yield


# GPU modules run core parity first; the autotuner (which times dozens of
# candidate launches) runs after everything that checks results.
_MODULE_ORDER = {"test_gpu_parity.py": 1, "test_gpu_options.py": 2, "test_gpu_shapes.py": 2, "test_gpu_adjoint.py": 3, "test_gpu_replan.py": 3, "test_gpu_drift.py": 3,
                 "test_gpu_periodic.py": 3,
                 "test_gpu_batch.py": 4, "test_gpu_graph.py": 4, "test_gpu_pm.py": 5, "test_gpu_workloads.py": 5,
                 "test_gpu_autotune.py": 6}


def pytest_collection_modifyitems(config, items):
    def rank(item):
        name = os.path.basename(str(item.fspath))
        return 9 if name.startswith("test_zz") else _MODULE_ORDER.get(name, 0)
    items.sort(key=rank)
