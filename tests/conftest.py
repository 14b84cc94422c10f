import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running (minutes of CPU oracle work)")


@pytest.fixture(scope="session")
def oracle_mod():
    # DCEM_ORACLE_PY names a planted-mistake copy of oracle.py (see
    # test_oracle_mutations.py); otherwise the real oracle
    alt = os.environ.get("DCEM_ORACLE_PY")
    if alt:
        import importlib.util
        spec = importlib.util.spec_from_file_location("oracle_mutant", alt)
        mod = importlib.util.module_from_spec(spec)
        sys.modules["oracle_mutant"] = mod   # dataclasses resolve their module by name
        spec.loader.exec_module(mod)
        return mod
    from oracle import oracle
    oracle.build()
    return oracle
