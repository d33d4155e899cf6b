import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)


# MPC_ORACLE_LIB names another build of the oracle for the whole session (the
# sanitizer test runs the pins against an ASan/UBSan build this way)
if os.environ.get("MPC_ORACLE_LIB"):
    import oracle

    oracle.use_library(os.environ["MPC_ORACLE_LIB"])


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: longer CPU test")
