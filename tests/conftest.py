import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


@pytest.fixture(scope="session")
def tiny_kg():
    import kggen
    return kggen.named_graph("tiny")


@pytest.fixture(scope="session")
def medium_kg():
    import kggen
    return kggen.named_graph("medium")


@pytest.fixture(scope="session")
def oracle_tiny(tiny_kg):
    import oracle
    return oracle.graph_from_kg(tiny_kg)


@pytest.fixture(scope="session")
def oracle_medium(medium_kg):
    import oracle
    return oracle.graph_from_kg(medium_kg)
