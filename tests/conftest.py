import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large-size case")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def ctx():
    """One library context on cuda:0 for the GPU tests (native pool allocator)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1807_01409_amd import Context
    c = Context(0)
    yield c
    c.close()


_GRAPHS = {}


@pytest.fixture(scope="session")
def graphs():
    """Memoised synthetic graphs by (config name, n)."""
    from synth import CONFIGS, make_graph

    def get(name, n=None):
        key = (name, n)
        if key not in _GRAPHS:
            spec = CONFIGS[name] if n is None else CONFIGS[name].with_n(n)
            _GRAPHS[key] = make_graph(spec)
        return _GRAPHS[key]
    return get
