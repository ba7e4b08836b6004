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


# Full-size graphs (500M and 1B triples) take minutes to draw.  Graph
# generation forks worker processes only while this process holds no GPU
# state, so when tests that need them are selected they are drawn here,
# after collection and before the first test initialises the GPU.
_FULL_SIZE = {"test_gpu_large": "large", "test_gpu_serving_size": "serving"}


def pytest_collection_finish(session):
    want = []
    for item in session.items:
        name = _FULL_SIZE.get(item.module.__name__.rsplit(".", 1)[-1])
        if name and name not in want:
            want.append(name)
    if not want:
        return
    try:
        import torch
        if torch.cuda.device_count() == 0:   # counts devices without initialising one
            return
    except Exception:  # noqa: BLE001
        return
    import time
    from synth import CONFIGS, make_graph
    for name in want:
        t0 = time.time()
        _GRAPHS[(name, None)] = make_graph(CONFIGS[name])
        print(f"\n[conftest] drew the {name} graph ({CONFIGS[name].n} triples) in "
              f"{time.time() - t0:.0f}s", flush=True)
