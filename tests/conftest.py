import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built libkc.so")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def kc():
    """The GPU binding; GPU tests fail loudly (not skip) when the library is missing."""
    import paper_2104_13209_amd as kcmod
    kcmod.lib()
    return kcmod


def load_counts(name):
    """A stored count fixture under tests/golden/: ({header: int}, {k: c_k}, {k: nodes})."""
    head, counts, nodes = {}, {}, {}
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "c":
                counts[int(parts[1])] = int(parts[2])
            elif parts[0] == "nodes":
                nodes[int(parts[1])] = int(parts[2])
            else:
                head[parts[0]] = int(parts[1])
    return head, counts, nodes
