import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU statistics test")


@pytest.fixture(scope="session")
def rootdir():
    return ROOT


@pytest.fixture(autouse=True)
def _nan_buffers(request, monkeypatch):
    """GPU tests: every workspace and linear-term state the binding hands to the library
    starts as NaN bytes (0xff), so a kernel that reads memory no kernel of the call wrote
    gives a non-finite result instead of silently using whatever a previous test left."""
    if request.node.get_closest_marker("gpu") is None:
        yield
        return
    try:
        import torch
        from paper_1105_2791_amd import api
    except Exception:
        yield
        return
    if not torch.cuda.is_available():
        yield
        return
    ws0, st0 = api.ModalContext.workspace, api.ModalContext.linear_state

    def workspace(self, op, S):
        t = ws0(self, op, S)
        if not torch.cuda.is_current_stream_capturing():
            t.fill_(255)
        return t

    def linear_state(self):
        t = st0(self)
        t.fill_(255)
        return t

    monkeypatch.setattr(api.ModalContext, "workspace", workspace)
    monkeypatch.setattr(api.ModalContext, "linear_state", linear_state)
    yield
