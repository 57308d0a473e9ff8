"""The smoke entry point runs on the GPU (one small tracking pass checked
bit for bit against the oracle, one refit and adjoint within tolerance)."""
import pytest

import __graft_entry__


@pytest.mark.gpu
def test_smoke_entry_point():
    __graft_entry__.smoke()
