"""The driver's smoke entry point runs and agrees with the oracle."""
import pytest

pytestmark = pytest.mark.gpu


def test_smoke_entry_point(gpu):
    import __graft_entry__
    __graft_entry__.smoke()
