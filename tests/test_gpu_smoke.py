"""The round-end smoke invocation (one small FP64 batch on cuda:0 against the
oracle) run as a test, so a change to the binding it calls is caught here."""
import pytest


@pytest.mark.gpu
def test_smoke_runs():
    import __graft_entry__

    __graft_entry__.smoke()
