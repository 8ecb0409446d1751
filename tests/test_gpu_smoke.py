"""The repository's smoke entry point runs as a GPU test too (needs an
MI355X): one small decomposition through the library, checked against the
oracle."""
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def test_smoke_entry_point(gpu_lib):
    import __graft_entry__ as entry
    entry.smoke()
