"""The packed (BFV / RLWE) CPU oracle against its pins (no GPU)."""
import pytest

from oracle import bfv
from tests import pins_bfv


@pytest.fixture(scope="module")
def orc():
    o = bfv.default()
    o.set_threads(8)
    return o


@pytest.mark.parametrize("check", pins_bfv.ALL_CHECKS, ids=lambda c: c.__name__)
def test_pin(orc, check):
    check(orc)
