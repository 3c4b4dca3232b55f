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


def test_packed_sets_match_the_golden_file():
    """The package's parameter sets are the ones the oracle's script wrote."""
    from paper_2003_05328_amd import configs

    gold = bfv.table2_params()
    assert set(gold) == set(configs.PACKED_SETS)
    for k, pr in gold.items():
        assert configs.PACKED_SETS[k] == dict(t=pr.t, q0=pr.q0, q1=pr.q1, n=pr.n)
