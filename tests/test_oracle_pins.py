"""The oracle against the paper's running example, its printed small facts,
independent brute-force formulations and the invariants it states."""
import pytest

from tests import pins


@pytest.mark.parametrize("check", pins.ALL_CHECKS, ids=lambda f: f.__name__)
def test_oracle_pin(orc, check):
    check(orc)
