"""The CPU oracle against the hand-written closed-form fixtures of tests/golden/: brute
force over all features and through the oracle's own grid at two cell sizes."""
import pytest

import oracle
from tests import golden_cases, pins


@pytest.mark.parametrize("name", golden_cases.ALL)
@pytest.mark.parametrize("cs", [None, 1.0, 2.5])
def test_oracle_matches_golden(name, cs):
    pins.check_golden(oracle.load(), name, cs)
