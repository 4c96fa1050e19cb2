"""The oracle still produces its stored regression outputs (written by
tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

from tests.golden.make_golden import OUT, build


def test_oracle_matches_stored_regression(orc):
    with open(OUT) as f:
        stored = json.load(f)
    assert build() == stored
