"""The oracle reproduces its committed golden fixture (tests/golden/make_golden.py)."""
import json
import os

from golden.make_golden import HERE, compute


def test_tiny_oracle_golden():
    with open(os.path.join(HERE, "tiny_oracle.json")) as f:
        want = json.load(f)
    assert compute() == want
