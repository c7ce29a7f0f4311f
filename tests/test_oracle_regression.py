"""The oracle still reproduces its own stored results bit for bit (tests/golden).

These values pin nothing about the method -- the closed forms, invariants and brute
force do that -- they make any change to the oracle's arithmetic visible."""
import json
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _stored():
    with open(os.path.join(GOLDEN, "oracle_regression.json")) as f:
        return json.load(f)


def _fresh():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_oracle_regression", os.path.join(GOLDEN, "make_oracle_regression.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return dict(mod.cases())


@pytest.fixture(scope="module")
def fresh(orc):
    return _fresh()


@pytest.mark.parametrize("name", sorted(_stored()))
def test_oracle_reproduces_stored_result(fresh, name):
    assert fresh[name] == _stored()[name]
