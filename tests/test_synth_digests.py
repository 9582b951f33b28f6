"""The seeded synthetic inputs are the same arrays the stored oracle values
were computed from: SHA-256 digests of every generated array against
tests/golden/digests.json (written by tests/golden/make_golden.py)."""
import json
import os

import pytest

import tnqe_synth as synth

DIG = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "digests.json")))


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_config_digests(k):
    assert synth.problem_digest(synth.make_config(k)) == DIG[f"config{k}"]


@pytest.mark.parametrize("rot", ["perm", "identity"])
@pytest.mark.parametrize("k", [2, 3])
def test_variant_digests(k, rot):
    p = synth.make_config(k, rot)
    assert synth.problem_digest(p) == DIG[p.name]


def test_batch_digests():
    got = [synth.problem_digest(p) for p in synth.make_batch()[:8]]
    assert got == DIG["batch"]
