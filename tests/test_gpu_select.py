"""Device truncation rule vs the oracle's, through the C ABI (MI355X only).

The gate step keeps, per ket, the keep = min(chi, #{s^2 > tau sum s^2})
largest singular values over all quantum-number blocks (App. A1), equal
values taken in block order and then in order within a block.  The kept
counts are integers and are compared exactly with oracle.mps.select_kept on
the same values; the discarded weight and the relative gap at the cut are
sums and ratios, compared to 1e-12.  Inputs include exact ties across and
within blocks, empty blocks, all-zero kets and values below the tau cut.
"""
import numpy as np
import pytest

import paper_2404_10223_amd as T
from oracle.mps import select_kept

pytestmark = pytest.mark.gpu
TAU = 1e-13


@pytest.fixture(scope="module")
def ctx():
    c = T.Context(0)
    yield c
    c.close()


def _oracle(blocks, chi, tau):
    kept, stats = [], []
    for b in blocks:
        allsv = np.concatenate([np.asarray(x, dtype=float) for x in b]) if b else np.zeros(0)
        mask, keep, _, gap, disc, _ = select_kept(allsv, chi, tau)
        o = 0
        for x in b:
            kept.append(int(mask[o:o + len(x)].sum()))
            o += len(x)
        stats.append((keep, disc, 1.0 if gap is None else gap))
    return np.array(kept, dtype=np.int64), np.array(stats)


def _check(ctx, blocks, chi, tau=TAU):
    print(f"kets={len(blocks)} blocks={sum(len(b) for b in blocks)} chi={chi}", flush=True)
    kept, stats = ctx.debug_select(blocks, chi, tau)
    ko, so = _oracle(blocks, chi, tau)
    np.testing.assert_array_equal(kept, ko)
    np.testing.assert_array_equal(stats[:, 0], so[:, 0])
    np.testing.assert_allclose(stats[:, 1], so[:, 1], rtol=1e-12, atol=0.0)
    np.testing.assert_allclose(stats[:, 2], so[:, 2], rtol=1e-12, atol=0.0)


def test_ties_zeros_and_threshold(ctx):
    blocks = [
        [[5.0, 4.0, 4.0, 1.0], [4.0, 4.0, 3.0], [4.0, 2.0]],   # ties across and within blocks at the cut
        [[3.0, 2.0], [1.0]],                                   # chi above the number of values
        [[0.0, 0.0], [0.0]],                                   # nothing to keep
        [[1.0, 1e-7], [1e-8]],                                 # below the tau cut: only one kept
        [[], [2.0, 2.0], []],                                  # empty blocks
        [[7.0]],
    ]
    for chi in (1, 2, 5, 6, 100):
        _check(ctx, blocks, chi)


def test_random_with_frequent_ties(ctx):
    rng = np.random.default_rng(11)
    for trial in range(6):
        blocks = []
        for _ in range(int(rng.integers(1, 40))):
            ket = []
            for _ in range(int(rng.integers(0, 30))):
                n = int(rng.integers(0, 60))
                # values from a small set (many exact ties), some zeros
                x = rng.integers(0, 12, size=n).astype(float) * 0.25
                ket.append(np.sort(x)[::-1].copy())
            blocks.append(ket)
        chi = int(rng.integers(0, 300))
        _check(ctx, blocks, chi)


def test_random_spread_values(ctx):
    rng = np.random.default_rng(12)
    blocks = []
    for _ in range(120):
        ket = [np.sort(np.exp(-rng.uniform(0, 20, size=int(rng.integers(1, 170)))))[::-1].copy()
               for _ in range(int(rng.integers(1, 24)))]
        blocks.append(ket)
    _check(ctx, blocks, 256)


def test_unsorted_input_rejected(ctx):
    with pytest.raises(T.TnqeError):
        ctx.debug_select([[[1.0, 2.0]]], 1, TAU)
