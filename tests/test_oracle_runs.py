"""Pins of the oracle's label runs (the stable partition of session indices
by label): hand-worked fixtures, numpy's stable sort by the two label bits,
and the four properties that determine the partition uniquely."""
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "label_runs_examples.txt")


def _cases():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        a, b, c = (x.strip() for x in line.split("|"))
        lab = np.array([] if a == "-" else [int(v) for v in a.split()], np.uint8)
        idx = np.array([] if b == "-" else [int(v) for v in b.split()], np.uint32)
        tot = np.array([int(v) for v in c.split()], np.uint64)
        out.append((lab, idx, tot))
    return out


@pytest.mark.parametrize("case", range(len(_cases())))
def test_hand_examples(case):
    lab, idx, tot = _cases()[case]
    got_idx, got_tot = oracle.label_runs(lab)
    assert np.array_equal(got_idx, idx) and np.array_equal(got_tot, tot)


@pytest.mark.parametrize("n,seed", [(0, 0), (1, 1), (1000, 2), (65_537, 3), (200_003, 4)])
def test_unique_properties_and_stable_sort(n, seed):
    """A permutation of 0..n-1, labels non-decreasing along it, indices
    increasing within a label, totals = the label counts: only the stable
    partition has all four; it equals numpy's stable argsort of label & 3."""
    rng = np.random.default_rng(seed)
    lab = rng.integers(0, 256, n).astype(np.uint8)
    idx, tot = oracle.label_runs(lab)
    key = (lab & 3).astype(np.int64)
    assert np.array_equal(np.sort(idx), np.arange(n, dtype=np.uint32))
    k = key[idx]
    assert np.all(np.diff(k) >= 0)
    same = np.diff(k) == 0
    assert np.all(np.diff(idx.astype(np.int64))[same] > 0)
    assert np.array_equal(tot, np.bincount(key, minlength=4).astype(np.uint64))
    assert np.array_equal(idx, np.argsort(key, kind="stable").astype(np.uint32))


def test_planted_mistake_fails():
    """Swapping two indices of one run breaks the in-run order property (the
    check above is not vacuous)."""
    lab = np.array([1, 1, 0, 1], np.uint8)
    idx, _ = oracle.label_runs(lab)
    bad = idx.copy()
    bad[1], bad[2] = bad[2], bad[1]
    k = (lab & 3)[bad]
    assert np.all(np.diff(k.astype(np.int64)) >= 0)
    assert not np.all(np.diff(bad.astype(np.int64))[np.diff(k.astype(np.int64)) == 0] > 0)
