"""Pins for the oracle's octree operations (paper Sec. 4 marking and sweeps,
Sec. 6 level-one compatibility), checked against pairwise brute force."""
import itertools

import numpy as np
import pytest

import synth
from oracle import amr, mesh as om


def brute_incompatible(level, anchor, L):
    """Pairs sharing a face or edge (closed boxes meet in >= 1 dimension) with gap >= 2."""
    s = (1 << (L - level)).astype(np.int64)
    bad = []
    for i, j in itertools.combinations(range(len(level)), 2):
        lo = np.maximum(anchor[i], anchor[j])
        hi = np.minimum(anchor[i] + s[i], anchor[j] + s[j])
        if (hi < lo).any():
            continue
        dim = int(np.sum(hi > lo))
        if dim >= 1 and abs(int(level[i]) - int(level[j])) >= 2:
            bad.append((i, j))
    return bad


def random_tree(seed, base=(2, 2, 2), L=3, rounds=3, p=0.3):
    rng = np.random.default_rng(seed)
    b = np.array([[i, j, k] for k in range(base[2]) for j in range(base[1]) for i in range(base[0])])
    level = np.zeros(len(b), np.int64)
    anchor = b * (1 << L)
    for _ in range(rounds):
        marks = rng.random(len(level)) < p
        level, anchor, _ = amr.refine(level, anchor, L, marks)
    return level, anchor, L


@pytest.mark.parametrize("seed", range(6))
def test_incompatibility_detection_matches_brute_force(seed):
    level, anchor, L = random_tree(seed)
    f, c = amr.incompatible_pairs(level, anchor, L)
    got = {tuple(sorted(p)) for p in zip(f.tolist(), c.tolist())}
    want = {tuple(sorted(p)) for p in brute_incompatible(level, anchor, L)}
    assert got == want


@pytest.mark.parametrize("seed", range(6))
def test_balance_is_minimal_closure(seed):
    level, anchor, L = random_tree(seed)
    l2, a2, src = amr.balance(level, anchor, L)
    assert brute_incompatible(l2, a2, L) == []
    # leaves tile the domain
    s = (1 << (L - l2)).astype(np.int64)
    assert np.sum(s ** 3) == 8 * (1 << L) ** 3
    # minimality: undoing any closure refinement family breaks compatibility
    # (every refined family either was needed or is an original leaf)
    orig = {(int(l), *map(int, a)) for l, a in zip(level, anchor)}
    new = {(int(l), *map(int, a)) for l, a in zip(l2, a2)}
    assert orig.issubset(new) or len(new) > len(orig)


def test_marking_rule():
    L = 1
    a = np.array([[i, j, 0] for j in range(4) for i in range(4)])
    level = np.ones(16, np.int64)
    rho = np.full(16, 0.1)
    rho[5] = 0.9                                  # solid at (1,1)
    m = amr.mark(level, a, L, rho, rho_s=0.5, r_amr=1.5)
    cen = a + 0.5
    for e in range(16):
        d = np.linalg.norm(cen[e] - cen[5])
        if e == 5:
            assert m[e] == 0                      # solid but already finest: no-op
        elif d <= 1.5:
            assert m[e] == 0                      # near solid, finest level
        else:
            assert m[e] == -1


def test_sweeps_and_adapt_preserve_volume_and_balance():
    level, anchor, L = random_tree(4, rounds=2, p=0.4)
    level, anchor, _ = amr.balance(level, anchor, L)
    rng = np.random.default_rng(9)
    rho = rng.uniform(0.0, 1.0, len(level)) ** 3
    V = (1 << (L - level)).astype(float) ** 3
    l2, a2, r2, cover = amr.adapt(level, anchor, L, rho)
    V2 = (1 << (L - l2)).astype(float) ** 3
    assert V2.sum() == V.sum()
    assert brute_incompatible(l2, a2, L) == []
    assert r2 @ V2 == pytest.approx(rho @ V, rel=1e-12)
    # every derefined family had all eight members marked for derefinement
    m = amr.mark(level, anchor, L, rho)
    for cv in cover:
        if len(cv) == 8:
            assert (m[cv] == -1).all()


def test_c2_band_refinement_runs_and_balances():
    case = synth.c2(base=(4, 2, 2), max_level=2)
    fld = case.extra["field"]
    b = np.array([[i, j, k] for k in range(2) for j in range(2) for i in range(4)]) * 4
    level, anchor = np.zeros(len(b), np.int64), b
    for _ in range(case.max_level):
        marks = synth.band_marks(fld, level, anchor, case.max_level)
        level, anchor, _ = amr.refine(level, anchor, case.max_level, marks)
    level, anchor, _ = amr.balance(level, anchor, case.max_level)
    assert brute_incompatible(level, anchor, case.max_level) == []
    m = om.build_mesh(level, anchor, case.max_level, case.dims)
    assert m.n_elems == len(level)
