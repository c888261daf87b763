"""Pins of the oracle's identical-particle ordering (CPU).

Two identical particles (the two pi- of Lambda_b -> p pi- pi+ pi-) are told
apart by their energy in the M rest frame: the faster goes to the channel's
first slot.  Swapping them flips the sign of C_T, so the order is part of the
definition.  The pins: a hand event whose class flips under the ordering, the
same event boosted, the negation of C_T under the swap (momentum conservation
in the rest frame), independence of the stored order, agreement with the
generator's own float64 ordering, exact brute force, and exact ties.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_1612_04705_amd import synth

CH = synth.CHANNELS["Lb_ppipipi"]          # p, pi-(fast), pi+, pi-(slow)
IDENT = (1, 3)


def _sample(rows, dtype=np.float64):
    n = len(rows)
    comps = np.zeros((4, 4, n), dtype=dtype)
    for i, r in enumerate(rows):
        comps[:, :, i] = np.asarray(r, dtype=np.float64).reshape(4, 4)
    return comps, np.zeros(n, dtype=np.int8)


def _boost_x(rows, gamma):
    beta = math.sqrt(1.0 - 1.0 / (gamma * gamma))
    out = []
    for E, px, py, pz in rows:
        out.append([gamma * (E + beta * px), gamma * (px + beta * E), py, pz])
    return out


# M at rest: the rest-frame energies are the stored ones.  Slot 1 holds E = 2,
# slot 3 E = 3, so the ordering exchanges them.  C_T = p0 . (p1 x p2):
# stored order (1,0,0).((0,1,0)x(0,0,1)) = +1 -> class I; ordered
# (1,0,0).((-1,-1,-1)x(0,0,1)) = (1,0,0).(-1,1,0) = -1 -> class II.
HAND = [[5.0, 1.0, 0.0, 0.0], [2.0, 0.0, 1.0, 0.0], [5.0, 0.0, 0.0, 1.0], [3.0, -1.0, -1.0, -1.0]]


@pytest.mark.parametrize("gamma", [None, 3.0, 40.0])
def test_hand_event_class_flips(gamma):
    rows = HAND if gamma is None else _boost_x(HAND, gamma)
    comps, tag = _sample([rows])
    plain = oracle.run(comps, tag, CH.triple, CH.planes, want_events=True)
    ordered = oracle.run(comps, tag, CH.triple, CH.planes, want_events=True, identical=IDENT)
    assert int(plain["cls"][0]) == exact.CLS_I
    assert int(ordered["cls"][0]) == exact.CLS_II
    # the exact resolver takes the same decision
    assert exact.exact_decision(rows, 0, CH.triple, CH.planes, [], IDENT)[0] == exact.CLS_II
    # already ordered input is left alone
    assert exact.order_identical(exact.order_identical(rows, IDENT), IDENT) == exact.order_identical(rows, IDENT)


def _swap13(comps, mask):
    c = comps.copy()
    c[1][:, mask], c[3][:, mask] = comps[3][:, mask], comps[1][:, mask]
    return c


@pytest.fixture(scope="module")
def lb():
    s = synth.generate(CH, 20000, 31, inj=synth.INJ_SIN)
    comps, tag = s.numpy()
    mask = np.random.default_rng(3).uniform(size=tag.shape[0]) < 0.5
    return comps, tag, mask


def test_swap_negates_ct(lb):
    # rest frame: p3 = -(p0 + p1 + p2), so p0.(p3 x p2) = -p0.(p1 x p2)
    comps, tag, mask = lb
    a = oracle.run(comps, tag, CH.triple, CH.planes, want_events=True)
    b = oracle.run(_swap13(comps, np.ones_like(mask)), tag, CH.triple, CH.planes, want_events=True)
    # the float64 rest-frame C_T carries ~u (1 + gamma^2) (p*)^3 of rounding;
    # p* < 3 GeV here, so (p*)^3 < 3e10 MeV^3
    x = comps.astype(np.float64)
    P = x.sum(axis=0)
    g2 = 1.0 + P[0] ** 2 / (P[0] ** 2 - P[1] ** 2 - P[2] ** 2 - P[3] ** 2)
    tol = 1e-12 * np.abs(a["ct"]) + 64 * 2.0 ** -53 * g2 * 3e10
    assert np.all(np.abs(a["ct"] + b["ct"]) <= tol)


def test_stored_order_does_not_matter(lb):
    comps, tag, mask = lb
    axes = [synth.absphi_axis(12), synth.mass_axis((0, 3), 1000.0, 5200.0, 8)]
    a = oracle.run(comps, tag, CH.triple, CH.planes, axes, identical=IDENT)
    b = oracle.run(_swap13(comps, mask), tag, CH.triple, CH.planes, axes, identical=IDENT)
    assert a["counts"] == b["counts"] and a["stats"] == b["stats"]
    # and it differs from taking the shuffled order as is
    c = oracle.run(_swap13(comps, mask), tag, CH.triple, CH.planes, axes)
    assert c["counts"] != a["counts"]


def test_agrees_with_generator_order(lb):
    # the generator ordered in float64 before the boost and storage: any event
    # the oracle reorders must be a near-tie of the rest-frame energies
    comps, tag, _ = lb
    plain = oracle.run(comps, tag, CH.triple, CH.planes, want_events=True)
    ordered = oracle.run(comps, tag, CH.triple, CH.planes, want_events=True, identical=IDENT)
    x = comps.astype(np.float64)
    P = x.sum(axis=0)
    M = np.sqrt(P[0] ** 2 - P[1] ** 2 - P[2] ** 2 - P[3] ** 2)
    Estar = [(P[0] * x[s][0] - P[1] * x[s][1] - P[2] * x[s][2] - P[3] * x[s][3]) / M for s in range(4)]
    differ = plain["cls"] != ordered["cls"]
    rel = np.abs(Estar[1] - Estar[3]) / (Estar[1] + Estar[3])
    assert np.all(rel[differ] < 1e-5)
    assert differ.sum() <= 3


def test_brute_force_matches(lb):
    comps, tag, mask = lb
    k = 1500
    c = _swap13(comps, mask)[:, :, :k].copy()
    axes = [synth.abscos_axis(1, 5)]
    want = oracle.brute_force(c, tag[:k], CH.triple, CH.planes, axes, identical=IDENT)
    got = oracle.run(c, tag[:k], CH.triple, CH.planes, axes, identical=IDENT)
    assert got["counts"] == want["counts"]


def tie_events(n, seed):
    """Events exactly at rest with E_1 == E_3 and |p_1| == |p_3| (p_3 a
    permutation of p_1's components): an exact tie of the rest-frame energies.
    Small integers, so every stored value and every sum is exact."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(n):
        a, b, c = (int(v) for v in rng.integers(-9, 10, size=3))
        u, v, w = (int(t) for t in rng.integers(-9, 10, size=3))
        E1 = 20 + int(rng.integers(0, 5))
        p1 = [E1, a, b, c]
        p3 = [E1, b, c, a]
        p0 = [30 + int(rng.integers(0, 5)), u, v, w]
        p2 = [30 + int(rng.integers(0, 5)), -(a + b) - u, -(b + c) - v, -(c + a) - w]
        rows.append([p0, p1, p2, p3])
    return rows


def test_exact_tie_keeps_stored_order():
    rows = tie_events(300, 5)
    comps, tag = _sample(rows, np.float32)
    a = oracle.run(comps, tag, CH.triple, CH.planes, want_events=True)
    b = oracle.run(comps, tag, CH.triple, CH.planes, want_events=True, identical=IDENT)
    assert b["n_flagged"] == len(rows)              # every one is a tie for the float64 pass
    assert np.array_equal(a["cls"], b["cls"])
    for r in rows[:20]:
        assert exact.order_identical(r, IDENT) == r
