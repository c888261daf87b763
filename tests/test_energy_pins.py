"""Pins of the energy-test oracle (CPU): hand-computed values, closed forms and
brute force, each chosen so that a dropped term, a wrong normalisation or a
wrong coefficient fails one of them."""
import math

import numpy as np
import pytest

from oracle import energy
from paper_1612_04705_amd import synth


def test_hand_example_eq2():
    # 1-D: X = {0, 2}, Xbar = {1, 3}, sigma = 1: psi(d) = exp(-d^2/2)
    Y = np.array([[0.0, 2.0, 1.0, 3.0]])
    lab = np.array([1, 1, 0, 0])
    want = math.exp(-2.0) / 2 + math.exp(-2.0) / 2 - (3 * math.exp(-0.5) + math.exp(-4.5)) / 4
    assert energy.T_eq2(Y, lab, 1.0) == pytest.approx(want, rel=1e-15, abs=1e-16)


def test_sigma_infinite_gives_zero_eq2_and_eq3():
    rng = np.random.default_rng(1)
    Y = rng.uniform(0, 1, size=(3, 57))
    lab = rng.integers(0, 2, size=57)
    assert abs(energy.T_eq2(Y, lab, 1e9)) < 1e-14
    # eq. (3): every psi = 1 makes each bracket w(w-1), w(w-1), w*wbar exactly,
    # which needs the b(b+1) coefficient of the background-background term
    main, mainb = rng.uniform(size=(3, 40)), rng.uniform(size=(3, 33))
    bkg, bkgb = rng.uniform(size=(3, 25)), rng.uniform(size=(3, 19))
    assert abs(energy.T_eq3(main, mainb, bkg, bkgb, 7, 5, 1e9)) < 1e-13


def test_identical_samples_closed_form():
    # Xbar a copy of X: T = 2 S / (n^2 (n-1)) - 1/n with S = sum_{i<j} psi over X
    Y = np.array([[0.0, 1.0, 0.5, 2.0]])
    X = Y.copy()
    Yall = np.concatenate([X, X], axis=1)
    lab = np.array([1] * 4 + [0] * 4)
    n = 4
    S = sum(math.exp(-(Y[0, i] - Y[0, j]) ** 2 / 2) for i in range(n) for j in range(i + 1, n))
    assert energy.T_eq2(Yall, lab, 1.0) == pytest.approx(2 * S / (n * n * (n - 1)) - 1 / n, rel=1e-14)


def test_swap_samples_symmetric():
    rng = np.random.default_rng(2)
    Y = rng.normal(size=(5, 80))
    lab = rng.integers(0, 2, size=80)
    assert energy.T_eq2(Y, lab, 0.7) == pytest.approx(energy.T_eq2(Y, 1 - lab, 0.7), rel=1e-13)


def test_eq3_without_background_is_eq2():
    rng = np.random.default_rng(3)
    main, mainb = rng.normal(size=(2, 30)), rng.normal(size=(2, 26))
    bkg, bkgb = rng.normal(size=(2, 11)), rng.normal(size=(2, 9))
    Y = np.concatenate([main, mainb], axis=1)
    lab = np.array([1] * 30 + [0] * 26)
    assert energy.T_eq3(main, mainb, bkg, bkgb, 0, 0, 0.8) == pytest.approx(energy.T_eq2(Y, lab, 0.8), rel=1e-13)


def test_brute_force_pairs():
    rng = np.random.default_rng(4)
    Y = rng.normal(size=(3, 23))
    lab = rng.integers(0, 2, size=23)
    s = 0.6
    psi = lambda i, j: math.exp(-sum((Y[k, i] - Y[k, j]) ** 2 for k in range(3)) / (2 * s * s))
    X = [i for i in range(23) if lab[i]]
    B = [i for i in range(23) if not lab[i]]
    sxx = sum(psi(X[a], X[b]) for a in range(len(X)) for b in range(a + 1, len(X)))
    sbb = sum(psi(B[a], B[b]) for a in range(len(B)) for b in range(a + 1, len(B)))
    sxb = sum(psi(i, j) for i in X for j in B)
    n, nb = len(X), len(B)
    want = sxx / (n * (n - 1)) + sbb / (nb * (nb - 1)) - sxb / (n * nb)
    assert energy.T_eq2(Y, lab, s) == pytest.approx(want, rel=1e-13)
    # blocked sums agree with one block
    assert energy.pair_sum(Y, Y, s, True, block=5) == pytest.approx(energy.pair_sum(Y, Y, s, True), rel=1e-14)


def test_p_value_counts_strictly_greater():
    assert energy.p_value(0.5, [0.1, 0.5, 0.7, 0.9]) == 0.5
    assert energy.p_value(1.0, [0.1, 0.2]) == 0.0


def test_invariant_masses_match_generated_pairs():
    ch = synth.CHANNELS["D0_KKpipi"]
    s = synth.generate(ch, 500, 9)
    comps, _ = s.numpy()
    m = energy.invariant_masses(comps, [0b0011, 0b1100])
    # generated in float64, stored in float32: each stored component is off by at
    # most 2^-24 of itself, so |m^2 - m_gen^2| <= 2 W (2^-24 W) + O(2^-48), with W the
    # L1 norm of the pair's components; the mass error is that over (m + m_gen)
    for k, (sl, ref) in enumerate((((0, 1), s.m12.numpy()), ((2, 3), s.m34.numpy()))):
        W = np.abs(comps[list(sl)].astype(np.float64)).sum(axis=(0, 1))
        tol = 2.0 * W * W * 2.0 ** -24 * 1.01 / (m[k] + ref)
        assert np.all(np.abs(m[k] - ref) <= tol)


def test_invariant_mass_hand_event():
    # two photons back to back, 1 GeV each: m = 2 GeV; one particle alone: m = 0
    comps = np.zeros((4, 4, 1))
    comps[0, :, 0] = [1.0, 0.0, 0.0, 1.0]
    comps[1, :, 0] = [1.0, 0.0, 0.0, -1.0]
    m = energy.invariant_masses(comps, [0b0011, 0b0001])
    assert m[0, 0] == 2.0 and m[1, 0] == 0.0


# ---- D0 -> pi+ pi- pi+ pi- labelling (Sect. 4.2): the pi+ pi- pair of largest
# invariant mass becomes pi3 pi4
D4PI_MASKS = [0b0011, 0b1001, 0b0110, 0b0111, 0b1011]     # m12, m14, m23, m123, m124 (Table 1)


def test_d4pi_hand_event():
    # at rest: pi+_0 = (5, 1, 0, 0), pi-_1 = (5, -1, 0, 0), pi+_2 = (4, 0, 1, 0), pi-_3 = (4, 0, -1, 0)
    # pair masses^2: (0,1) 100, (2,3) 64, (0,3) = (9, 1, -1, 0) -> 79, (2,1) -> 79;
    # the largest, (0,1), becomes pi3 pi4: new order (2, 3, 0, 1), so
    # m12^2 = 64, m14^2 = m23^2 = 79, m123^2 = m124^2 = 13^2 - 1 = 168
    comps = np.array([[5, 1, 0, 0], [5, -1, 0, 0], [4, 0, 1, 0], [4, 0, -1, 0]], dtype=np.float64).reshape(4, 4, 1)
    assert list(energy.d4pi_perm(comps)) == [1]
    m2 = energy.invariant_masses(comps, D4PI_MASKS, relabel="d4pi")[:, 0] ** 2
    assert np.allclose(m2, [64, 79, 79, 168, 168], rtol=1e-15)


def test_d4pi_labels_do_not_depend_on_stored_order():
    ch = synth.CHANNELS["D0_pipipipi"]
    comps, _ = synth.generate(ch, 4000, 12).numpy()
    want = energy.invariant_masses(comps, D4PI_MASKS, relabel="d4pi")
    for perm in ((2, 1, 0, 3), (0, 3, 2, 1), (2, 3, 0, 1)):      # swap pi+, swap pi-, swap both
        got = energy.invariant_masses(comps[list(perm)], D4PI_MASKS, relabel="d4pi")
        assert np.array_equal(got, want)
    # without the rule the coordinates do depend on it
    assert not np.array_equal(energy.invariant_masses(comps[[2, 1, 0, 3]], D4PI_MASKS),
                              energy.invariant_masses(comps, D4PI_MASKS))


def test_d4pi_largest_pair_is_pi3_pi4():
    ch = synth.CHANNELS["D0_pipipipi"]
    comps, _ = synth.generate(ch, 3000, 13).numpy()
    m = energy.invariant_masses(comps, [0b1100, 0b0011, 0b1001, 0b0110], relabel="d4pi")
    # every pi+ pi- pair of the labelled event: (3,4), (1,2), (1,4), (3,2) in 1-based slots
    assert np.all(m[0] >= m[1:].max(axis=0))


def test_d4pi_exact_tie_keeps_first_pair():
    # (0,3) and (2,1) tie for the largest mass: the earlier of the two, (0,3), wins
    comps = np.array([[5, 1, 0, 0], [5, 0, 1, 0], [5, -1, 0, 0], [5, 0, -1, 0]], dtype=np.float64).reshape(4, 4, 1)
    # (0,1): (10, 1, 1, 0) -> 98; (2,3): (10, -1, -1, 0) -> 98; (0,3): (10, 1, -1, 0) -> 98; (2,1) -> 98
    # all four tie: the stored labelling stays
    assert list(energy.d4pi_perm(comps)) == [0]
    comps2 = np.array([[6, 1, 0, 0], [5, 0, 1, 0], [6, -1, 0, 0], [5, 0, -1, 0]], dtype=np.float64).reshape(4, 4, 1)
    # (0,1) = (11, 1, 1, 0) -> 119 = (2,3); (0,3) = (11, 1, -1, 0) -> 119 = (2,1): all tie again
    assert list(energy.d4pi_perm(comps2)) == [0]
    comps3 = np.array([[6, 1, 0, 0], [5, 0, 1, 0], [6, -1, 0, 0], [5, 0, 1, 0]], dtype=np.float64).reshape(4, 4, 1)
    # (2,3) = (11, -1, 1, 0) -> 119, (0,1) = (11, 1, 1, 0) -> 119, (0,3) = (11, 1, 1, 0) -> 119,
    # (2,1) = (11, -1, 1, 0) -> 119: ties keep the stored labelling
    assert list(energy.d4pi_perm(comps3)) == [0]
    comps4 = np.array([[6, 1, 0, 0], [5, 1, 0, 0], [6, -1, 0, 0], [5, -1, 0, 0]], dtype=np.float64).reshape(4, 4, 1)
    # (2,3) = (11, -2, 0, 0) -> 117, (0,1) = (11, 2, 0, 0) -> 117, (0,3) = (11, 0, 0, 0) -> 121,
    # (2,1) = (11, 0, 0, 0) -> 121: (0,3) and (2,1) tie above the others; (0,3) comes first
    assert list(energy.d4pi_perm(comps4)) == [2]


def test_column_pair_sums_brute_force():
    """Every entry of the column pair-sum matrix against explicit pairs, and eq. (2)
    from it against T_eq2 (several blocks, ragged last block)."""
    rng = np.random.default_rng(5)
    n, s = 41, 0.7
    Y = rng.normal(size=(3, n))
    G = (rng.uniform(size=(n, 4)) < 0.5).astype(np.float64)
    psi = lambda i, j: math.exp(-sum((Y[k, i] - Y[k, j]) ** 2 for k in range(3)) / (2 * s * s))
    M = energy.column_pair_sums(Y, G, s, block=16)
    for c in range(4):
        for d in range(4):
            want = sum(G[i, c] * psi(i, j) * G[j, d] for i in range(n) for j in range(n) if i != j)
            assert M[c, d] == pytest.approx(want, rel=1e-13)
    lab = G[:, 0].astype(np.int64)
    cols = np.stack([lab, 1 - lab], axis=1)
    M2 = energy.column_pair_sums(Y, cols, s, block=16)
    nx = int(lab.sum())
    assert energy.T_eq2_columns(M2, 0, 1, nx, n - nx) == pytest.approx(energy.T_eq2(Y, lab, s), rel=1e-12)


def test_eq3_from_column_pair_sums():
    """eq. (3) from the column pair-sum matrix against the direct double sums."""
    rng = np.random.default_rng(6)
    main, mainb = rng.normal(size=(2, 23)), rng.normal(size=(2, 19))
    bkg, bkgb = rng.normal(size=(2, 11)), rng.normal(size=(2, 9))
    Y = np.concatenate([main, mainb, bkg, bkgb], axis=1)
    sizes = [23, 19, 11, 9]
    G = np.zeros((62, 4))
    o = 0
    for k, m in enumerate(sizes):
        G[o:o + m, k] = 1
        o += m
    M = energy.column_pair_sums(Y, G, 0.9, block=8)
    got = energy.T_eq3_columns(M, 0, 1, 2, 3, 23, 19, 11, 9, 4.0, 3.0)
    assert got == pytest.approx(energy.T_eq3(main, mainb, bkg, bkgb, 4.0, 3.0, 0.9), rel=1e-12)
    t1, t2, t3 = energy.T_eq3_columns(M, 0, 1, 2, 3, 23, 19, 11, 9, 4.0, 3.0, terms=True)
    assert sum(t1) + sum(t2) - sum(t3) == pytest.approx(got, rel=1e-15)
