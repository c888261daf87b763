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
