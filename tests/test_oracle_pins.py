"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: the hand-built events carry
results derived by hand (tests/golden/handbuilt.txt), the identities compare
the float64 textbook rest-frame path with the exact determinant path, and the
statistical checks compare with closed forms of the injected asymmetries.
"""
import math
import os
from fractions import Fraction as F

import mpmath
import numpy as np
import pytest
import torch

import oracle
from oracle import exact
from paper_1612_04705_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load_handbuilt():
    rows = []
    with open(os.path.join(GOLD, "handbuilt.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            t = line.split()
            name, tag = t[0], int(t[1])
            v = [float(x) for x in t[2:18]]
            cls, b10, b12, m03 = int(t[18]), int(t[19]), int(t[20]), float(t[21])
            rows.append((name, tag, v, cls, b10, b12, m03))
    return rows


def _as_sample(rows, dtype=np.float32):
    n = len(rows)
    comps = np.zeros((4, 4, n), dtype=dtype)
    tag = np.zeros(n, dtype=np.int8)
    for i, r in enumerate(rows):
        comps[:, :, i] = np.array(r[2], dtype=dtype).reshape(4, 4)
        tag[i] = r[1]
    return comps, tag


TRIPLE, PLANES = (0, 1, 2), (0, 1, 2, 3)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_handbuilt_golden(oracle_lib, dtype):
    rows = _load_handbuilt()
    comps, tag = _as_sample(rows, dtype)
    for nphi, col in ((10, 4), (12, 5)):
        ax = [synth.absphi_axis(nphi)]
        r = oracle.run(comps, tag, TRIPLE, PLANES, ax, want_events=True)
        bf = oracle.brute_force(comps, tag, TRIPLE, PLANES, ax)
        assert r["counts"] == bf["counts"] and r["stats"] == bf["stats"]
        for i, row in enumerate(rows):
            assert r["cls"][i] == row[3], row[0]
            assert bf["cls"][i] == row[3], row[0]
            if row[3] < 4:
                # the single-event decision of the exact path
                c, b = exact.exact_decision([[float(x) for x in comps[s, :, i]] for s in range(4)],
                                            int(tag[i]), TRIPLE, PLANES,
                                            [(a.kind, a.slots, a.edges) for a in ax])
                assert (c, b) == (row[3], row[col]), row[0]
    # the 90-degree events sit exactly on the 12-bin edge and must have been flagged
    r = oracle.run(comps, tag, TRIPLE, PLANES, [synth.absphi_axis(12)])
    assert r["n_flagged"] >= 4


def test_handbuilt_mass_and_abscos_edges(oracle_lib):
    rows = {r[0]: r for r in _load_handbuilt()}
    comps, tag = _as_sample([rows["H1"], rows["H7"], rows["H5"]])
    # m03 = 6 exactly for H1/H5: on an inner edge, on the closed last edge, and outside
    for edges, want in (([5.0, 6.0, 7.0], 1), ([4.0, 5.0, 6.0], 1), ([6.5, 7.0, 8.0], -1),
                        ([6.0, 7.0, 8.0], 0)):
        ax = [synth.Axis(synth.AXIS_MASS, np.array(edges), 0b1001)]
        for i in (0, 2):
            c, b = exact.exact_decision([[float(x) for x in comps[s, :, i]] for s in range(4)],
                                        int(tag[i]), TRIPLE, PLANES, [(1, 0b1001, np.array(edges))])
            assert b == want
        r = oracle.run(comps, tag, TRIPLE, PLANES, ax)
        bf = oracle.brute_force(comps, tag, TRIPLE, PLANES, ax)
        assert r["counts"] == bf["counts"] and r["stats"] == bf["stats"]
    # H7: |cos theta| of slot 0 is exactly 3/5, which lies below the double 0.6000000000000001
    # (numpy.linspace's 4th edge) and above the double nearest 0.6 (0.59999999999999998)
    e_lin = np.linspace(0.0, 1.0, 6)
    e_lit = np.array([0.0, 0.2, 0.4, 0.6, 0.8, 1.0])
    assert F(e_lin[3]) > F(3, 5) > F(e_lit[3])
    h7 = [[float(x) for x in comps[s, :, 1]] for s in range(4)]
    assert exact.exact_decision(h7, 0, TRIPLE, PLANES, [(2, 0, e_lin)]) == (0, 2)
    assert exact.exact_decision(h7, 0, TRIPLE, PLANES, [(2, 0, e_lit)]) == (0, 3)
    # H5: slot 0 moves along the flight axis (|cos| = 1, closed last bin), slot 1 perpendicular
    h5 = [[float(x) for x in comps[s, :, 2]] for s in range(4)]
    assert exact.exact_decision(h5, 0, TRIPLE, PLANES, [(2, 0, e_lin)])[1] == 4
    assert exact.exact_decision(h5, 0, TRIPLE, PLANES, [(2, 1, e_lin)])[1] == 0
    assert exact.exact_decision(h5, 0, TRIPLE, PLANES, [(2, 3, e_lin)])[1] == 1
    for sl in range(4):
        ax = [synth.Axis(synth.AXIS_ABSCOS, e_lit, sl)]
        r = oracle.run(comps, tag, TRIPLE, PLANES, ax)
        bf = oracle.brute_force(comps, tag, TRIPLE, PLANES, ax)
        assert r["counts"] == bf["counts"] and r["stats"] == bf["stats"]


def test_handbuilt_mass_values(oracle_lib):
    rows = _load_handbuilt()
    comps, tag = _as_sample(rows, np.float64)
    ax = [synth.Axis(synth.AXIS_MASS, np.array([0.0, 1000.0]), 0b1001)]
    r = oracle.run(comps, tag, TRIPLE, PLANES, ax, want_events=True)
    for i, row in enumerate(rows):
        if row[3] < 4:      # class-zero events are decided before any coordinate is formed
            assert r["coord"][i, 0] == pytest.approx(row[6], rel=1e-14, abs=1e-12), row[0]


def _sample(chname, n, seed, dtype=torch.float32, **kw):
    ch = synth.CHANNELS[chname]
    s = synth.generate(ch, n, seed, dtype=dtype, **kw)
    comps, tag = s.numpy()
    return ch, s, comps, tag


def _rest_frame_exact(comps, i, triple):
    """det[P; A; B; C] / M in exact arithmetic (M via mpmath at 100 digits)."""
    ev = exact.ExactEvent([[float(comps[s, c, i]) for c in range(4)] for s in range(4)], 0)
    d = ev.det_triple(triple)
    mpmath.mp.dps = 100
    M = mpmath.sqrt(mpmath.mpf(ev.M2.numerator) / ev.M2.denominator)
    return float(mpmath.mpf(d.numerator) / d.denominator / M)


@pytest.mark.parametrize("fixed_gamma", [None, 50.0, 2000.0])
def test_rest_frame_triple_product_identity(oracle_lib, fixed_gamma):
    """The textbook boost + triple product equals det[P;A;B;C]/M (exact) to float64 accuracy."""
    ch, s, comps, tag = _sample("Lb_pKpipi", 300, 11, dtype=torch.float64, fixed_gamma=fixed_gamma)
    r = oracle.run(comps, tag, ch.triple, ch.planes, want_events=True)
    g = float(fixed_gamma or s.gamma.max())
    for i in range(0, 300, 7):
        want = _rest_frame_exact(comps, i, ch.triple)
        got = r["ct"][i]
        assert abs(got - want) <= 1e-13 * (1 + g * g) * abs(want) + 1e-300, (i, got, want)


def test_plane_angle_matches_generated(oracle_lib):
    """Measured cos Phi equals cos(phi_gen) and sign(C_T) = sign(sin phi_gen) (float64 storage)."""
    ch, s, comps, tag = _sample("Lb_pKpipi", 5000, 12, dtype=torch.float64)
    r = oracle.run(comps, tag, ch.triple, ch.planes, [synth.absphi_axis(10)], want_events=True)
    phi = s.phi_gen.numpy()
    assert np.abs(r["coord"][:, 0] - np.cos(phi)).max() < 1e-8
    sgn = np.where(tag == 0, np.where(r["cls"] == 0, 1, -1), np.where(r["cls"] == 3, 1, -1))
    assert np.array_equal(sgn, np.sign(np.sin(phi)).astype(int))


def test_mass_matches_generated_pair(oracle_lib):
    """m(0,1) and m(2,3) are the generated pair masses (D0 -> K+ K- pi+ pi-, float64 storage)."""
    ch = synth.CHANNELS["D0_KKpipi"]
    s = synth.generate(ch, 3000, 13, dtype=torch.float64)
    comps, tag = s.numpy()
    ax = [synth.mass_axis((0, 1), 987.354, 1585.7, 32), synth.mass_axis((2, 3), 279.14, 877.486, 32)]
    r = oracle.run(comps, tag, ch.triple, ch.planes, ax, want_events=True)
    keep = np.ones(3000, bool)
    keep[r["flagged"]] = False          # flagged events stop before their coordinates
    g2 = 1 + s.gamma.numpy() ** 2
    m01 = np.sqrt(r["coord"][:, 0])
    m23 = np.sqrt(r["coord"][:, 1])
    assert (np.abs(m01 - s.m12.numpy()) <= 1e-14 * g2 * m01)[keep].all()
    assert (np.abs(m23 - s.m34.numpy()) <= 1e-14 * g2 * m01)[keep].all()
    assert r["stats"][3] == 0


def _mirror(comps):
    m = comps.copy()
    m[:, 1:, :] *= -1
    return m


def test_parity_flips_sign_exactly(oracle_lib):
    ch, s, comps, tag = _sample("Lb_ppipipi", 20000, 14)
    ax = [synth.absphi_axis(12)]
    a = oracle.run(comps, tag, ch.triple, ch.planes, ax)
    b = oracle.run(_mirror(comps), tag, ch.triple, ch.planes, ax)
    for ra, rb in zip(a["counts"], b["counts"]):
        assert ra == [rb[1], rb[0], rb[3], rb[2]]
    assert a["stats"] == b["stats"]


def test_cp_transform_swaps_I_III(oracle_lib):
    """CP image (flavour flipped, momenta negated) maps [I] <-> [III], [II] <-> [IV] (Sect. 5)."""
    ch, s, comps, tag = _sample("Lb_pKpipi", 20000, 15)
    ax = [synth.absphi_axis(10), synth.lb_mass03_axis(ch)]
    a = oracle.run(comps, tag, ch.triple, ch.planes, ax)
    b = oracle.run(_mirror(comps), (1 - tag).astype(np.int8), ch.triple, ch.planes, ax)
    for ra, rb in zip(a["counts"], b["counts"]):
        assert ra == [rb[2], rb[3], rb[0], rb[1]]


def test_mirrored_sample_has_zero_A_T(oracle_lib):
    ch, s, comps, tag = _sample("Lb_pKpipi", 10000, 16, inj=synth.INJ_SIN)
    both = np.concatenate([comps, _mirror(comps)], axis=2)
    tags = np.concatenate([tag, tag])
    r = oracle.run(both, tags, ch.triple, ch.planes, [synth.absphi_axis(10)])
    for row in r["counts"]:
        assert row[0] == row[1] and row[2] == row[3]
        a = exact.asym_row(row)
        if row[0] + row[1]:
            assert a["A_T"][0] == 0


def test_slot_permutation_parity(oracle_lib):
    """Swapping two slots of the triple flips the sign; a cyclic shift keeps it."""
    ch, s, comps, tag = _sample("Lb_pKpipi", 5000, 17)
    base = oracle.run(comps, tag, (0, 1, 2), ch.planes)["counts"][0]
    swp = oracle.run(comps, tag, (1, 0, 2), ch.planes)["counts"][0]
    cyc = oracle.run(comps, tag, (1, 2, 0), ch.planes)["counts"][0]
    assert swp == [base[1], base[0], base[3], base[2]]
    assert cyc == base
    # with four momenta summing to P, the triple (0,2,3) equals the triple (0,1,2)
    # (rest frame: p3 = -(p0+p1+p2)); (0,1,3) has the opposite sign
    assert oracle.run(comps, tag, (0, 2, 3), ch.planes)["counts"][0] == base
    t013 = oracle.run(comps, tag, (0, 1, 3), ch.planes)["counts"][0]
    assert t013 == [base[1], base[0], base[3], base[2]]


def test_identical_particle_swap_flips_sign(oracle_lib):
    ch, s, comps, tag = _sample("Lb_ppipipi", 5000, 18)
    sw = comps[[0, 3, 2, 1]].copy()
    a = oracle.run(comps, tag, ch.triple, ch.planes)["counts"][0]
    b = oracle.run(sw, tag, ch.triple, ch.planes)["counts"][0]
    assert b == [a[1], a[0], a[3], a[2]]


def test_lorentz_invariance_of_classes(oracle_lib):
    """Re-boosting the stored events (float64) leaves every class and |Phi| bin unchanged."""
    ch, s, comps, tag = _sample("Lb_pKpipi", 3000, 19, dtype=torch.float64)
    bx, by, bz = 0.3, -0.5, 0.6
    g = 1 / math.sqrt(1 - bx * bx - by * by - bz * bz)
    out = comps.copy()
    for sl in range(4):
        E, px, py, pz = comps[sl]
        bp = bx * px + by * py + bz * pz
        k = (g - 1) * bp / (bx * bx + by * by + bz * bz) + g * E
        out[sl] = [g * (E + bp), px + k * bx, py + k * by, pz + k * bz]
    ax = [synth.absphi_axis(10)]
    a = oracle.run(comps, tag, ch.triple, ch.planes, ax, want_events=True)
    b = oracle.run(out, tag, ch.triple, ch.planes, ax, want_events=True)
    assert np.array_equal(a["cls"], b["cls"])
    keep = np.ones(3000, bool)
    keep[a["flagged"]] = False
    keep[b["flagged"]] = False
    assert np.abs(a["coord"][:, 0] - b["coord"][:, 0])[keep].max() < 1e-8


@pytest.mark.parametrize("chname,axes", [
    ("Lb_ppipipi", lambda ch: [synth.absphi_axis(10)]),
    ("Lb_pKpipi", lambda ch: [synth.absphi_axis(10), synth.lb_mass03_axis(ch)]),
    ("Lb_ppiKK", lambda ch: [synth.abscos_axis(0, 5), synth.absphi_axis(10)]),
    ("D0_KKpipi", lambda ch: [synth.mass_axis((0, 1), 987.354, 1585.7, 32),
                              synth.mass_axis((2, 3), 279.14, 877.486, 32)]),
])
def test_float64_path_equals_exact_brute_force(oracle_lib, chname, axes):
    ch, s, comps, tag = _sample(chname, 1500, 20)
    ax = axes(ch)
    r = oracle.run(comps, tag, ch.triple, ch.planes, ax)
    bf = oracle.brute_force(comps, tag, ch.triple, ch.planes, ax)
    assert r["counts"] == bf["counts"]
    assert r["stats"] == bf["stats"]


def test_coplanar_events_are_zero(oracle_lib):
    ch, s, comps, tag = _sample("Lb_pKpipi", 2000, 21)
    flat = comps.copy()
    flat[:, 3, :] = 0.0          # all pz = 0: the four momenta span a 3-d subspace
    r = oracle.run(flat, tag, ch.triple, ch.planes, [synth.absphi_axis(10)])
    assert r["stats"][1] == 2000 - r["stats"][2]
    assert sum(r["counts"][0]) == 0


def test_invalid_inputs(oracle_lib):
    ch, s, comps, tag = _sample("Lb_pKpipi", 64, 22)
    c = comps.copy()
    t = tag.copy()
    c[1, 2, 3] = np.nan
    c[2, 0, 5] = np.inf
    t[7] = 7
    c[:, 0, 9] = 0.0      # E = 0 for every daughter: P is space-like
    r = oracle.run(c, t, ch.triple, ch.planes, [synth.absphi_axis(10)])
    assert r["stats"][2] == 4
    assert r["stats"][0] == 64


def _binned_a_t(counts):
    out = []
    for row in counts[1:]:
        n = row[0] + row[1]
        out.append((row[0] - row[1]) / n if n else float("nan"))
    return out


def test_injected_sin_phi_closed_form(oracle_lib):
    """w = 1 + eps sin(phi): A_T = 2 eps / pi globally and eps (cos a - cos b)/(b - a) per |Phi| bin."""
    ch, s, comps, tag = _sample("Lb_pKpipi", 200000, 23, inj=synth.INJ_SIN)
    r = oracle.run(comps, tag, ch.triple, ch.planes, [synth.absphi_axis(12)])
    a = exact.asym_row(r["counts"][0])
    for key, want in (("A_T", 0.2 / math.pi), ("Abar_T", -0.1 / math.pi),
                      ("a_CP", 0.15 / math.pi), ("a_P", 0.05 / math.pi)):
        val, sig = a[key]
        assert abs(float(val) - want) < 5 * sig, (key, float(val), want, sig)
    w = math.pi / 6
    for j in range(6):
        row = r["counts"][1 + j]
        n = row[0] + row[1]
        want = 0.1 * (math.cos(j * w) - math.cos((j + 1) * w)) / w
        got = (row[0] - row[1]) / n
        assert abs(got - want) < 5 * math.sqrt((1 - want * want) / n), (j, got, want)


def test_injected_sin2phi_closed_form(oracle_lib):
    """w = 1 + 0.03 sin 2phi (M only): global A_T = 0, A_T(|Phi| bin) = 0.03 (cos 2a - cos 2b)/(2w)."""
    ch, s, comps, tag = _sample("Lb_pKpipi", 200000, 24, inj=synth.INJ_SIN2, frac_m=0.52)
    r = oracle.run(comps, tag, ch.triple, ch.planes, [synth.absphi_axis(10)])
    w = math.pi / 5
    for j in range(5):
        row = r["counts"][1 + j]
        n = row[0] + row[1]
        want = 0.03 * (math.cos(2 * j * w) - math.cos(2 * (j + 1) * w)) / (2 * w)
        got = (row[0] - row[1]) / n
        assert abs(got - want) < 5 * math.sqrt(1 / n), (j, got, want)
    a = exact.asym_row(r["counts"][0])
    assert abs(float(a["A_T"][0])) < 5 * a["A_T"][1]
    nm = sum(r["counts"][0][:2])
    assert abs(nm / 200000 - 0.52) < 5 * math.sqrt(0.25 / 200000)


def test_uniform_absphi_and_abscos_in_phase_space(oracle_lib):
    """Pure phase space: |Phi| and |cos theta| are uniform (chi^2 of equal-width bins)."""
    from scipy.stats import chi2
    ch, s, comps, tag = _sample("Lb_ppiKK", 100000, 25)
    r = oracle.run(comps, tag, ch.triple, ch.planes, [synth.abscos_axis(0, 5), synth.absphi_axis(10)])
    tot = np.array([sum(row) for row in r["counts"][1:]]).reshape(5, 5)
    for marg in (tot.sum(axis=0), tot.sum(axis=1)):
        exp_ = marg.sum() / len(marg)
        x2 = float(((marg - exp_) ** 2 / exp_).sum())
        assert chi2.sf(x2, len(marg) - 1) > 1e-4, marg


def test_asymmetry_golden(oracle_lib):
    with open(os.path.join(GOLD, "asym_counts.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            t = line.split()
            n = [int(x) for x in t[:4]]
            want = [None if x == "None" else F(x) for x in t[4:12]]
            a = exact.asym_row(n)
            keys = ["A_T", "Abar_T", "a_CP", "a_P", "A_plus", "A_minus", "A_even", "A_odd"]
            for k, w in zip(keys, want):
                assert a[k][0] == w, (n, k, a[k][0], w)
            if n == [7, 0, 0, 0]:
                assert a["A_T"][1] == 0.0 and math.isnan(a["Abar_T"][1])
    # binomial sigma of A = 0.2 over 100 events
    a = exact.asym_row([60, 40, 45, 55])
    assert a["A_T"][1] == pytest.approx(math.sqrt(0.96 / 100), rel=1e-15)
    assert a["a_CP"][1] == pytest.approx(0.5 * math.sqrt(0.96 / 100 + 0.99 / 100), rel=1e-15)


def test_scp_chi2(oracle_lib):
    """eq. (1): identical histograms give S = 0, chi^2 = 0, p = 1; a hand-computed case."""
    s, x2, ndf, p = exact.scp([10, 20, 30], [20, 40, 60])
    assert x2 == 0 and ndf == 2 and p == 1.0
    # alpha = 2: S = (30 - 2*10)/sqrt(30 + 4*10) = 10/sqrt(70); second bin (10 - 2*20)/sqrt(10 + 4*20)
    s, x2, ndf, p = exact.scp([30, 10], [10, 10])
    assert s[0] == pytest.approx(10 / math.sqrt(70), rel=1e-15)
    assert s[1] == pytest.approx(-10 / math.sqrt(50), rel=1e-15)
    assert ndf == 1 and p == pytest.approx(math.erfc(math.sqrt(x2 / 2)), rel=1e-12)
