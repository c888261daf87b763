"""GPU parity of the energy test (pair sums on the matrix cores) against the oracle.

Tolerance.  The device forms coordinates in float32 (relative rounding 2^-24 of
masses ~1-2 GeV) and psi in float32 with the hardware exp2 (a few ulp): the
distance error d * |delta d| / sigma^2 with |delta d| <~ 4e-7 GeV puts each psi
within ~1e-6 (relative) of the float64 value at sigma = 0.3 GeV.  The squared
distance itself is a dot product of centred vectors split into float16 terms on
the matrix cores (rounding ~2^-22 * (2 |v_i|^2 + 2 |v_j|^2) with |v|^2 < 3 here:
in an emulation on these coordinates, psi within 2e-6, rms 3e-7, of random
sign).  The matrix
cores take psi as two float16 terms whose sum is within 2^-20 (~1e-6) of it,
and accumulate exact products in float32 tiles that are reduced into float64
every 1024 j: 128 accumulation roundings of 2^-24 (worst case ~8e-6, typically
~3e-7 as they are of random sign).  Each of the three terms of T inherits these
relative errors; the test allows 1e-5 of the sum of the three terms' magnitudes.
"""
import numpy as np
import pytest
import torch

from oracle import energy
from paper_1612_04705_amd import synth

pytestmark = pytest.mark.gpu

# D0 -> K+ K- pi+ pi- coordinates (Sect. 4.2, Table 1): m12, m14, m23, m34, m134
MASKS = [0b0011, 0b1001, 0b0110, 0b1100, 0b1101]


@pytest.fixture(scope="module")
def tp():
    from paper_1612_04705_amd import tpasym
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    tpasym.load()
    return tpasym


def sample(n, seed):
    ch = synth.CHANNELS["D0_KKpipi"]
    return ch, synth.generate(ch, n, seed, inj=synth.INJ_SGN)


def terms(Y, lab, sigma):
    Y = np.asarray(Y, dtype=np.float64)
    lab = np.asarray(lab).astype(bool)
    X, B = Y[:, lab], Y[:, ~lab]
    n, nb = X.shape[1], B.shape[1]
    return (0.5 * energy.pair_sum(X, X, sigma, True) / (n * (n - 1)),
            0.5 * energy.pair_sum(B, B, sigma, True) / (nb * (nb - 1)),
            energy.pair_sum(X, B, sigma, False) / (n * nb))


def eq3_term_magnitude(main, main_bar, bkg, bkg_bar, b, b_bar, sigma):
    """Sum of the magnitudes of the ten coefficient x pair-sum terms of eq. (3)."""
    S = lambda A, B, same=False: energy.pair_sum(A, B, sigma, same)
    n, nb, bs, bsb = main.shape[1], main_bar.shape[1], bkg.shape[1], bkg_bar.shape[1]
    w, wb = n - b, nb - b_bar
    t1 = [S(main, main, True), 2 * b / bs * S(main, bkg), b * (b + 1) / (bs * (bs - 1)) * S(bkg, bkg, True)]
    t2 = [S(main_bar, main_bar, True), 2 * b_bar / bsb * S(main_bar, bkg_bar),
          b_bar * (b_bar + 1) / (bsb * (bsb - 1)) * S(bkg_bar, bkg_bar, True)]
    t3 = [S(main, main_bar), b_bar / bsb * S(main, bkg_bar), b / bs * S(bkg, main_bar),
          b * b_bar / (bs * bsb) * S(bkg, bkg_bar)]
    return sum(t1) / (2 * w * (w - 1)) + sum(t2) / (2 * wb * (wb - 1)) + sum(t3) / (w * wb)


def test_coords_match_oracle(tp):
    ch, s = sample(3001, 80)
    ds = tp.DeviceSample.from_sample(s)
    Yg = tp.coords(ds, MASKS, 1e-3).cpu().numpy().astype(np.float64)
    comps, _ = s.numpy()
    Yo = energy.invariant_masses(comps, MASKS) * 1e-3
    # float32 output: within 2^-24 of the float64 value beyond the inputs' own rounding
    W = np.stack([np.abs(comps[[t for t in range(4) if m & (1 << t)]].astype(np.float64)).sum(axis=(0, 1))
                  for m in MASKS]) * 1e-3
    tol = 2.0 * W * W * 2.0 ** -53 * 64 / np.maximum(Yo, 1e-3) + 2.0 ** -23 * Yo
    assert np.all(np.abs(Yg - Yo) <= tol)


@pytest.mark.parametrize("n,sigma", [(2000, 0.3), (1277, 0.8)])
def test_eq2_observed_and_permutations(tp, n, sigma):
    ch, s = sample(n, 81 + n)
    ds = tp.DeviceSample.from_sample(s)
    # P-odd split (Sect. 5): X = classes I and IV, Xbar = II and III
    cls, _, _ = tp.compute(ds, tp.channel(ch.triple, ch.planes), tp.TP_PREC_F64)
    cls = cls.cpu().numpy()
    assert np.all(cls < 4)
    lab = ((cls == 0) | (cls == 3)).astype(np.uint8)
    rng = np.random.default_rng(7)
    nperm = 14
    C = 32
    cols = np.zeros((n, C), dtype=np.uint8)
    cols[:, 0] = 1                      # all ones
    cols[:, 1] = lab
    perms = [rng.permutation(lab) for _ in range(nperm)]
    for k, pl in enumerate(perms):
        cols[:, 2 + k] = pl
    Yg = tp.coords(ds, MASKS, 1e-3)
    sums = tp.pairsums(Yg, torch.from_numpy(cols).cuda(), sigma, nrow=1)
    torch.cuda.synchronize()
    T = tp.energy_eq2(sums, cols.sum(axis=0), n, ones_row=0, ones_col=0)
    comps, _ = s.numpy()
    Yo = energy.invariant_masses(comps, MASKS) * 1e-3
    want = [energy.T_eq2(Yo, lab, sigma)] + [energy.T_eq2(Yo, pl, sigma) for pl in perms]
    for k, w in enumerate(want):
        a, b, c = terms(Yo, lab if k == 0 else perms[k - 1], sigma)
        tol = 1e-5 * (abs(a) + abs(b) + abs(c))
        assert abs(T[1 + k] - w) <= tol, (k, T[1 + k], w, tol)
    # p-value: permutations strictly above the observed T; a permutation whose
    # oracle T lies within the tolerance of the observed one may go either way
    tol0 = 1e-5 * sum(abs(t) for t in terms(Yo, lab, sigma))
    sure = [abs(w - want[0]) > 2 * tol0 for w in want[1:]]
    got_above = [T[2 + k] > T[1] for k in range(nperm)]
    want_above = [w > want[0] for w in want[1:]]
    assert all(g == w for g, w, s_ in zip(got_above, want_above, sure) if s_)


def test_eq2_sigma_infinite_is_zero(tp):
    ch, s = sample(777, 90)
    ds = tp.DeviceSample.from_sample(s)
    lab = (np.arange(777) % 3 == 0).astype(np.uint8)
    cols = np.zeros((777, 32), dtype=np.uint8)
    cols[:, 0] = 1
    cols[:, 1] = lab
    sums = tp.pairsums(tp.coords(ds, MASKS, 1e-3), torch.from_numpy(cols).cuda(), 1e12)
    torch.cuda.synchronize()
    S = sums.cpu().numpy()
    # every psi is exactly 1: ordered-pair counts
    assert S[0, 1] == 777 * 776 and S[1, 0] == lab.sum() * (lab.sum() - 1)
    T = tp.energy_eq2(S, cols.sum(axis=0), 777)
    assert abs(T[1]) < 1e-15


def test_eq3_against_oracle(tp):
    # main samples with background, background samples from a flat (different) source
    ch, sig = sample(1500, 91)
    _, bk = sample(900, 92)
    ds_s, ds_b = tp.DeviceSample.from_sample(sig), tp.DeviceSample.from_sample(bk)
    Ys = tp.coords(ds_s, MASKS, 1e-3)
    Yb = tp.coords(ds_b, MASKS, 1e-3)
    rng = np.random.default_rng(11)
    fl_main = (rng.uniform(size=1500) < 0.6).astype(np.uint8)     # flavour X in the main samples
    fl_bkg = (rng.uniform(size=900) < 0.6).astype(np.uint8)
    n = 2400
    Y = torch.cat([Ys, Yb], dim=1).contiguous()
    main = np.r_[np.ones(1500), np.zeros(900)].astype(np.uint8)
    bkgc = 1 - main
    perms = [(fl_main, fl_bkg)] + [(rng.permutation(fl_main), rng.permutation(fl_bkg)) for _ in range(5)]
    C = 32
    cols = np.zeros((n, C), dtype=np.uint8)
    cols[:, 0], cols[:, 1] = main, bkgc
    triples = []
    for k, (fm, fb) in enumerate(perms):
        a = np.r_[fm, np.zeros(900)].astype(np.uint8)
        beta = np.r_[np.zeros(1500), fb].astype(np.uint8)
        cols[:, 2 + 3 * k], cols[:, 3 + 3 * k], cols[:, 4 + 3 * k] = a, beta, a + beta
        triples.append((2 + 3 * k, 3 + 3 * k, 4 + 3 * k))
    sums = tp.pairsums(Y, torch.from_numpy(cols).cuda(), 0.4, nrow=2)
    torch.cuda.synchronize()
    nm, nmb = int(fl_main.sum()), 1500 - int(fl_main.sum())
    nb_, nbb = int(fl_bkg.sum()), 900 - int(fl_bkg.sum())
    b, b_bar = 0.3 * nm, 0.3 * nmb
    T = tp.energy_eq3(sums, 0, 1, 0, 1, triples, nm, nmb, nb_, nbb, b, b_bar)
    cs, _ = sig.numpy()
    cb, _ = bk.numpy()
    Yso = energy.invariant_masses(cs, MASKS) * 1e-3
    Ybo = energy.invariant_masses(cb, MASKS) * 1e-3
    for k, (fm, fb) in enumerate(perms[:3]):
        fm, fb = fm.astype(bool), fb.astype(bool)
        w = energy.T_eq3(Yso[:, fm], Yso[:, ~fm], Ybo[:, fb], Ybo[:, ~fb], b, b_bar, 0.4)
        # the same relative sum error as for eq. (2) (1e-5), applied to every one of
        # the ten pair-sum terms of eq. (3) with its coefficient
        mag = eq3_term_magnitude(Yso[:, fm], Yso[:, ~fm], Ybo[:, fb], Ybo[:, ~fb], b, b_bar, 0.4)
        assert abs(T[k] - w) <= 1e-5 * mag, (k, T[k], w)


def test_full_size_sampled_sums(tp):
    """At 1e6 events: a column holding 64 scattered events makes each of its sums
    O(n x 64) pairs, which the oracle evaluates directly."""
    n = 1_000_000
    spec = synth.SampleSpec(synth.CHANNELS["D0_KKpipi"], n, 77, [], inj=synth.INJ_SGN)
    s = synth.make_sample(spec)
    ds = tp.DeviceSample.from_sample(s)
    Y = tp.coords(ds, MASKS, 1e-3)
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(n, 64, replace=False))
    cols = np.zeros((n, 32), dtype=np.uint8)
    cols[:, 0] = 1
    cols[pick, 1] = 1
    sums = tp.pairsums(Y, torch.from_numpy(cols).cuda(), 0.3, nrow=1)
    torch.cuda.synchronize()
    S = sums.cpu().numpy()
    comps, _ = s.numpy()
    Yo = energy.invariant_masses(comps, MASKS) * 1e-3
    # every event against the picked ones, minus the 64 self-pairs (psi = 1)
    want_all = energy.pair_sum(Yo, Yo[:, pick], 0.3, False) - 64.0
    want_diag = energy.pair_sum(Yo[:, pick], Yo[:, pick], 0.3, True)
    assert abs(S[1, 1] - want_all) <= 1e-5 * want_all
    assert abs(S[1, 0] - want_diag) <= 1e-5 * want_diag


D4PI_MASKS = [0b0011, 0b1001, 0b0110, 0b0111, 0b1011]     # m12, m14, m23, m123, m124 (Sect. 4.2, Table 1)


def _d4pi_check(tp, comps, label):
    s = synth.Sample(synth.CHANNELS["D0_pipipipi"],
                     [[torch.from_numpy(np.ascontiguousarray(comps[a][b])) for b in range(4)] for a in range(4)],
                     torch.zeros(comps.shape[2], dtype=torch.int8))
    ds = tp.DeviceSample.from_sample(s)
    Yg = tp.coords(ds, D4PI_MASKS, 1e-3, relabel=tp.TP_RELABEL_D4PI).cpu().numpy().astype(np.float64)
    Yo = energy.invariant_masses(comps, D4PI_MASKS, relabel="d4pi") * 1e-3
    W = np.abs(comps.astype(np.float64)).sum(axis=(0, 1)) * 1e-3
    tol = 2.0 * W * W * 2.0 ** -53 * 64 / np.maximum(Yo, 1e-3) + 2.0 ** -23 * Yo
    bad = np.abs(Yg - Yo) > tol
    print(f"[coords] {label}: {int(bad.any(axis=0).sum())} of {comps.shape[2]} events off", flush=True)
    assert not bad.any()


def test_coords_d4pi_relabel_matches_oracle(tp):
    ch = synth.CHANNELS["D0_pipipipi"]
    comps, _ = synth.generate(ch, 5003, 82).numpy()
    # store the identical pions in a random order per event
    k = np.random.default_rng(4).integers(0, 4, size=comps.shape[2])
    perms = np.array(energy.D4PI_PERMS)[k]
    idx = np.arange(comps.shape[2])
    shuffled = np.stack([comps[perms[:, t], :, idx].T for t in range(4)])
    _d4pi_check(tp, shuffled, "shuffled pions")


def test_coords_d4pi_float64_storage(tp):
    ch = synth.CHANNELS["D0_pipipipi"]
    comps, _ = synth.generate(ch, 2001, 83, dtype=torch.float64).numpy()
    k = np.random.default_rng(5).integers(0, 4, size=comps.shape[2])
    perms = np.array(energy.D4PI_PERMS)[k]
    idx = np.arange(comps.shape[2])
    _d4pi_check(tp, np.stack([comps[perms[:, t], :, idx].T for t in range(4)]), "float64 storage")


def test_coords_d4pi_exact_ties(tp):
    # small-integer events with tied pair masses (exact path, stored-order ties)
    rng = np.random.default_rng(6)
    rows = []
    for _ in range(257):
        a, b = (int(v) for v in rng.integers(1, 6, size=2))
        E1, E2 = (int(v) for v in rng.integers(10, 14, size=2))
        rows.append([[E1, a, 0, 0], [E2, 0, b, 0], [E1, -a, 0, 0], [E2, 0, -b, 0]])
    comps = np.array(rows, dtype=np.float32).transpose(1, 2, 0).copy()
    _d4pi_check(tp, comps, "ties")


@pytest.mark.parametrize("C,nrow,n", [(32, 0, 1500), (64, 1, 2051), (64, 3, 1729), (128, 2, 2051), (128, 3, 1300),
                                      (32, 1, 2), (32, 1, 3), (64, 2, 127), (32, 3, 129), (128, 1, 300)])
def test_raw_pair_sums_all_tile_counts(tp, C, nrow, n):
    """sums[c][0] = sum_{i != j} G_ic psi_ij G_jc and sums[c][1+q] = sum_{i != j} G_iq psi_ij G_jc
    against the dense float64 psi matrix, for every column-tile count and row-weight count
    (ragged n: several workgroup pieces and a partial last block)."""
    ch, s = sample(n, 200 + C + nrow)
    ds = tp.DeviceSample.from_sample(s)
    Yg = tp.coords(ds, MASKS, 1e-3)
    rng = np.random.default_rng(C + nrow)
    G = (rng.uniform(size=(n, C)) < rng.uniform(0.1, 0.9, size=C)).astype(np.uint8)
    sums = tp.pairsums(Yg, torch.from_numpy(G).cuda(), 0.35, nrow=nrow)
    torch.cuda.synchronize()
    S = sums.cpu().numpy()
    comps, _ = s.numpy()
    Yo = energy.invariant_masses(comps, MASKS) * 1e-3
    Psi = energy.psi_block(Yo, Yo, 0.35)
    np.fill_diagonal(Psi, 0.0)
    Gf = G.astype(np.float64)
    V = Psi @ Gf                                  # [n][C]
    want0 = np.einsum("ic,ic->c", Gf, V)
    assert np.all(np.abs(S[:, 0] - want0) <= 1e-5 * want0 + 1e-9)
    for q in range(nrow):
        wq = Gf[:, q] @ V                         # sum_i G_iq (Psi G)_ic
        assert np.all(np.abs(S[:, 1 + q] - wq) <= 1e-5 * wq + 1e-9), q


@pytest.mark.parametrize("sigma", [0.05, 0.1, 2.0])
def test_raw_pair_sums_sigma_range(tp, sigma):
    """Pair sums against the dense float64 psi matrix for narrow and wide kernels.  The
    squared distances are a float16-split dot product of centred vectors, whose rounding grows
    with the squared distance of the events from the centre in units of sigma (|v|^2 up to
    ~100 at sigma = 0.05 GeV here): single psi values lose accuracy (an emulation on these
    coordinates gives up to ~7e-5 relative at sigma = 0.05), but the errors are of
    random sign, so the sums stay within the same 1e-5 as at sigma = 0.3."""
    n, C, nrow = 2051, 64, 2
    ch, s = sample(n, 911)
    ds = tp.DeviceSample.from_sample(s)
    Yg = tp.coords(ds, MASKS, 1e-3)
    rng = np.random.default_rng(912)
    G = (rng.uniform(size=(n, C)) < rng.uniform(0.1, 0.9, size=C)).astype(np.uint8)
    sums = tp.pairsums(Yg, torch.from_numpy(G).cuda(), sigma, nrow=nrow)
    torch.cuda.synchronize()
    S = sums.cpu().numpy()
    comps, _ = s.numpy()
    Yo = energy.invariant_masses(comps, MASKS) * 1e-3
    Psi = energy.psi_block(Yo, Yo, sigma)
    np.fill_diagonal(Psi, 0.0)
    Gf = G.astype(np.float64)
    V = Psi @ Gf
    want0 = np.einsum("ic,ic->c", Gf, V)
    assert np.all(np.abs(S[:, 0] - want0) <= 1e-5 * want0 + 1e-9)
    for q in range(nrow):
        wq = Gf[:, q] @ V
        assert np.all(np.abs(S[:, 1 + q] - wq) <= 1e-5 * wq + 1e-9), q


def _dense_check(tp, Yh, G, sigma, nrow, tol=1e-5):
    """Pair sums of float32 coordinates Yh [D][n] against the dense float64 psi matrix."""
    sums = tp.pairsums(torch.from_numpy(np.ascontiguousarray(Yh)).cuda(), torch.from_numpy(G).cuda(), sigma, nrow=nrow)
    torch.cuda.synchronize()
    S = sums.cpu().numpy()
    assert np.all(np.isfinite(S))
    Psi = energy.psi_block(Yh.astype(np.float64), Yh.astype(np.float64), sigma)
    np.fill_diagonal(Psi, 0.0)
    Gf = G.astype(np.float64)
    V = Psi @ Gf
    want0 = np.einsum("ic,ic->c", Gf, V)
    assert np.all(np.abs(S[:, 0] - want0) <= tol * want0 + 1e-9)
    for q in range(nrow):
        wq = Gf[:, q] @ V
        assert np.all(np.abs(S[:, 1 + q] - wq) <= tol * wq + 1e-9), q
    return S


def test_pair_sums_far_events(tp):
    """Events far from the centre (the mean of the first 256 events) in sigma units --
    beyond the range in which the matrix-core distances are accurate -- take direct
    float32 differences in every chunk of pairs that holds them: the sums match the dense
    float64 psi.  Far events are placed as rows of the first block, as columns of a late
    chunk, and as two far events close to each other (their pair's psi is large)."""
    n, C, sigma = 1300, 32, 0.3
    rng = np.random.default_rng(31)
    Yh = rng.normal(1.0, 0.3, size=(2, n)).astype(np.float32)
    G = (rng.uniform(size=(n, C)) < 0.5).astype(np.uint8)
    Yfar = Yh.copy()
    Yfar[:, n - 1] = 20.0                       # ~ (19 GeV / 0.3 GeV) * 0.85 = 54 scaled units
    Yfar[:, n - 2] = 20.05                      # close to the previous one: psi ~ 0.97
    Yfar[:, 5] = -40.0                          # a row of the first block
    Yfar[:, 700] = [1e4, -3e3]                  # very far: every psi with it underflows
    _dense_check(tp, Yfar, G, sigma, 1)
    _dense_check(tp, Yfar, G, sigma, 2)


def test_pair_sums_after_autotune(tp):
    """The per-stream range flag of the pair sums survives autotuning: pair sums with far
    events (the flag is set, then cleared by the safe form), two autotunes whose counter
    scratch grows (batches of 8 and 16 samples of 1024 bins), pair sums again on the same
    stream; both calls match the dense float64 psi.  (The autotuner once freed the flags
    when it grew its scratch, leaving the pair sums a freed flag.)"""
    n, C, sigma = 1300, 32, 0.3
    rng = np.random.default_rng(41)
    Yh = rng.normal(1.0, 0.3, size=(2, n)).astype(np.float32)
    Yh[:, 3] = 30.0
    G = (rng.uniform(size=(n, C)) < 0.5).astype(np.uint8)
    _dense_check(tp, Yh, G, sigma, 1)
    ch, s = sample(4099, 42)
    ds = tp.DeviceSample.from_sample(s)
    bn = tp.Binning([synth.abscos_axis(0, 32), synth.mass_axis((0, 1), 980.0, 1600.0, 32)])
    for copies in (8, 16):
        items = [(ds, tp.channel(ch.triple, ch.planes), bn, *tp.new_counts(bn)) for _ in range(copies)]
        tp.Batch(items).autotune(tp.TP_PREC_F64)
    _dense_check(tp, Yh, G, sigma, 1)
    _dense_check(tp, Yh, G, sigma, 2)


@pytest.mark.parametrize("sigma,far_min", [(0.15, 0.0), (0.04, 0.3)])
def test_pair_sums_lambda_b_masses(tp, sigma, far_min):
    """Lambda_b -> p K- pi+ pi- invariant masses (spreads of several GeV) against the dense
    float64 psi at sigma = 0.15 GeV and at sigma = 0.04 GeV, where about half of the events lie
    beyond the matrix-core range around the first 256 events' mean."""
    ch = synth.CHANNELS["Lb_pKpipi"]
    s = synth.generate(ch, 2051, 35)
    masks = [0b0011, 0b1001, 0b0110, 0b1100, 0b0111]
    Yg = tp.coords(tp.DeviceSample.from_sample(s), masks, 1e-3)
    comps, _ = s.numpy()
    Yo = energy.invariant_masses(comps, masks) * 1e-3
    yscale = np.sqrt(np.log2(np.e) / (2 * sigma ** 2))
    far = ((Yo - Yo[:, :256].mean(axis=1, keepdims=True)) ** 2).sum(axis=0) * yscale ** 2 > 1024
    print(f"[energy] Lambda_b masses at sigma {sigma}: {far.mean():.2f} of the events beyond the matrix-core "
          f"range", flush=True)
    assert far.mean() >= far_min
    rng = np.random.default_rng(36)
    G = (rng.uniform(size=(2051, 64)) < rng.uniform(0.1, 0.9, size=64)).astype(np.uint8)
    _dense_check(tp, Yg.cpu().numpy(), G, sigma, 2)


ALL_MASKS = [0b0011, 0b0101, 0b0110, 0b1001, 0b1010, 0b1100, 0b0111, 0b1011, 0b1101, 0b1110, 0b1111]


@pytest.mark.parametrize("D,C,nrow", [(1, 32, 0), (2, 128, 3), (3, 64, 2), (4, 128, 1), (6, 32, 3), (7, 64, 1),
                                      (8, 128, 2), (8, 32, 1)])
def test_raw_pair_sums_coordinate_counts(tp, D, C, nrow):
    """Pair sums against the dense float64 psi matrix for 1 to 8 coordinates per event (the
    distance operands hold D + 2 components, split into float16 slots, so every coordinate
    count has its own layout) and each row-weight reduction."""
    n = 1543
    ch, s = sample(n, 700 + D)
    masks = ALL_MASKS[:D]
    ds = tp.DeviceSample.from_sample(s)
    Yg = tp.coords(ds, masks, 1e-3)
    rng = np.random.default_rng(800 + D)
    G = (rng.uniform(size=(n, C)) < rng.uniform(0.1, 0.9, size=C)).astype(np.uint8)
    sums = tp.pairsums(Yg, torch.from_numpy(G).cuda(), 0.3, nrow=nrow)
    torch.cuda.synchronize()
    S = sums.cpu().numpy()
    comps, _ = s.numpy()
    Yo = energy.invariant_masses(comps, masks) * 1e-3
    Psi = energy.psi_block(Yo, Yo, 0.3)
    np.fill_diagonal(Psi, 0.0)
    Gf = G.astype(np.float64)
    V = Psi @ Gf
    want0 = np.einsum("ic,ic->c", Gf, V)
    assert np.all(np.abs(S[:, 0] - want0) <= 1e-5 * want0 + 1e-9)
    for q in range(nrow):
        wq = Gf[:, q] @ V
        assert np.all(np.abs(S[:, 1 + q] - wq) <= 1e-5 * wq + 1e-9), q


def test_T_at_scale_against_oracle(tp):
    """T of eq. (2) and of eq. (3) at n = 30000 events, where the permutation spread of T
    (~1e-5 at sigma = 0.3 GeV) is small against the three terms (~0.3 each): every
    column against the oracle's column pair sums (float64, one pass over the pairs).

    Tolerance from the pair sums' accuracy: the float32 tiles accumulate errors of
    random sign, the sums come out within ~1e-9 relative at sigma = 0.3 (an emulation
    of the float16 split and float32 accumulation on these coordinates); allowing
    1e-8 relative on every sum, |delta T| <= 1e-8 x (sum of the terms' magnitudes).
    The test checks that this tolerance is below 2 % of the permutation spread, so it
    tells a right T from a wrong one, and that every p-value decision (permutation T
    above the observed T) agrees where the two differ by more than twice the tolerance."""
    import oracle
    n, sigma, nperm = 30000, 0.3, 14
    ch = synth.CHANNELS["D0_KKpipi"]
    s = synth.generate(ch, n, 333, inj=synth.INJ_SGN)
    comps, tag = s.numpy()
    # the P-odd split of Sect. 5 ([I + IV] against [II + III]) from the oracle's classes
    cls = oracle.run(comps, tag, ch.triple, ch.planes, want_events=True)["cls"]
    assert np.all(cls < 4)
    lab = ((cls == 0) | (cls == 3)).astype(np.uint8)
    rng = np.random.default_rng(334)
    labels = [lab] + [rng.permutation(lab) for _ in range(nperm)]
    # eq. (3): the first 24000 events are the main samples, the last 6000 the
    # background samples, flavour X = the split above; its permutations shuffle the
    # flavour within the main and within the background events separately
    nm = 24000
    b3 = [(lab[:nm], lab[nm:])] + [(rng.permutation(lab[:nm]), rng.permutation(lab[nm:])) for _ in range(4)]
    # device: all-ones, observed split, permutations (eq. 2); main, background and the
    # triples (a, beta, a + beta) per flavour assignment (eq. 3)
    cols2 = np.zeros((n, 32), dtype=np.uint8)
    cols2[:, 0] = 1
    for k, l in enumerate(labels):
        cols2[:, 1 + k] = l
    main = np.r_[np.ones(nm), np.zeros(n - nm)].astype(np.uint8)
    cols3 = np.zeros((n, 32), dtype=np.uint8)
    cols3[:, 0], cols3[:, 1] = main, 1 - main
    triples = []
    for k, (fm, fb) in enumerate(b3):
        a = np.r_[fm, np.zeros(n - nm)].astype(np.uint8)
        beta = np.r_[np.zeros(nm), fb].astype(np.uint8)
        cols3[:, 2 + 3 * k], cols3[:, 3 + 3 * k], cols3[:, 4 + 3 * k] = a, beta, a + beta
        triples.append((2 + 3 * k, 3 + 3 * k, 4 + 3 * k))
    Yg = tp.coords(tp.DeviceSample.from_sample(s), MASKS, 1e-3)
    sums2 = tp.pairsums(Yg, torch.from_numpy(cols2).cuda(), sigma, nrow=1)
    sums3 = tp.pairsums(Yg, torch.from_numpy(cols3).cuda(), sigma, nrow=2)
    torch.cuda.synchronize()
    T2 = tp.energy_eq2(sums2, cols2.sum(axis=0), n, ones_row=0, ones_col=0)[1:1 + len(labels)]
    nx_m = [int(fm.sum()) for fm, _ in b3]
    nx_b = [int(fb.sum()) for _, fb in b3]
    b, b_bar = 0.25 * nx_m[0], 0.25 * (nm - nx_m[0])
    T3 = tp.energy_eq3(sums3, 0, 1, 0, 1, triples, nx_m[0], nm - nx_m[0], nx_b[0], (n - nm) - nx_b[0], b, b_bar)

    # oracle: one pass over the pairs for every set that eq. (2) and eq. (3) use
    Yo = energy.invariant_masses(comps, MASKS) * 1e-3
    sets = []
    for l in labels:
        sets += [l, 1 - l]
    for fm, fb in b3:
        sets += [np.r_[fm, 0 * fb], np.r_[1 - fm, 0 * fb], np.r_[0 * fm, fb], np.r_[0 * fm, 1 - fb]]
    M = energy.column_pair_sums(Yo, np.stack(sets, axis=1), sigma)
    want2, mag2 = [], []
    for k, l in enumerate(labels):
        a, c = 2 * k, 2 * k + 1
        nx = int(l.sum())
        want2.append(energy.T_eq2_columns(M, a, c, nx, n - nx))
        mag2.append(0.5 * M[a, a] / (nx * (nx - 1)) + 0.5 * M[c, c] / ((n - nx) * (n - nx - 1))
                    + M[a, c] / (nx * (n - nx)))
    want2, mag2 = np.array(want2), np.array(mag2)
    tol2 = 1e-8 * mag2
    spread2 = np.std(want2[1:])
    print(f"[energy at scale] eq2: spread {spread2:.3e}, tol {tol2.max():.3e}, "
          f"max |dT| {np.abs(np.array(T2) - want2).max():.3e}", flush=True)
    assert tol2.max() <= 0.02 * spread2
    assert np.all(np.abs(np.array(T2) - want2) <= tol2)
    sure = np.abs(want2[1:] - want2[0]) > 2 * tol2.max()
    assert np.array_equal((np.array(T2[1:]) > T2[0])[sure], (want2[1:] > want2[0])[sure])

    # eq. (3) from the same pair sums, each term with the paper's coefficient
    o = 2 * len(labels)
    want3, mag3 = [], []
    for k in range(len(b3)):
        cols = (o + 4 * k, o + 4 * k + 1, o + 4 * k + 2, o + 4 * k + 3)
        cnt = (nx_m[k], nm - nx_m[k], nx_b[k], (n - nm) - nx_b[k])
        want3.append(energy.T_eq3_columns(M, *cols, *cnt, b, b_bar))
        t1, t2, t3 = energy.T_eq3_columns(M, *cols, *cnt, b, b_bar, terms=True)
        mag3.append(sum(abs(t) for t in t1 + t2 + t3))
    want3, tol3 = np.array(want3), 1e-8 * np.array(mag3)
    spread3 = np.std(want3[1:])
    print(f"[energy at scale] eq3: spread {spread3:.3e}, tol {tol3.max():.3e}, "
          f"max |dT| {np.abs(np.array(T3[:len(b3)]) - want3).max():.3e}", flush=True)
    assert tol3.max() <= 0.02 * spread3
    assert np.all(np.abs(np.array(T3[:len(b3)]) - want3) <= tol3)
