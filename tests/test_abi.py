"""libtpasym loads, exports every entry point of include/tpasym.h, and its
host-only parts (validation, asymmetries, S_CP) behave.  CPU only: no call here
reaches the GPU (argument checks run before anything is enqueued)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import exact

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def tp():
    from paper_1612_04705_amd import tpasym
    if not os.path.exists(tpasym.LIB_PATH):
        from paper_1612_04705_amd import build
        build.build()
    tpasym.load()
    return tpasym


def header_functions():
    src = open(os.path.join(ROOT, "include", "tpasym.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tp_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(tp):
    lib = tp.load()
    names = header_functions()
    assert "tp_batch" in names and "tp_bin" in names and "tp_compute" in names and "tp_asym" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tp.exported_symbols())
    assert tp.version() == 10000


def test_asym_matches_exact_fractions(tp):
    rng = np.random.default_rng(5)
    rows = [[60, 40, 45, 55], [7, 0, 0, 0], [0, 0, 0, 0], [1, 1, 1, 1], [0, 3, 5, 0]]
    rows += rng.integers(0, 10 ** 9, size=(200, 4)).tolist()
    rows += rng.integers(0, 50, size=(50, 4)).tolist()
    rows += [[2 ** 40 + 3, 2 ** 40 - 7, 2 ** 39, 3 * 2 ** 38 + 1]]
    got = tp.asym(np.array(rows).ravel())
    for r, g in zip(rows, got):
        want = exact.asym_row(r)
        assert g["N"] == tuple(r)
        for k in tp.ASYM_KEYS:
            wv, ws = want[k]
            gv, gs = g[k]
            if wv is None:
                assert math.isnan(gv) and math.isnan(gs)
                continue
            assert abs(gv - float(wv)) <= 1e-15 * abs(float(wv)) + 1e-300, (r, k, gv, float(wv))
            assert abs(gs - ws) <= 1e-12 * ws + 1e-300, (r, k, gs, ws)
    assert got[2]["flags"] == 15 and got[1]["flags"] == 2 | 8


def test_scp_matches_oracle(tp):
    rng = np.random.default_rng(6)
    for mode in (0, 1):
        for nb in (1, 2, 5, 40, 1024):
            c = rng.integers(0, 5000, size=(nb + 1, 4))
            c[0] = c[1:].sum(axis=0)
            s, chi2, ndf, p = tp.scp(c.ravel(), mode)
            if mode == 0:
                x, xb = c[1:, 0] + c[1:, 1], c[1:, 2] + c[1:, 3]
            else:
                x, xb = c[1:, 0] + c[1:, 3], c[1:, 1] + c[1:, 2]
            ws, wchi2, wndf, wp = exact.scp([int(v) for v in x], [int(v) for v in xb])
            assert ndf == wndf
            np.testing.assert_allclose(s, ws, rtol=1e-13, atol=1e-15)
            assert chi2 == pytest.approx(wchi2, rel=1e-12)
            if nb > 1:
                assert p == pytest.approx(wp, rel=1e-9, abs=1e-300)


def _events(tp, n=16, dtype=0, ptr=0x100000):
    e = tp._Events()
    e.n = n
    e.dtype = dtype
    for k in range(16):
        e.p[k] = ptr + 64 * k
    e.tag = ptr + 4096
    return e


def _bn(tp, axes):
    return tp.Binning(axes)


def test_validation_errors_reach_no_device(tp):
    from paper_1612_04705_amd import synth
    lib = tp.load()
    ch = tp.channel((0, 1, 2), (0, 1, 2, 3))
    good = _bn(tp, [synth.absphi_axis(10)])
    cnt = ctypes.c_void_p(0x200000)
    st = ctypes.c_void_p(0x300000)

    def rc_bin(ev, chx, bnx, prec=0, counts=cnt, stats=st):
        return lib.tp_bin(ctypes.byref(ev) if ev is not None else None,
                          ctypes.byref(chx) if chx is not None else None,
                          ctypes.byref(bnx.b) if bnx is not None else None, prec, counts, stats, None)

    assert rc_bin(None, ch, good) == -1
    assert rc_bin(_events(tp), None, good) == -1
    assert rc_bin(_events(tp), ch, None) == -1
    assert rc_bin(_events(tp, n=-1), ch, good) == -1
    assert rc_bin(_events(tp, dtype=7), ch, good) == -1
    assert rc_bin(_events(tp, dtype=1), ch, good, prec=1) == -2      # F32 recheck needs float32
    assert rc_bin(_events(tp), ch, good, prec=5) == -1
    assert rc_bin(_events(tp), tp.channel((0, 0, 2)), good) == -1
    assert rc_bin(_events(tp), tp.channel((0, 1, 4)), good) == -1
    assert rc_bin(_events(tp), tp.channel((0, 1, 2), (0, 1, 1, 3)), good) == -1
    # identical particles: two distinct slots of 0..3; with a plane angle binned
    # they must sit at positions (0, 2) or (1, 3) of planes
    assert rc_bin(_events(tp), tp.channel((0, 1, 2), identical=(1, 1)), good) == -1
    assert rc_bin(_events(tp), tp.channel((0, 1, 2), identical=(1, 4)), good) == -1
    assert rc_bin(_events(tp), tp.channel((0, 1, 2), identical=(1, -1)), good) == -1
    assert rc_bin(_events(tp), tp.channel((0, 1, 2), identical=(0, 1)), good) == -2
    assert rc_bin(_events(tp), tp.channel((0, 1, 2), (0, 1, 3, 2), identical=(1, 3)), good) == -2
    e = _events(tp)
    e.p[5] = None
    assert rc_bin(e, ch, good) == -1
    assert rc_bin(_events(tp), ch, good, counts=None) == -1
    bad_phi = synth.Axis(synth.AXIS_ABSPHI, np.array([1.0, 0.3, 0.5, -1.0]))
    assert rc_bin(_events(tp), ch, _bn(tp, [bad_phi])) == -1
    short_phi = synth.Axis(synth.AXIS_ABSPHI, np.array([0.9, 0.0, -1.0]))
    assert rc_bin(_events(tp), ch, _bn(tp, [short_phi])) == -1
    bad_mass = synth.Axis(synth.AXIS_MASS, np.array([1.0, 3.0, 2.0]), 0b11)
    assert rc_bin(_events(tp), ch, _bn(tp, [bad_mass])) == -1
    one_slot = synth.Axis(synth.AXIS_MASS, np.array([1.0, 2.0]), 0b1)
    assert rc_bin(_events(tp), ch, _bn(tp, [one_slot])) == -1
    neg_mass = synth.Axis(synth.AXIS_MASS, np.array([-1.0, 2.0]), 0b11)
    assert rc_bin(_events(tp), ch, _bn(tp, [neg_mass])) == -1
    bad_cos = synth.Axis(synth.AXIS_ABSCOS, np.array([0.0, 0.5, 0.9]), 0)
    assert rc_bin(_events(tp), ch, _bn(tp, [bad_cos])) == -1
    nan_edge = synth.Axis(synth.AXIS_MASS, np.array([1.0, np.nan, 3.0]), 0b11)
    assert rc_bin(_events(tp), ch, _bn(tp, [nan_edge])) == -1
    two_phi = _bn(tp, [synth.absphi_axis(4), synth.absphi_axis(4)])
    assert rc_bin(_events(tp), ch, two_phi) == -1
    big = _bn(tp, [synth.mass_axis((0, 1), 0, 1, 64), synth.mass_axis((2, 3), 0, 1, 32)])
    assert rc_bin(_events(tp), ch, big) == -5
    assert b"1024" in lib.tp_strerror(-5)
    # tp_compute needs cls_out; tp_batch checks its list
    assert lib.tp_compute(ctypes.byref(_events(tp)), ctypes.byref(ch), 0, None, None, st, None) == -1
    assert lib.tp_batch(None, 3, 0, None, 0, None) == -1
    assert lib.tp_batch(None, 0, 0, None, 4, None) == -1
    assert lib.tp_asym(None, 1, None) == -1
    assert lib.tp_scp(None, 1, 0, None, None, None, None) == -1


def test_energy_entry_points_validate_before_any_launch(tp):
    lib = tp.load()
    P = ctypes.c_void_p
    Y, G, S = P(0x200000), P(0x300000), P(0x400000)

    def ps(coords=Y, dims=5, ld=1000, n=1000, sigma=0.3, cols=G, ncols=32, nrow=1, sums=S):
        return lib.tp_pairsums(coords, dims, ld, n, sigma, cols, ncols, nrow, sums, None)

    assert ps(coords=None) == -1 and ps(cols=None) == -1 and ps(sums=None) == -1
    assert ps(dims=0) == -5 and ps(dims=9) == -5
    assert ps(n=-1) == -5 and ps(ld=999) == -1
    assert ps(ncols=48) == -1 and ps(ncols=256) == -1
    assert ps(nrow=4) == -5 and ps(nrow=-1) == -5
    assert ps(cols=P(0x300001)) == -1                      # columns must be 16-byte aligned
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        assert ps(sigma=bad) == -1
    assert ps(n=1, ld=1) == 0                              # fewer than two events: nothing to do
    e = _events(tp, n=1000)
    m = (ctypes.c_int32 * 5)(3, 9, 6, 12, 13)

    def co(ev=e, masks=m, ncoord=5, scale=1e-3, relabel=0, out=Y, ld=1000):
        return lib.tp_coords(ctypes.byref(ev) if ev is not None else None, masks, ncoord, scale, relabel, out, ld,
                             None)

    assert co(ev=None) == -1 and co(out=None) == -1
    assert co(relabel=2) == -1
    assert co(ncoord=0) == -5 and co(ncoord=9) == -5
    assert co(masks=(ctypes.c_int32 * 5)(3, 9, 0, 12, 13)) == -1
    assert co(masks=(ctypes.c_int32 * 5)(3, 9, 16, 12, 13)) == -1
    assert co(scale=0.0) == -1 and co(ld=999) == -1
    assert co(ev=_events(tp, n=0)) == 0


def test_energy_host_forms_vanish_when_psi_is_one(tp):
    # psi = 1 for every pair: every ordered-pair sum is a product of counts, and
    # both eq. (2) and eq. (3) reduce to 0 (the b(b+1) coefficient of eq. (3) is
    # what makes its background brackets cancel)
    rng = np.random.default_rng(9)
    n, C = 1000, 32
    G = (rng.uniform(size=(n, C)) < 0.4).astype(np.int64)
    G[:, 0] = 1
    k = G.sum(axis=0)
    S = np.zeros((C, 2))
    S[:, 0] = k * (k - 1)
    S[:, 1] = (n - 1) * k                                      # sum_i sum_{j != i} 1 * G_jc
    T = tp.energy_eq2(S, k, n, ones_row=0, ones_col=0)
    assert np.all(np.abs(T[1:]) < 1e-12)
    # eq. (3): main rows 0..599, background rows 600..999; flavour columns a, beta, gamma
    nm = 600
    main = np.r_[np.ones(nm), np.zeros(n - nm)]
    bkg = 1 - main
    cols = [main, bkg]
    triples = []
    for t in range(3):
        fa = (rng.uniform(size=n) < 0.5) * main
        fb = (rng.uniform(size=n) < 0.5) * bkg
        triples.append((len(cols), len(cols) + 1, len(cols) + 2))
        cols += [fa, fb, fa + fb]
    Gc = np.stack(cols, axis=1)
    kk = Gc.sum(axis=0)
    S3 = np.zeros((Gc.shape[1], 3))
    S3[:, 0] = kk * (kk - 1)                                   # sum_{i != j} G_ic G_jc
    for q in range(2):                                         # sum_{i != j} G_iq G_jc
        S3[:, 1 + q] = kk[q] * kk - Gc[:, q] @ Gc
    for (ca, cb, cg) in triples:
        nx, nxb = int(kk[ca]), nm - int(kk[ca])
        bx, bxb = int(kk[cb]), n - nm - int(kk[cb])
        T3 = tp.energy_eq3(S3, 0, 1, 0, 1, [(ca, cb, cg)], nx, nxb, bx, bxb, 0.3 * nx, 0.3 * nxb)
        assert abs(T3[0]) < 1e-12


def test_binding_refuses_host_tensors(tp):
    # the kernels take raw device pointers: host memory must be refused by the binding
    import torch
    from paper_1612_04705_amd import synth
    s = synth.generate(synth.CHANNELS["D0_KKpipi"], 64, 1)
    ds = tp.DeviceSample([s.comps[a][b] for a in range(4) for b in range(4)], s.tag)   # host tensors
    with pytest.raises(tp.TPError):
        ds.events()
    with pytest.raises(tp.TPError):
        tp.pairsums(torch.zeros((5, 64)), torch.zeros((64, 32), dtype=torch.uint8), 0.3)
    with pytest.raises(tp.TPError):      # Y narrower than the columns
        tp.pairsums(torch.zeros((5, 10)), torch.zeros((64, 32), dtype=torch.uint8), 0.3)
    with pytest.raises(tp.TPError):      # wrong sums shape
        tp.pairsums(torch.zeros((5, 64)), torch.zeros((64, 32), dtype=torch.uint8), 0.3,
                    sums=torch.zeros((32, 3), dtype=torch.float64))


def test_energy_eq2_degenerate_samples_give_nan(tp):
    # a column whose sample or complement has fewer than two events has no T
    n = 10
    S = np.ones((4, 2))
    nx = np.array([n, 1, n - 1, 5])          # all ones (complement empty), one event, one left out, fine
    T = tp.energy_eq2(S, nx, n)
    assert np.isnan(T[0]) and np.isnan(T[1]) and np.isnan(T[2]) and not np.isnan(T[3])
    # bad indices are refused
    lib = tp.load()
    P = ctypes.POINTER
    Sc = np.ascontiguousarray(S)
    nxc = np.ascontiguousarray(nx.astype(np.int64))
    out = np.zeros(4)
    assert lib.tp_energy_eq2(Sc.ctypes.data_as(P(ctypes.c_double)), 4, 1, 1, 0,
                             nxc.ctypes.data_as(P(ctypes.c_int64)), n, out.ctypes.data_as(P(ctypes.c_double))) == -1
    assert lib.tp_energy_eq2(Sc.ctypes.data_as(P(ctypes.c_double)), 4, 1, 0, 4,
                             nxc.ctypes.data_as(P(ctypes.c_int64)), n, out.ctypes.data_as(P(ctypes.c_double))) == -1


def test_noalloc_limits_checked_before_the_device(tp):
    """tp_bin_noalloc validates like tp_bin and rejects, before any device call, a call
    beyond its scratch array: more than 2^22 events or more than 384 doubles of edges."""
    from paper_1612_04705_amd import synth
    lib = tp.load()
    ch = tp.channel((0, 1, 2), (0, 1, 2, 3))
    good = _bn(tp, [synth.absphi_axis(10)])
    cnt = ctypes.c_void_p(0x200000)
    st = ctypes.c_void_p(0x300000)

    def rc(ev, bnx):
        return lib.tp_bin_noalloc(ctypes.byref(ev), ctypes.byref(ch), ctypes.byref(bnx.b), 0, cnt, st, None)

    assert rc(_events(tp, n=(1 << 22) + 1), good) == -5
    wide = synth.Axis(synth.AXIS_MASS, np.linspace(1000.0, 5000.0, 201), 0b1001)
    assert rc(_events(tp), _bn(tp, [wide])) == -5
    assert "384" in tp.load().tp_strerror(-5).decode()
    assert rc(_events(tp, n=-1), good) == -1
    assert rc(_events(tp, dtype=7), good) == -1
    assert lib.tp_bin_noalloc(ctypes.byref(_events(tp)), ctypes.byref(ch), ctypes.byref(good.b), 0, None, st,
                              None) == -1


def test_empty_samples_are_no_work(tp):
    """A sample of n = 0 events may carry NULL pointers and is no work for every
    entry point: each returns TP_OK before any device call (here, with no GPU, a
    device call would fail).  tp_batch leaves empty samples out of its plan, so a
    batch of only empty samples launches nothing (graph flag or not), and
    tp_autotune of such a batch returns the default shape."""
    from paper_1612_04705_amd import synth
    lib = tp.load()
    ch = tp.channel((0, 1, 2), (0, 1, 2, 3))
    bins = [_bn(tp, [synth.absphi_axis(10)]), _bn(tp, [synth.abscos_axis(0, 5), synth.absphi_axis(10)]), _bn(tp, [])]
    cnt = ctypes.c_void_p(0x200000)
    st = ctypes.c_void_p(0x300000)
    def empty(dtype):
        e = _events(tp, n=0, dtype=dtype)
        for k in range(16):
            e.p[k] = None
        e.tag = None
        return e

    for dtype in (0, 1):
        e = empty(dtype)
        assert lib.tp_bin(ctypes.byref(e), ctypes.byref(ch), ctypes.byref(bins[0].b), 0, cnt, st, None) == 0
        assert lib.tp_bin_noalloc(ctypes.byref(e), ctypes.byref(ch), ctypes.byref(bins[0].b), 0, cnt, st,
                                  None) == 0
        assert lib.tp_compute(ctypes.byref(e), ctypes.byref(ch), 0, cnt, None, st, None) == 0
        m = (ctypes.c_int32 * 2)(0b0011, 0b1100)
        assert lib.tp_coords(ctypes.byref(e), m, 2, 1.0, 0, cnt, 0, None) == 0
        arr = (tp._Sample * 3)()
        for i, bn in enumerate(bins):
            arr[i].ev = e
            arr[i].ch = ch
            arr[i].bn = bn.b
            arr[i].counts = 0x200000 + 4096 * i
            arr[i].stats = 0x300000 + 4096 * i
        for flags in (0, 1):
            assert lib.tp_batch(arr, 3, 0, None, flags, None) == 0
        t = tp.Tuning()
        assert lib.tp_autotune(arr, 3, 0, None, ctypes.byref(t)) == 0
        assert (t.block, t.wg_per_cu, t.lds_copies, t.unroll) == (256, 4, 4, 1)
    e = empty(0)
    assert lib.tp_probe_f32(ctypes.byref(e), ctypes.byref(ch), cnt, cnt, cnt, cnt, None) == 0
    # validation still applies to an empty sample
    assert lib.tp_bin(ctypes.byref(empty(7)), ctypes.byref(ch), ctypes.byref(bins[0].b), 0, cnt, st, None) == -1
    assert lib.tp_bin(ctypes.byref(empty(0)), ctypes.byref(ch), ctypes.byref(bins[0].b), 0, None, st, None) == -1


def test_compute_output_checks(tp):
    """tp_compute: with events, cls_out is required (NULL cls_out or no output at all
    is TP_EINVAL before any device call); with none, NULL outputs are accepted."""
    lib = tp.load()
    ch = tp.channel((0, 1, 2), (0, 1, 2, 3))
    st = ctypes.c_void_p(0x300000)
    ct = ctypes.c_void_p(0x400000)
    assert lib.tp_compute(ctypes.byref(_events(tp)), ctypes.byref(ch), 0, None, ct, st, None) == -1
    assert lib.tp_compute(ctypes.byref(_events(tp)), ctypes.byref(ch), 0, None, None, st, None) == -1
    assert lib.tp_compute(ctypes.byref(_events(tp)), ctypes.byref(ch), 0, ct, None, None, None) == -1
    assert lib.tp_compute(ctypes.byref(_events(tp, n=0)), ctypes.byref(ch), 0, None, None, st, None) == 0
