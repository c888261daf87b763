"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Counts and statistics must be bit-exact; asymmetries within 1e-12 relative.
Sizes are small enough for the oracle to finish in seconds while spanning many
tiles, several workgroups and ragged tails.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import exact
from paper_1612_04705_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    from paper_1612_04705_amd import tpasym
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    tpasym.load()
    return tpasym


def u64(t):
    return t.cpu().numpy().view(np.uint64).astype(object)


def gpu_bin(tp, sample, ch, axes, prec, tuning=None, graph=False):
    ds = tp.DeviceSample.from_sample(sample)
    bn = tp.Binning(axes)
    counts, stats = tp.new_counts(bn)
    if tuning is None and not graph:
        tp.bin(ds, tp.channel(ch.triple, ch.planes), bn, prec, counts, stats)
    else:
        b = tp.Batch([(ds, tp.channel(ch.triple, ch.planes), bn, counts, stats)])
        b.run(prec, tuning, graph)
    torch.cuda.synchronize()
    c = [int(x) for x in u64(counts)]
    return [c[4 * r:4 * r + 4] for r in range(bn.nrows)], [int(x) for x in u64(stats)]


def check(tp, sample, ch, axes, precisions=None, label=""):
    comps, tag = sample.numpy()
    want = oracle.run(comps, tag, ch.triple, ch.planes, axes)
    if precisions is None:
        precisions = [tp.TP_PREC_F64] + ([tp.TP_PREC_F32_RECHECK] if comps.dtype == np.float32 else [])
    out = []
    for prec in precisions:
        counts, stats = gpu_bin(tp, sample, ch, axes, prec)
        print(f"[parity] {label} prec={prec} n={sample.n} stats={stats}", flush=True)
        assert stats[6] == 0, "unresolved events"
        assert counts == want["counts"], label
        assert stats[:4] == want["stats"], label
        out.append((counts, stats))
    return want, out


@pytest.mark.parametrize("workload,scale", [("lb_ppipipi_f64_1e5", 0.2), ("lb_ppipipi_1e7_phi12", 0.003),
                                            ("lb_pkpipi_1e8_phi10xm8", 0.0004),
                                            ("d0_kkpipi_5e8_m32x32", 0.0001)])
def test_workload_shapes(tp, workload, scale):
    for spec in synth.workload_specs(workload, scale):
        s = synth.make_sample(spec)
        check(tp, s, spec.channel, spec.axes, label=workload)


def test_batch_workload_shape(tp):
    specs = synth.workload_specs("lb_batch64_1e3to1e7", 0.002)
    items, wants = [], []
    for spec in specs:
        s = synth.make_sample(spec)
        comps, tag = s.numpy()
        wants.append(oracle.run(comps, tag, spec.channel.triple, spec.channel.planes, spec.axes))
        ds = tp.DeviceSample.from_sample(s)
        bn = tp.Binning(spec.axes)
        counts, stats = tp.new_counts(bn)
        items.append((ds, tp.channel(spec.channel.triple, spec.channel.planes), bn, counts, stats))
    b = tp.Batch(items)
    for prec in (tp.TP_PREC_F32_RECHECK, tp.TP_PREC_F64):
        b.autotune(prec)      # later runs without a shape take the per-scheme tuned ones
        for graph, reps in ((False, 1), (True, 3)):
            for it in items:
                it[3].zero_()
                it[4].zero_()
            for _ in range(reps):
                b.run(prec, None, graph)
            torch.cuda.synchronize()
            for (ds, ch, bn, counts, stats), w in zip(items, wants):
                c = [int(x) for x in u64(counts)]
                c = [c[4 * r:4 * r + 4] for r in range(bn.nrows)]
                st = [int(x) for x in u64(stats)]
                assert c == [[reps * v for v in row] for row in w["counts"]], (prec, graph)
                assert st[:4] == [reps * v for v in w["stats"]]
                assert st[6] == 0


def test_batch_with_six_scheme_groups(tp):
    """A batch of six binning schemes (|Phi|, |Phi| x mass, |cos theta| x |Phi|, mass,
    |cos theta| and none): six scheme groups, launched on parallel branches (more groups
    than side streams, so branches are shared), eager and as a graph replayed three
    times with eager work between the replays, every run against the oracle."""
    ch = synth.CHANNELS["Lb_pKpipi"]
    schemes = [[synth.absphi_axis(10)], [synth.absphi_axis(10), synth.lb_mass03_axis(ch)],
               [synth.abscos_axis(0, 5), synth.absphi_axis(10)], [synth.lb_mass03_axis(ch, 6)],
               [synth.abscos_axis(0, 4)], []]
    items, wants = [], []
    for k in range(12):
        axes = schemes[k % 6]
        s = synth.generate(ch, 3000 + 1777 * k, 900 + k, inj=synth.INJ_SIN2)
        comps, tag = s.numpy()
        wants.append(oracle.run(comps, tag, ch.triple, ch.planes, axes))
        bn = tp.Binning(axes)
        items.append((tp.DeviceSample.from_sample(s), tp.channel(ch.triple, ch.planes), bn, *tp.new_counts(bn)))
    b = tp.Batch(items)

    def verify(reps, label):
        torch.cuda.synchronize()
        for (ds, _, bn, counts, stats), w in zip(items, wants):
            c = [int(x) for x in u64(counts)]
            c = [c[4 * r:4 * r + 4] for r in range(bn.nrows)]
            st = [int(x) for x in u64(stats)]
            assert c == [[reps * v for v in row] for row in w["counts"]], label
            assert st[:4] == [reps * v for v in w["stats"]], label
            assert st[6] == 0, label

    for prec in (tp.TP_PREC_F32_RECHECK, tp.TP_PREC_F64):
        for it in items:
            it[3].zero_()
            it[4].zero_()
        b.run(prec, None, False)
        n = 1
        verify(n, ("eager", prec))
        for k in range(3):
            b.run(prec, None, True)
            n += 1
            verify(n, ("graph replay", k, prec))
            b.run(prec, None, False)          # eager work between the replays
            n += 1
            verify(n, ("eager after replay", k, prec))


def test_release_and_reuse(tp):
    """tp_release frees every device resource the library holds (plans, graphs,
    workspaces, side streams and their events, the pair-sum flags); the next calls
    recreate them.  A three-scheme batch (parallel branches), eager and graphed, and a
    pair-sum launch before and after a release, each against the oracle."""
    from oracle import energy
    ch = synth.CHANNELS["Lb_ppipipi"]
    schemes = [[synth.absphi_axis(10)], [synth.absphi_axis(10), synth.lb_mass03_axis(ch)],
               [synth.abscos_axis(0, 5), synth.absphi_axis(10)]]
    samples = [synth.generate(ch, 4000 + 999 * k, 950 + k, inj=synth.INJ_SIN) for k in range(3)]
    wants = []
    for s_, axes in zip(samples, schemes):
        comps, tag = s_.numpy()
        wants.append(oracle.run(comps, tag, ch.triple, ch.planes, axes))
    rng = np.random.default_rng(951)
    Y = rng.normal(1.0, 0.3, size=(3, 700)).astype(np.float32)
    G = (rng.uniform(size=(700, 32)) < 0.5).astype(np.uint8)
    Psi = energy.psi_block(Y.astype(np.float64), Y.astype(np.float64), 0.3)
    np.fill_diagonal(Psi, 0.0)
    want_sums = np.einsum("ic,ic->c", G.astype(np.float64), Psi @ G.astype(np.float64))

    def once(label):
        items = []
        for s_, axes in zip(samples, schemes):
            bn = tp.Binning(axes)
            items.append((tp.DeviceSample.from_sample(s_), tp.channel(ch.triple, ch.planes), bn, *tp.new_counts(bn)))
        b = tp.Batch(items)
        b.run(tp.TP_PREC_F32_RECHECK, None, False)
        b.run(tp.TP_PREC_F32_RECHECK, None, True)
        torch.cuda.synchronize()
        for (ds, _, bn, counts, stats), w in zip(items, wants):
            c = [int(x) for x in u64(counts)]
            c = [c[4 * r:4 * r + 4] for r in range(bn.nrows)]
            assert c == [[2 * v for v in row] for row in w["counts"]], label
            assert [int(x) for x in u64(stats)][:4] == [2 * v for v in w["stats"]], label
        sums = tp.pairsums(torch.from_numpy(Y).cuda(), torch.from_numpy(G).cuda(), 0.3, nrow=0)
        torch.cuda.synchronize()
        got = sums.cpu().numpy()[:, 0]
        assert np.all(np.abs(got - want_sums) <= 1e-5 * want_sums + 1e-9), label

    once("before release")
    torch.cuda.synchronize()
    tp.release()
    once("after release")


def test_empty_samples(tp):
    """Samples of no events (empty device tensors: NULL data pointers) are no work:
    tp_bin, tp_compute and a batch of only such samples leave counts and statistics as
    they are, eager and as a graph; in a batch beside non-empty samples of three
    schemes (one scheme holding only an empty sample) the others match the oracle,
    eager and on graph replays, and autotuning that batch works."""
    ch = synth.CHANNELS["Lb_ppipipi"]
    dev = torch.device("cuda")

    def empty(dtype=torch.float32):
        return tp.DeviceSample([torch.empty(0, dtype=dtype, device=dev) for _ in range(16)],
                               torch.empty(0, dtype=torch.int8, device=dev))

    def sentinel(bn):
        counts, stats = tp.new_counts(bn)
        counts.fill_(7)
        stats.fill_(3)
        return counts, stats

    def untouched(counts, stats, label):
        assert bool((counts == 7).all()) and bool((stats == 3).all()), label

    chan = tp.channel(ch.triple, ch.planes)
    bn = tp.Binning([synth.absphi_axis(10)])
    for dtype, prec in ((torch.float32, tp.TP_PREC_F32_RECHECK), (torch.float64, tp.TP_PREC_F64)):
        e = empty(dtype)
        counts, stats = sentinel(bn)
        tp.bin(e, chan, bn, prec, counts, stats, check=False)   # the sentinel counts 3 unresolved
        cls, ct, st = tp.compute(e, chan, prec)
        torch.cuda.synchronize()
        untouched(counts, stats, ("tp_bin", dtype))
        assert cls.numel() == 0 and int(st.abs().sum()) == 0
        items = [(empty(dtype), chan, b, *sentinel(b))
                 for b in (bn, tp.Binning([synth.abscos_axis(0, 5), synth.absphi_axis(10)]), tp.Binning([]))]
        b = tp.Batch(items)
        for graph in (False, True, True):
            b.run(prec, None, graph)
        t = b.autotune(prec)
        assert (t.block, t.wg_per_cu, t.lds_copies, t.unroll) == (256, 4, 4, 1)
        torch.cuda.synchronize()
        for it in items:
            untouched(it[3], it[4], ("all-empty batch", dtype))

    schemes = [[synth.absphi_axis(10)], [synth.abscos_axis(0, 5), synth.absphi_axis(10)],
               [synth.lb_mass03_axis(ch)]]
    items, wants = [], []
    for k, axes in enumerate([schemes[0], schemes[1], schemes[0], schemes[2], schemes[1]]):
        bnk = tp.Binning(axes)
        if k in (2, 3):             # scheme 2 holds only this empty sample
            items.append((empty(), chan, bnk, *sentinel(bnk)))
            wants.append(None)
            continue
        s = synth.generate(ch, 2000 + 1311 * k, 970 + k, inj=synth.INJ_SIN)
        comps, tag = s.numpy()
        wants.append(oracle.run(comps, tag, ch.triple, ch.planes, axes))
        items.append((tp.DeviceSample.from_sample(s), chan, bnk, *tp.new_counts(bnk)))
    b = tp.Batch(items)
    b.autotune(tp.TP_PREC_F32_RECHECK)
    n = 0
    for graph in (False, True, True, False):
        b.run(tp.TP_PREC_F32_RECHECK, None, graph)
        n += 1
        torch.cuda.synchronize()
        for (ds, _, bnk, counts, stats), w in zip(items, wants):
            if w is None:
                untouched(counts, stats, ("empty in a mixed batch", graph, n))
                continue
            c = [int(x) for x in u64(counts)]
            c = [c[4 * r:4 * r + 4] for r in range(bnk.nrows)]
            assert c == [[n * v for v in row] for row in w["counts"]], (graph, n)
            assert [int(x) for x in u64(stats)][:4] == [n * v for v in w["stats"]], (graph, n)


@pytest.mark.parametrize("chname,gamma", [("Lb_pKKK", 1e4), ("Lb_ppipipi", 3e3)])
def test_abscos_absphi_at_high_boost(tp, chname, gamma):
    """|cos theta| x |Phi| bins at boosts of 3e3 and 1e4, where the first pass defers most
    events to the later tiers (double words, then exact integers): counts bit-exact against
    the oracle, eager and as a graph, with thousands of events through those tiers."""
    ch = synth.CHANNELS[chname]
    axes = [synth.abscos_axis(0, 5), synth.absphi_axis(10)]
    s = synth.generate(ch, 8000, 61, fixed_gamma=gamma)
    comps, tag = s.numpy()
    want = oracle.run(comps, tag, ch.triple, ch.planes, axes)
    for graph in (False, True):
        counts, stats = gpu_bin(tp, s, ch, axes, tp.TP_PREC_F32_RECHECK, graph=graph)
        print(f"[parity] {chname} gamma={gamma} graph={graph} stats={stats}", flush=True)
        assert stats[5] > 100 and stats[6] == 0
        assert counts == want["counts"] and stats[:4] == want["stats"]


def test_compute_per_event_classes(tp):
    ch = synth.CHANNELS["Lb_ppipipi"]
    s = synth.generate(ch, 30011, 41)
    comps, tag = s.numpy()
    want = oracle.run(comps, tag, ch.triple, ch.planes, want_events=True)
    ds = tp.DeviceSample.from_sample(s)
    for prec in (tp.TP_PREC_F64, tp.TP_PREC_F32_RECHECK):
        cls, ct, stats = tp.compute(ds, tp.channel(ch.triple, ch.planes), prec)
        torch.cuda.synchronize()
        g = cls.cpu().numpy()
        assert np.array_equal(g, want["cls"])
        ctv = ct.cpu().numpy()
        ok = want["cls"] < 4
        # C_T^inv = M * C_T: same sign as the oracle's rest-frame value
        assert np.array_equal(np.sign(ctv[ok]), np.sign(want["ct"][ok]))


def test_asymmetries_from_gpu_counts(tp):
    spec = synth.workload_specs("lb_ppipipi_1e7_phi12", 0.003)[0]
    s = synth.make_sample(spec)
    want, outs = check(tp, s, spec.channel, spec.axes)
    counts = outs[0][0]
    got = tp.asym(np.array(counts).ravel())
    for row, g in zip(counts, got):
        w = exact.asym_row(row)
        for k in tp.ASYM_KEYS:
            if w[k][0] is None:
                assert math.isnan(g[k][0])
            else:
                assert abs(g[k][0] - float(w[k][0])) <= 1e-12 * abs(float(w[k][0])) + 1e-300
                assert abs(g[k][1] - w[k][1]) <= 1e-12 * w[k][1] + 1e-300


@pytest.mark.parametrize("n", [1, 3, 4, 63, 64, 65, 255, 1027, 4099])
def test_ragged_sizes(tp, n):
    ch = synth.CHANNELS["Lb_pKpipi"]
    s = synth.generate(ch, n, 50 + n)
    check(tp, s, ch, [synth.absphi_axis(10), synth.lb_mass03_axis(ch)], label=f"n={n}")


def test_unaligned_views_take_scalar_path(tp):
    ch = synth.CHANNELS["Lb_pKpipi"]
    s = synth.generate(ch, 5001, 60)
    axes = [synth.absphi_axis(10), synth.lb_mass03_axis(ch)]
    comps, tag = s.numpy()
    want = oracle.run(comps[:, :, 1:], tag[1:], ch.triple, ch.planes, axes)
    big = [torch.cat([torch.zeros(1, dtype=t.dtype), t]).cuda() for t in s.arrays()]
    ds = tp.DeviceSample([t[2:] for t in big], torch.cat([torch.zeros(1, dtype=torch.int8), s.tag]).cuda()[2:])
    bn = tp.Binning(axes)
    for prec in (tp.TP_PREC_F64, tp.TP_PREC_F32_RECHECK):
        counts, stats = tp.bin(ds, tp.channel(ch.triple, ch.planes), bn, prec)
        torch.cuda.synchronize()
        c = [int(x) for x in u64(counts)]
        assert [c[4 * r:4 * r + 4] for r in range(bn.nrows)] == want["counts"]


def test_adversarial_inputs(tp):
    from test_oracle_pins import _load_handbuilt, _as_sample
    rows = _load_handbuilt()
    hb, hbt = _as_sample(rows)
    ch = synth.CHANNELS["Lb_pKpipi"]
    s = synth.generate(ch, 3000, 61)
    comps, tag = s.numpy()
    c = comps.copy()
    t = tag.copy()
    c[:, 3, :300] = 0.0                         # coplanar -> zero class (exact tier)
    c[1, 2, 300] = np.nan
    c[2, 0, 301] = np.inf
    t[302] = 9
    c[:, 0, 303] = 0.0                          # no rest frame
    c[0, 1, 304] = np.float32(1e-30)
    c[2, :, 305] = c[1, :, 305]                 # two equal daughters -> zero
    reps = np.concatenate([np.tile(hb, (1, 1, 40)), c], axis=2)
    rept = np.concatenate([np.tile(hbt, 40), t])
    samp = synth.Sample(ch, [[torch.from_numpy(np.ascontiguousarray(reps[a, b])) for b in range(4)]
                             for a in range(4)], torch.from_numpy(rept))
    for axes in ([synth.absphi_axis(12)], [synth.absphi_axis(10), synth.lb_mass03_axis(ch)],
                 [synth.abscos_axis(0, 5), synth.absphi_axis(10)],
                 [synth.Axis(synth.AXIS_MASS, np.array([5.0, 6.0, 7.0, 5000.0]), 0b1001)]):
        want, outs = check(tp, samp, synth.Channel("t", 0, (0,) * 4, (0, 1, 2)), axes, label="adversarial")
        for counts, stats in outs:
            assert stats[5] > 0          # the exact tier was used


@pytest.mark.parametrize("gamma", [300.0, 3000.0, 1.0e4])
def test_high_boost_needs_recheck(tp, gamma):
    ch = synth.CHANNELS["D0_KKpipi"]
    s = synth.generate(ch, 20000, 62, fixed_gamma=gamma)
    want, outs = check(tp, s, ch, [synth.mass_axis((0, 1), 987.354, 1585.7, 32),
                                   synth.mass_axis((2, 3), 279.14, 877.486, 32)], label=f"gamma={gamma}")
    # float32 path at high boost needs the float64 recheck of the sign for some events
    assert outs[1][1][4] > 0


def test_tuning_invariance(tp):
    spec = synth.workload_specs("d0_kkpipi_5e8_m32x32", 0.00005)[0]
    s = synth.make_sample(spec)
    ref = None
    for block in (256, 512):
        for wpc in (1, 3, 8):
            for copies in (1, 2, 4):
                t = tp.Tuning(block, wpc, copies, 1)
                got = gpu_bin(tp, s, spec.channel, spec.axes, tp.TP_PREC_F32_RECHECK, tuning=t)
                if ref is None:
                    ref = got
                assert got == ref, t.as_dict()


def test_fine_ranges_match_the_oracle(tp):
    """16 and 32 workgroups per CU (the finest launch shapes the autotuner tries) on a
    sample large enough that every workgroup of the grid gets its own range of several
    tiles: counts bit-exact against the oracle for each shape."""
    spec = synth.workload_specs("d0_kkpipi_5e8_m32x32", 0.0084)[0]
    s = synth.make_sample(spec)
    comps, tag = s.numpy()
    want = oracle.run(comps, tag, spec.channel.triple, spec.channel.planes, spec.axes)
    assert s.n > 256 * 32 * 256     # more tiles than workgroups at 32 per CU
    for wpc in (8, 16, 32):
        for copies, epl in ((1, 1), (4, 2)):
            t = tp.Tuning(256, wpc, copies, epl)
            counts, stats = gpu_bin(tp, s, spec.channel, spec.axes, tp.TP_PREC_F32_RECHECK, tuning=t)
            print(f"[parity] fine ranges {t.as_dict()} n={s.n}", flush=True)
            assert counts == want["counts"], t.as_dict()
            assert stats[:4] == want["stats"] and stats[6] == 0, t.as_dict()


def test_chunked_equals_whole(tp):
    spec = synth.workload_specs("lb_pkpipi_1e8_phi10xm8", 0.0003)[0]
    s = synth.make_sample(spec)
    ch = tp.channel(spec.channel.triple, spec.channel.planes)
    bn = tp.Binning(spec.axes)
    whole = gpu_bin(tp, s, spec.channel, spec.axes, tp.TP_PREC_F32_RECHECK)
    counts, stats = tp.new_counts(bn)
    ds = tp.DeviceSample.from_sample(s)
    n = ds.n
    cuts = [0, 7, 4096, 10001, n // 2 + 3, n]
    for a, b in zip(cuts[:-1], cuts[1:]):
        part = tp.DeviceSample([t[a:b] for t in ds.comps], ds.tag[a:b])
        tp.bin(part, ch, bn, tp.TP_PREC_F32_RECHECK, counts, stats)
    torch.cuda.synchronize()
    c = [int(x) for x in u64(counts)]
    assert [c[4 * r:4 * r + 4] for r in range(bn.nrows)] == whole[0]
    assert [int(x) for x in u64(stats)][:4] == whole[1][:4]


@pytest.mark.parametrize("dtype,k", [(torch.float64, -560), (torch.float64, 250),
                                     (torch.float32, -80), (torch.float32, 80)])
def test_scale_invariance(tp, dtype, k):
    """Classes and |Phi|, |cos theta| bins are invariant under p -> 2^k p (mass bins
    when their edges scale too).  At these scales products underflow or overflow
    float64, so the fast bounds must defer and the later tiers decide."""
    ch = synth.CHANNELS["Lb_pKpipi"]
    s = synth.generate(ch, 2003, 70, dtype=dtype)
    comps, tag = s.numpy()
    f = 2.0 ** k
    scaled = [[t * f for t in row] for row in s.comps]
    for row, srow in zip(s.comps, scaled):
        for t, st in zip(row, srow):
            assert torch.equal(st / f, t), "scaling must be exact"
    ss = synth.Sample(ch, scaled, s.tag)
    mass = synth.lb_mass03_axis(ch)
    for axes in ([synth.absphi_axis(12)], [synth.abscos_axis(0, 5), synth.absphi_axis(10)],
                 [synth.absphi_axis(10), mass]):
        want = oracle.run(comps, tag, ch.triple, ch.planes, axes)
        sax = [synth.Axis(a.kind, a.edges * f, a.slots) if a.kind == synth.AXIS_MASS else a for a in axes]
        precs = [tp.TP_PREC_F64] + ([tp.TP_PREC_F32_RECHECK] if dtype == torch.float32 else [])
        for prec in precs:
            counts, stats = gpu_bin(tp, ss, ch, sax, prec)
            print(f"[scale] k={k} {dtype} prec={prec} stats={stats}", flush=True)
            assert stats[6] == 0
            assert counts == want["counts"]
            assert stats[:4] == want["stats"]


def test_event_order_does_not_matter(tp):
    """Integer histograms are order-independent: a shuffled copy of a sample gives
    the same counts and statistics, in every scheme and precision (also with the
    identical particles ordered on the fly)."""
    ch = synth.CHANNELS["Lb_ppipipi"]
    s = synth.generate(ch, 50021, 61, inj=synth.INJ_SIN)
    perm = torch.from_numpy(np.random.default_rng(2).permutation(s.n))
    sh = synth.Sample(ch, [[t[perm].contiguous() for t in row] for row in s.comps], s.tag[perm].contiguous())
    for axes in ([synth.absphi_axis(12)], [synth.abscos_axis(0, 6), synth.absphi_axis(10)],
                 [synth.mass_axis((0, 3), 1000.0, 5200.0, 9)]):
        for ident in (None, ch.identical):
            for prec in (tp.TP_PREC_F32_RECHECK, tp.TP_PREC_F64):
                out = []
                for smp in (s, sh):
                    ds = tp.DeviceSample.from_sample(smp)
                    counts, stats = tp.bin(ds, tp.channel(ch.triple, ch.planes, ident), tp.Binning(axes), prec)
                    torch.cuda.synchronize()
                    out.append(([int(x) for x in u64(counts)], [int(x) for x in u64(stats)]))
                assert out[0] == out[1], (axes, ident, prec)


@pytest.mark.parametrize("wl,ch_name", [("lb_pkpipi_1e8_phi10xm8", "Lb_pKpipi"), ("d0_kkpipi_5e8_m32x32", "D0_KKpipi")])
def test_scp_from_gpu_counts(tp, wl, ch_name):
    """Binned S_CP of eq. (1) in both splits of Sect. 5 (P-even: [I+II] vs [III+IV];
    P-odd: [I+IV] vs [II+III]) from the pass's counts, against the exact oracle
    on the oracle's counts of the same events."""
    spec = synth.workload_specs(wl, scale=2e-4 if wl.startswith("d0") else 1e-3)[0]
    s = synth.make_sample(spec)
    ch = spec.channel
    comps, tag = s.numpy()
    want = oracle.run(comps, tag, ch.triple, ch.planes, spec.axes)
    got, stats = gpu_bin(tp, s, ch, spec.axes, tp.TP_PREC_F32_RECHECK)
    assert got == want["counts"] and stats[6] == 0
    c = np.array(got, dtype=np.int64).ravel()
    w = np.array(want["counts"], dtype=object)
    for mode in (0, 1):
        S, chi2, ndf, p = tp.scp(c, mode)
        if mode == 0:
            x, xb = w[1:, 0] + w[1:, 1], w[1:, 2] + w[1:, 3]
        else:
            x, xb = w[1:, 0] + w[1:, 3], w[1:, 1] + w[1:, 2]
        ws, wchi2, wndf, wp = exact.scp([int(v) for v in x], [int(v) for v in xb])
        print(f"[scp] {wl} mode {mode}: chi2 {chi2:.4f} ndf {ndf} p {p:.4g}", flush=True)
        assert ndf == wndf == len(x) - 1
        np.testing.assert_allclose(S, ws, rtol=1e-12, atol=1e-15)
        assert chi2 == pytest.approx(wchi2, rel=1e-12)
        assert p == pytest.approx(wp, rel=1e-9, abs=1e-300)


def test_graph_replay_after_plan_eviction(tp):
    """More than 256 distinct requests evict the first request's launch plan (device
    tables); a later graphed replay of that request must rebuild the plan and its graph,
    not replay a graph whose tables were freed: counts stay bit-exact against the oracle."""
    ch = synth.CHANNELS["Lb_ppipipi"]
    axes = [synth.absphi_axis(10)]
    s = synth.generate(ch, 3001, 41)
    comps, tag = s.numpy()
    want = oracle.run(comps, tag, ch.triple, ch.planes, axes)
    ds = tp.DeviceSample.from_sample(s)
    bn = tp.Binning(axes)
    chan = tp.channel(ch.triple, ch.planes)
    counts, stats = tp.new_counts(bn)
    b = tp.Batch([(ds, chan, bn, counts, stats)])
    b.run(tp.TP_PREC_F32_RECHECK, None, True, check=True)
    c = [int(x) for x in u64(counts)]
    assert [c[4 * r:4 * r + 4] for r in range(bn.nrows)] == want["counts"]
    # 300 other requests (distinct counter buffers make distinct plans), each graphed
    others = [tp.new_counts(bn) for _ in range(300)]
    for oc, os_ in others:
        tp.Batch([(ds, chan, bn, oc, os_)]).run(tp.TP_PREC_F32_RECHECK, None, True)
    torch.cuda.synchronize()
    for oc, _ in others[::37]:
        c = [int(x) for x in u64(oc)]
        assert [c[4 * r:4 * r + 4] for r in range(bn.nrows)] == want["counts"]
    # the first request again, twice (its plan was evicted): counts accumulate
    counts.zero_()
    stats.zero_()
    b.run(tp.TP_PREC_F32_RECHECK, None, True)
    b.run(tp.TP_PREC_F32_RECHECK, None, True, check=True)
    c = [int(x) for x in u64(counts)]
    assert [c[4 * r:4 * r + 4] for r in range(bn.nrows)] == [[2 * v for v in row] for row in want["counts"]]


def test_more_deferred_events_than_a_million(tp):
    """2^20 + 4099 exactly coplanar events (Delta = 0) all defer to the exact tiers and
    land in n_zero; nothing is unresolved (the deferral list holds every event of a launch)."""
    n = (1 << 20) + 4099
    rng = np.random.default_rng(12)
    # four momenta in the x-y plane: every 4x4 determinant with a zero pz column vanishes
    comps = np.zeros((4, 4, n), dtype=np.float32)
    for slot in range(4):
        px = rng.integers(-50, 50, size=n).astype(np.float32)
        py = rng.integers(-50, 50, size=n).astype(np.float32)
        comps[slot, 0] = np.sqrt(px.astype(np.float64) ** 2 + py.astype(np.float64) ** 2 + 140.0 ** 2).astype(np.float32)
        comps[slot, 1], comps[slot, 2] = px, py
    tag = (rng.uniform(size=n) < 0.5).astype(np.int8)
    sample = synth.Sample(synth.CHANNELS["Lb_ppipipi"],
                          [[torch.from_numpy(np.ascontiguousarray(comps[a][b])) for b in range(4)] for a in range(4)],
                          torch.from_numpy(tag))
    ch = synth.CHANNELS["Lb_ppipipi"]
    for axes in ([], [synth.absphi_axis(10)]):
        counts, stats = gpu_bin(tp, sample, ch, axes, tp.TP_PREC_F32_RECHECK)
        print(f"[deferral] axes={len(axes)} stats={stats}", flush=True)
        assert stats[0] == n and stats[1] == n and stats[6] == 0
        assert stats[5] >= n                              # every event through the exact tiers
        assert all(v == 0 for row in counts for v in row)


@pytest.mark.parametrize("chname,gamma", [("D0_KKpipi", None), ("Lb_ppipipi", None), ("Lb_pKpipi", 300.0)])
def test_fp32_tier_probe(tp, chname, gamma):
    """The float32 tier's raw contraction (tp_probe_f32) against the float64 one and the
    oracle: its running bound covers its error (|det32 - det64| <= bound32 + 8.1 u S),
    every raw float32 sign that disagrees with the oracle's certified class lies among the
    events the bound sends to the recheck, and the recheck fraction equals the pass's n_tier2
    on the same events (global counts, TP_PREC_F32_RECHECK)."""
    ch = synth.CHANNELS[chname]
    s = synth.generate(ch, 20011, 61, fixed_gamma=gamma) if gamma else synth.generate(ch, 20011, 61)
    comps, tag = s.numpy()
    want = oracle.run(comps, tag, ch.triple, ch.planes, want_events=True)
    cls = np.asarray(want["cls"])
    ds = tp.DeviceSample.from_sample(s)
    d32, b32, d64, s64 = [t.cpu().numpy().astype(np.float64) for t in tp.probe_f32(ds, tp.channel(ch.triple, ch.planes))]
    assert np.all(np.abs(d32 - d64) <= b32 + 8.1 * 2.0 ** -53 * s64)
    # eq. (4): the class fixes the sign of C_T for M (tag 0) and of -Cbar_T ... i.e. sign(C_T^inv)
    sgn = np.where(np.isin(cls, (0, 3)), 1.0, np.where(np.isin(cls, (1, 2)), -1.0, 0.0))
    decided = sgn != 0
    wrong = decided & (np.sign(d32) != sgn)
    rechecked = np.abs(d32) <= b32
    print(f"[fp32 probe] {chname} gamma={gamma}: rechecked {rechecked.mean():.2e}, raw wrong signs "
          f"{int(wrong.sum())}", flush=True)
    assert not np.any(wrong & ~rechecked)
    counts, stats = gpu_bin(tp, s, ch, [], tp.TP_PREC_F32_RECHECK)
    assert stats[4] == int(rechecked.sum())
