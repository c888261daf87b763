"""GPU parity of the identical-particle ordering fused into the pass.

The stored order of the two identical particles is shuffled per event; the
pass, told which slots they are, must reproduce the oracle's counts (which
orders them by rest-frame energy) bit for bit, in every binning scheme and
both precisions, including the schemes whose relabelling moves the pair to
kernel slots (0, 2).  Exact ties go to the exact tier and keep the stored order.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1612_04705_amd import synth

pytestmark = pytest.mark.gpu

IDENT = (1, 3)


@pytest.fixture(scope="module")
def tp():
    from paper_1612_04705_amd import tpasym
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    tpasym.load()
    return tpasym


def u64(t):
    return t.cpu().numpy().view(np.uint64).astype(object)


def shuffled(name, n, seed, dtype=torch.float32):
    ch = synth.CHANNELS[name]
    s = synth.generate(ch, n, seed, inj=synth.INJ_SIN, dtype=dtype)
    mask = torch.from_numpy(np.random.default_rng(seed).uniform(size=n) < 0.5)
    for c in range(4):
        a, b = s.comps[1][c].clone(), s.comps[3][c].clone()
        s.comps[1][c] = torch.where(mask, b, a)
        s.comps[3][c] = torch.where(mask, a, b)
    return ch, s


def gpu_counts(tp, sample, ch, axes, prec, batch=False):
    ds = tp.DeviceSample.from_sample(sample)
    bn = tp.Binning(axes)
    counts, stats = tp.new_counts(bn)
    chan = tp.channel(ch.triple, ch.planes, identical=IDENT)
    if batch:
        tp.Batch([(ds, chan, bn, counts, stats)]).run(prec, None, False)
    else:
        tp.bin(ds, chan, bn, prec, counts, stats)
    torch.cuda.synchronize()
    c = [int(x) for x in u64(counts)]
    return [c[4 * r:4 * r + 4] for r in range(bn.nrows)], [int(x) for x in u64(stats)]


SCHEMES = {
    "global": [],
    "absphi": [synth.absphi_axis(20)],
    "mass03": [synth.mass_axis((0, 3), 1000.0, 5200.0, 16)],
    "abscos_fast": [synth.abscos_axis(1, 10)],            # relabelling puts the pair at (0, 2)
    "abscos_slow_x_phi": [synth.abscos_axis(3, 6), synth.absphi_axis(8)],
    "mass12_x_abscos0": [synth.mass_axis((1, 2), 200.0, 3000.0, 6), synth.abscos_axis(0, 5)],
}


@pytest.mark.parametrize("name", ["Lb_ppipipi", "Lb_pKKK"])
@pytest.mark.parametrize("scheme", list(SCHEMES))
def test_shuffled_identical_match_oracle(tp, name, scheme):
    ch, s = shuffled(name, 60001, 17)
    axes = SCHEMES[scheme]
    comps, tag = s.numpy()
    want = oracle.run(comps, tag, ch.triple, ch.planes, axes, identical=IDENT)
    for prec in (tp.TP_PREC_F64, tp.TP_PREC_F32_RECHECK):
        counts, stats = gpu_counts(tp, s, ch, axes, prec)
        print(f"[order] {name} {scheme} prec={prec} stats={stats}", flush=True)
        assert stats[6] == 0
        assert counts == want["counts"]
        assert stats[:4] == want["stats"]
    counts, _ = gpu_counts(tp, s, ch, axes, tp.TP_PREC_F32_RECHECK, batch=True)
    assert counts == want["counts"]


def test_classes_match_oracle(tp):
    ch, s = shuffled("Lb_ppipipi", 20011, 23)
    comps, tag = s.numpy()
    want = oracle.run(comps, tag, ch.triple, ch.planes, want_events=True, identical=IDENT)
    ds = tp.DeviceSample.from_sample(s)
    for prec in (tp.TP_PREC_F64, tp.TP_PREC_F32_RECHECK):
        cls, ct, stats = tp.compute(ds, tp.channel(ch.triple, ch.planes, identical=IDENT), prec)
        torch.cuda.synchronize()
        assert np.array_equal(cls.cpu().numpy(), want["cls"])


def test_exact_ties_keep_stored_order(tp):
    from test_order_pins import tie_events, _sample   # tests/ is on sys.path (rootdir conftest)
    ch = synth.CHANNELS["Lb_ppipipi"]
    rows = tie_events(700, 9)
    comps, tag = _sample(rows, np.float32)
    want = oracle.run(comps, tag, ch.triple, ch.planes, [synth.absphi_axis(8)], identical=IDENT)
    s = synth.Sample(ch, [[torch.from_numpy(np.ascontiguousarray(comps[a][b])) for b in range(4)] for a in range(4)],
                     torch.from_numpy(tag))
    for prec in (tp.TP_PREC_F64, tp.TP_PREC_F32_RECHECK):
        counts, stats = gpu_counts(tp, s, ch, [synth.absphi_axis(8)], prec)
        print(f"[order] ties prec={prec} stats={stats}", flush=True)
        assert stats[5] > 0                     # the ties went to the exact tier
        assert counts == want["counts"]


def test_float64_storage(tp):
    ch, s = shuffled("Lb_pKKK", 30011, 29, dtype=torch.float64)
    axes = SCHEMES["abscos_slow_x_phi"]
    comps, tag = s.numpy()
    want = oracle.run(comps, tag, ch.triple, ch.planes, axes, identical=IDENT)
    counts, stats = gpu_counts(tp, s, ch, axes, tp.TP_PREC_F64)
    assert stats[6] == 0
    assert counts == want["counts"] and stats[:4] == want["stats"]
