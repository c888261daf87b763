"""Parity at the workloads' full sizes (1e5 ... 5e8 events), in the launch
configuration the benchmark times (batched, HIP graph, tuned shapes).

The oracle cannot decide 5e8 events, so at full size the checks are
* properties that hold at any size: the float32-recheck path, the plain
  float64 path and the batched graph path give bit-identical counts and
  statistics; row 0 of the counts totals the classified events; every event is
  counted once;
* sampled outputs the oracle computes one by one: the per-event classes of
  4096 randomly chosen events (tp_compute on the whole sample) against the
  oracle on exactly those events.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1612_04705_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    from paper_1612_04705_amd import tpasym
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    tpasym.load()
    return tpasym


def u64(t):
    return [int(x) for x in t.cpu().numpy().view(np.uint64)]


@pytest.mark.parametrize("workload", ["lb_ppipipi_f64_1e5", "lb_ppipipi_1e7_phi12", "lb_pkpipi_1e8_phi10xm8",
                                      "d0_kkpipi_5e8_m32x32"])
def test_full_size(tp, workload):
    dev = torch.device("cuda:0")
    (spec,) = synth.workload_specs(workload, 1.0)
    s = synth.make_sample(spec, device=dev)
    s.phi_gen = s.gamma = s.m12 = s.m34 = None
    torch.cuda.empty_cache()
    n = s.n
    print(f"[full] {workload}: {n} events generated", flush=True)
    ds = tp.DeviceSample([s.comps[a][b] for a in range(4) for b in range(4)], s.tag)
    ch = tp.channel(spec.channel.triple, spec.channel.planes)
    bn = tp.Binning(spec.axes)
    f32 = spec.dtype == torch.float32
    results = []
    for prec in ([tp.TP_PREC_F32_RECHECK] if f32 else []) + [tp.TP_PREC_F64]:
        counts, stats = tp.bin(ds, ch, bn, prec)
        torch.cuda.synchronize()
        results.append((prec, u64(counts), u64(stats)))
    # the benchmark's launch configuration: batched, tuned shapes, HIP graph, three steps
    counts, stats = tp.new_counts(bn)
    b = tp.Batch([(ds, ch, bn, counts, stats)])
    prec = tp.TP_PREC_F32_RECHECK if f32 else tp.TP_PREC_F64
    b.autotune(prec)
    counts.zero_()
    stats.zero_()
    for _ in range(3):
        b.run(prec, None, True)
    torch.cuda.synchronize()
    c3, s3 = u64(counts), u64(stats)
    results.append((prec, [v // 3 for v in c3], [v // 3 for v in s3]))
    assert all(v % 3 == 0 for v in c3 + s3)
    # counts and the event statistics agree everywhere; the tier statistics
    # (float64 rechecks of float32 signs, listed events) only within one precision
    for pr, c_, st_ in results[1:]:
        assert c_ == results[0][1]
        assert st_[:4] == results[0][2][:4] and st_[6] == results[0][2][6]
        same = [r for r in results if r[0] == pr]
        assert all(r[2] == same[0][2] for r in same)
    _, c, st = results[0]
    assert st[6] == 0                                   # nothing unresolved
    assert st[0] == n
    assert sum(c[:4]) == n - st[1] - st[2]              # row 0: every classified event once
    if bn.nrows > 1:
        binned = np.array(c[4:]).reshape(-1, 4).sum(axis=0)
        assert int(binned.sum()) == sum(c[:4]) - st[3]  # in range or counted out of range
    print(f"[full] {workload}: counts equal across paths, tier2={st[4]} tier3={st[5]}", flush=True)

    # sampled per-event classes against the oracle
    cls, _, _ = tp.compute(ds, ch, prec, want_ct=False)
    torch.cuda.synchronize()
    idx = torch.from_numpy(np.sort(np.random.default_rng(11).choice(n, 4096, replace=False))).to(dev)
    comps = np.stack([s.comps[a][b].index_select(0, idx).cpu().numpy() for a in range(4) for b in range(4)])
    comps = comps.reshape(4, 4, -1)
    tag = s.tag.index_select(0, idx).cpu().numpy()
    want = oracle.run(comps, tag, spec.channel.triple, spec.channel.planes, want_events=True)
    assert np.array_equal(cls.index_select(0, idx).cpu().numpy(), want["cls"])
    del ds, s, b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("tuning", [None, (256, 8, 4, 4)])
def test_sample_past_2_to_32_bytes_per_array(tp, tuning):
    """A float32 sample of 1025 * 2^20 events, more than 2^30: its component arrays pass
    2^32 bytes, so the host splits it into two descriptors (the kernels index each array
    with 32-bit offsets from a descriptor's base).  The sample is one 2^20-event sample
    tiled 1025 times, so every count is exactly 1025 times the oracle's count for the
    tile; scalar loads (default shape) and 16-byte vector loads (4 events per lane)."""
    ch = synth.CHANNELS["Lb_pKpipi"]
    axes = [synth.absphi_axis(10), synth.lb_mass03_axis(ch)]
    small = synth.generate(ch, 1 << 20, 77, inj=synth.INJ_SIN2)
    comps, tag = small.numpy()
    want = oracle.run(comps, tag, ch.triple, ch.planes, axes)
    reps = 1025
    print(f"[full] {reps} x 2^20 events ({reps << 20}), tuning {tuning}", flush=True)
    big = [torch.from_numpy(np.ascontiguousarray(comps[a, b])).cuda().repeat(reps) for a in range(4) for b in range(4)]
    big_tag = torch.from_numpy(np.ascontiguousarray(tag)).cuda().repeat(reps)
    ds = tp.DeviceSample(big, big_tag)
    assert ds.n == reps << 20 and ds.n > (1 << 30)
    bn = tp.Binning(axes)
    chan = tp.channel(ch.triple, ch.planes)
    counts, stats = tp.new_counts(bn)
    if tuning is None:
        tp.bin(ds, chan, bn, tp.TP_PREC_F32_RECHECK, counts, stats)
    else:
        tp.Batch([(ds, chan, bn, counts, stats)]).run(tp.TP_PREC_F32_RECHECK, tp.Tuning(*tuning), False, check=True)
    torch.cuda.synchronize()
    c = u64(counts)
    c = [c[4 * r:4 * r + 4] for r in range(bn.nrows)]
    st = u64(stats)
    del big, big_tag, ds
    torch.cuda.empty_cache()
    assert c == [[reps * v for v in row] for row in want["counts"]]
    assert st[:4] == [reps * v for v in want["stats"]]
    assert st[6] == 0


def test_full_size_batch(tp):
    """The batched workload at full size (64 samples, 1.118e8 events) in the benchmark's
    launch configuration: per-scheme tuned shapes, the scheme groups on parallel branches
    (the largest at 16 workgroups per CU, the others at most 4), HIP graph, three steps.
    Counts and statistics of every sample equal three times the plain single-sample float64
    path's; the 16 smallest samples, whole, against the oracle."""
    dev = torch.device("cuda:0")
    specs = synth.workload_specs("lb_batch64_1e3to1e7", 1.0)
    items, samples = [], []
    for spec in specs:
        s = synth.make_sample(spec, device=dev)
        ds = tp.DeviceSample([s.comps[a][b] for a in range(4) for b in range(4)], s.tag)
        bn = tp.Binning(spec.axes)
        items.append((ds, tp.channel(spec.channel.triple, spec.channel.planes), bn, *tp.new_counts(bn, dev)))
        samples.append((spec, s))
    torch.cuda.synchronize()
    print(f"[full] batch: {len(items)} samples, {sum(s.n for _, s in samples)} events generated", flush=True)
    b = tp.Batch(items)
    b.autotune(tp.TP_PREC_F32_RECHECK)
    for _ in range(3):
        b.run(tp.TP_PREC_F32_RECHECK, None, True)
    torch.cuda.synchronize()
    got = [(u64(it[3]), u64(it[4])) for it in items]
    for k, ((ds, ch, bn, _, _), (c3, s3)) in enumerate(zip(items, got)):
        c64, s64 = tp.bin(ds, ch, bn, tp.TP_PREC_F64)
        c64, s64 = u64(c64), u64(s64)
        assert c3 == [3 * v for v in c64], k
        assert s3[:4] == [3 * v for v in s64[:4]] and s3[6] == 0, k
    print("[full] batch: counts equal to the float64 single-sample path", flush=True)
    for k in sorted(range(len(samples)), key=lambda i: samples[i][1].n)[:16]:
        spec, s = samples[k]
        comps = np.stack([s.comps[a][b].cpu().numpy() for a in range(4) for b in range(4)]).reshape(4, 4, -1)
        want = oracle.run(comps, s.tag.cpu().numpy(), spec.channel.triple, spec.channel.planes, spec.axes)
        assert got[k][0] == [3 * v for row in want["counts"] for v in row], k
        assert got[k][1][:4] == [3 * v for v in want["stats"]], k
    del items, samples, b
    torch.cuda.empty_cache()
