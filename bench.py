"""Benchmark of the T-odd triple-product asymmetry pass on one MI355X.

Workload (default): the batched workload -- 64 independent samples, sizes
log-uniform in [1e3, 1e7] events, four Lambda_b channels x three binning
schemes (|Phi|; |Phi| x m(0,3); |cos theta_p| x |Phi|), float32 SoA storage,
one persistent launch per binning scheme on parallel branches of one HIP
graph, each scheme's launch shape tuned by the autotuner.
One step = one pass of the whole hot path over the whole batch (every event:
contraction, certified sign, class, bins, histogram, flush; the exact tier's
list pass).  Inputs are generated on the GPU before timing and stay in HBM.

Prints ONE JSON line (see the roofline / cpu_baseline objects).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_F32 = 65      # 16 x 4 B components + 1 B tag per event
BYTES_F64 = 129


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_hash():
    h = hashlib.sha256()
    for f in ("tp_pass.hip", "tp_kernel.h", "tp_host.cpp"):
        with open(os.path.join(ROOT, "paper_1612_04705_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    fn = os.path.join(ROOT, "profiles", "tp_pass_kernel_counters.json")
    if not os.path.exists(fn):
        return None
    with open(fn) as f:
        d = json.load(f)
    e = d.get(workload)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def make_workload(name, device, scale):
    import torch
    from paper_1612_04705_amd import synth, tpasym
    specs = synth.workload_specs(name, scale)
    items, samples = [], []
    t0 = time.time()
    for spec in specs:
        s = synth.make_sample(spec, device=device)
        ds = tpasym.DeviceSample([s.comps[a][b] for a in range(4) for b in range(4)], s.tag)
        bn = tpasym.Binning(spec.axes)
        counts, stats = tpasym.new_counts(bn, device)
        items.append((ds, tpasym.channel(spec.channel.triple, spec.channel.planes), bn, counts, stats))
        samples.append((spec, s))
    torch.cuda.synchronize()
    log(f"generated {len(specs)} samples, {sum(s.n for _, s in samples)} events in {time.time() - t0:.1f}s")
    return specs, samples, items


def cpu_baseline(samples, budget_events, want_counts_of):
    """Time the oracle (float64 pass + exact resolution) on the first whole samples
    up to ``budget_events`` events; return the cpu_baseline object and the
    oracle counts per sample index for the parity check."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    nthreads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    done, secs, used = 0, 0.0, []
    t_pass = t_exact = 0.0
    flagged = 0
    out = {}
    for i, (spec, s) in enumerate(samples):
        if done > 0 and done + s.n > budget_events:
            continue
        comps = np.stack([s.comps[a][b].cpu().numpy() for a in range(4) for b in range(4)]).reshape(4, 4, -1)
        tag = s.tag.cpu().numpy()
        t0 = time.perf_counter()
        r = oracle.run(comps, tag, spec.channel.triple, spec.channel.planes, spec.axes, nthreads=nthreads)
        secs += time.perf_counter() - t0
        t_pass += r["seconds"]
        t_exact += r["seconds_exact"]
        flagged += r["n_flagged"]
        done += s.n
        used.append(i)
        if i in want_counts_of:
            out[i] = r
        if done >= budget_events:
            break
    try:
        model = [l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name")][0]
    except Exception:
        model = "unknown"
    # one thread on the first events of the largest sample timed above
    spec, s = samples[max(used, key=lambda i: samples[i][1].n)]
    m = min(s.n, 500000)
    comps = np.stack([s.comps[a][b][:m].cpu().numpy() for a in range(4) for b in range(4)]).reshape(4, 4, -1)
    t0 = time.perf_counter()
    oracle.run(comps, s.tag[:m].cpu().numpy(), spec.channel.triple, spec.channel.planes, spec.axes, nthreads=1)
    one = time.perf_counter() - t0
    return {"value": done / secs, "unit": "events/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{len(used)} whole samples of the same workload ({done} events; float64 pass on "
                      f"{nthreads} threads, then exact rational resolution of the {flagged} events it flags, "
                      f"one at a time on one thread; {model})",
            "seconds": secs,
            # where the time goes: the threaded float64 pass, the serial exact stage
            "seconds_float64_pass": t_pass, "seconds_exact_serial": t_exact, "flagged": flagged,
            "single_thread": {"value": m / one, "unit": "events/s", "events": m, "seconds": one}}, out


# MI355X: 256 compute units x 4 SIMDs x 16 lanes x 2.4 GHz, one float32 vector
# operation per lane per cycle (packed float32 is not used)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
MFMA_F16_PEAK_TFLOPS = 2500.0   # dense float16 matrix-core peak


def energy_leg(n, nperm, dev, per_pass=126, cpu_events=0):
    """The energy test at the paper's scale: D0 -> K+ K- pi+ pi- events, five
    invariant-mass coordinates, the P-odd split ([I+IV] vs [II+III]) and
    ``nperm`` permutations of it, ``per_pass`` of them per launch of the pair
    sums (each launch also carries an all-ones column and the observed split)."""
    import numpy as np
    import torch
    from paper_1612_04705_amd import synth, tpasym
    ch = synth.CHANNELS["D0_KKpipi"]
    spec = synth.SampleSpec(ch, n, 77, [], inj=synth.INJ_SGN)
    s = synth.make_sample(spec, device=dev)
    ds = tpasym.DeviceSample([s.comps[a][b] for a in range(4) for b in range(4)], s.tag)
    masks = [0b0011, 0b1001, 0b0110, 0b1100, 0b1101]          # m12, m14, m23, m34, m134
    Y = tpasym.coords(ds, masks, 1e-3)
    cls, _, _ = tpasym.compute(ds, tpasym.channel(ch.triple, ch.planes), tpasym.TP_PREC_F32_RECHECK)
    lab = ((cls == 0) | (cls == 3)).to(torch.uint8)
    # permutations drawn on the host (seeded numpy; random numbers are inputs of the
    # library), one shuffled copy of the split per permutation column
    rng = np.random.default_rng(1234)
    lab_h = lab.cpu().numpy()
    ks = [min(per_pass, nperm - p0) for p0 in range(0, nperm, per_pass)]
    colsets = []
    for k in ks:
        ncol = k + 2
        C = 32 if ncol <= 32 else (64 if ncol <= 64 else 128)
        if ncol > 128:
            raise SystemExit("at most 126 permutations per launch")
        cols = np.zeros((n, C), dtype=np.uint8)
        cols[:, 0] = 1
        cols[:, 1] = lab_h
        cols[:, 2:2 + k] = rng.permuted(np.broadcast_to(lab_h, (k, n)), axis=1).T
        colsets.append(torch.from_numpy(cols).to(dev))
    sigma = 0.3
    tpasym.pairsums(Y, colsets[0], sigma)                      # warm-up
    torch.cuda.synchronize()
    sums = [torch.zeros((c.shape[1], 2), dtype=torch.float64, device=dev) for c in colsets]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for c, sm in zip(colsets, sums):
        tpasym.pairsums(Y, c, sigma, sums=sm)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    T_obs_passes, T_perm = [], []
    for c, sm, k in zip(colsets, sums, ks):
        nx = c.sum(dim=0, dtype=torch.int64).cpu().numpy()
        T = tpasym.energy_eq2(sm.cpu().numpy(), nx, n)
        T_obs_passes.append(float(T[1]))
        T_perm.extend(float(t) for t in T[2:2 + k])
    T_obs = T_obs_passes[0]
    T_perm = np.array(T_perm)
    # psi is symmetric: the kernel forms each unordered pair once per launch.  Per
    # pair and launch it spends two units, which on gfx950 do not overlap
    # (measured), so its bound is the sum of their minimum times:
    #   float16 matrix cores: the distances x_i . x_j as one contraction over
    #     32 float16 slots (split terms), 64 flops; the contraction with the C
    #     columns as two float16 terms, 4 C flops;
    #   vector ALU: exp2, the float16 split (half a pack, one residual, half a
    #     pack): 3 lane operations (exp2 counted as one issue slot, which if
    #     anything overstates the peak).
    # The method's own psi arithmetic (D differences, D multiply-adds, one exp2:
    # 2 D + 1 lane operations per pair) over the vector-ALU peak is reported
    # beside it for comparison with an all-vector-ALU design.
    pairs = n * (n - 1) / 2.0
    D = len(masks)
    npairs = pairs * len(ks)
    ops = (2 * D + 1) * npairs
    mfma_flops = sum(4.0 * c.shape[1] * pairs for c in colsets)
    dist_flops = 64.0 * npairs
    valu_ops = 3.0 * npairs
    t_bound = (dist_flops + mfma_flops) / (MFMA_F16_PEAK_TFLOPS * 1e12) + valu_ops / (VALU_PEAK_TOPS * 1e12)
    C0 = colsets[0].shape[1]
    # method-level bound, independent of how the kernel splits its work: psi once per
    # unordered pair on the vector ALU (D differences, D multiply-adds, one exp:
    # 2 D + 1 lane operations) and one multiply-add per pair and column (2 flops
    # per column, on the float16 matrix cores at their dense peak)
    t_method = ops / (VALU_PEAK_TOPS * 1e12) + sum(2.0 * c.shape[1] * pairs for c in colsets) / \
        (MFMA_F16_PEAK_TFLOPS * 1e12)
    log(f"energy test: {n} events, {nperm} permutations in {len(ks)} launches of {C0} columns, "
        f"{sec * 1e3:.1f} ms, {sec * 1e3 / nperm:.2f} ms per permutation, T = {T_obs:.4e}")
    cpu = None
    if cpu_events > 0:
        # the oracle (plain float64 pair sums, numpy) on the first cpu_events
        # events of the same coordinates: one T of eq. (2) = every ordered pair once
        from oracle import energy
        m = int(cpu_events)
        Yh = Y[:, :m].double().cpu().numpy()
        lh = lab[:m].cpu().numpy()
        t0 = time.perf_counter()
        energy.T_eq2(Yh, lh, sigma)
        csec = time.perf_counter() - t0
        rate = m * (m - 1) / csec
        cpu = {"value": rate, "unit": "ordered pairs/s", "cores": 1, "kind": "oracle",
               "sample": f"T of eq. (2) for the observed split of the first {m} events (float64 numpy, one thread)",
               "seconds": csec,
               "seconds_per_permutation_at_full_size": n * (n - 1) / rate}
        log(f"energy oracle: {rate:.3e} ordered pairs/s ({csec:.1f} s for {m} events); "
            f"one permutation at {n} events ~{n * (n - 1) / rate:.0f} s")
    return {"cpu_baseline": cpu,"events": n, "coordinates": 5, "sigma_GeV": sigma, "columns": C0, "permutations": nperm,
            "launches": len(ks), "seconds": sec, "seconds_per_pass": sec / len(ks),
            "ms_per_permutation": sec * 1e3 / nperm,
            "unordered_pairs_per_s": pairs * len(ks) / sec,
            "roofline": {"bound": "mfma+alu", "achieved": npairs / sec / 1e12, "peak": npairs / t_bound / 1e12,
                         "unit": "Tpair/s", "frac": t_bound / sec,
                         "per_pair": {"mfma_f16_flops_distance": 64, "mfma_f16_flops_columns": 4 * C0,
                                      "valu_lane_ops": 3},
                         "mfma_f16_frac": (dist_flops + mfma_flops) / sec / 1e12 / MFMA_F16_PEAK_TFLOPS,
                         "valu_frac": valu_ops / sec / 1e12 / VALU_PEAK_TOPS,
                         "method_alu_tops": ops / sec / 1e12, "method_alu_frac": ops / sec / 1e12 / VALU_PEAK_TOPS,
                         "method_lane_ops_per_pair": 2 * D + 1,
                         "method_bound": {"seconds": t_method, "frac": t_method / sec,
                                          "per_pair": {"valu_lane_ops": 2 * D + 1, "mfma_f16_flops_per_column": 2}},
                         "dtype": "f16 x2 (distances, products), f32 (psi, tiles), f64 (sums)"},
            "T_obs": T_obs, "T_obs_spread_over_launches": max(T_obs_passes) - min(T_obs_passes),
            "p_value": float(np.count_nonzero(T_perm > T_obs)) / nperm,
            "paper_context": "one permutation at 1e6 events took ~30 min on NVIDIA M2070 / K40c (Sect. 6)"}


def energy_bkg_leg(n, nperm, dev, bkg_frac=0.2, per_launch=41):
    """Background-subtracted energy test (eq. (3)) at the same scale: a main
    sample and a background (side-band) sample of the same coordinates, the
    P-odd flavour split in each, and ``nperm`` permutations that shuffle the
    flavour within the main and within the background sample.  One launch of
    128 columns carries the two sample indicators (also the row weights), the
    observed flavour triple and ``per_launch`` permuted triples."""
    import numpy as np
    import torch
    from paper_1612_04705_amd import synth, tpasym
    ch = synth.CHANNELS["D0_KKpipi"]
    nb = int(n * bkg_frac)
    nm = n - nb
    masks = [0b0011, 0b1001, 0b0110, 0b1100, 0b1101]
    Ys, labs = [], []
    for size, seed, inj in ((nm, 78, synth.INJ_SGN), (nb, 79, None)):
        spec = synth.SampleSpec(ch, size, seed, [], inj=inj)
        smp = synth.make_sample(spec, device=dev)
        ds = tpasym.DeviceSample([smp.comps[a][b] for a in range(4) for b in range(4)], smp.tag)
        Ys.append(tpasym.coords(ds, masks, 1e-3))
        cls, _, _ = tpasym.compute(ds, tpasym.channel(ch.triple, ch.planes), tpasym.TP_PREC_F32_RECHECK)
        labs.append(((cls == 0) | (cls == 3)).to(torch.uint8))
    Y = torch.cat(Ys, dim=1).contiguous()
    fm, fb = labs
    fm_h, fb_h = fm.cpu().numpy(), fb.cpu().numpy()
    rng = np.random.default_rng(4321)
    ks = [min(per_launch, nperm - p0) for p0 in range(0, nperm, per_launch)]
    colsets = []
    for k in ks:
        cols = np.zeros((n, 128), dtype=np.uint8)
        cols[:nm, 0] = 1
        cols[nm:, 1] = 1
        for q in range(k + 1):            # triple 0: the observed flavours
            a = fm_h if q == 0 else rng.permutation(fm_h)
            bt = fb_h if q == 0 else rng.permutation(fb_h)
            cols[:nm, 2 + 3 * q] = a
            cols[nm:, 3 + 3 * q] = bt
            cols[:nm, 4 + 3 * q] = a
            cols[nm:, 4 + 3 * q] = bt
        colsets.append(torch.from_numpy(cols).to(dev))
    sigma = 0.3
    tpasym.pairsums(Y, colsets[0], sigma, nrow=2)               # warm-up
    torch.cuda.synchronize()
    sums = [torch.zeros((128, 3), dtype=torch.float64, device=dev) for _ in colsets]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for c, sm in zip(colsets, sums):
        tpasym.pairsums(Y, c, sigma, nrow=2, sums=sm)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    n_x, n_xb = int(fm.sum()), nm - int(fm.sum())
    b_x, b_xb = int(fb.sum()), nb - int(fb.sum())
    # expected background in the main sample: the main sample is read as
    # signal plus a background like the side band, in proportion bkg_frac
    b, b_bar = bkg_frac * n_x, bkg_frac * n_xb
    T_obs, T_perm = None, []
    for sm, k in zip(sums, ks):
        triples = [(2 + 3 * q, 3 + 3 * q, 4 + 3 * q) for q in range(k + 1)]
        T = tpasym.energy_eq3(sm.cpu().numpy(), 0, 1, 0, 1, triples, n_x, n_xb, b_x, b_xb, b, b_bar)
        if T_obs is None:
            T_obs = float(T[0])
        T_perm.extend(float(t) for t in T[1:])
    T_perm = np.array(T_perm)
    log(f"energy test with background (eq. 3): {nm} + {nb} events, {nperm} permutations in {len(ks)} "
        f"launches, {sec * 1e3:.1f} ms, {sec * 1e3 / nperm:.2f} ms per permutation, T = {T_obs:.4e}")
    return {"events_main": nm, "events_background": nb, "permutations": nperm, "launches": len(ks),
            "seconds": sec, "ms_per_permutation": sec * 1e3 / nperm, "b": b, "b_bar": b_bar,
            "T_obs": T_obs, "p_value": float(np.count_nonzero(T_perm > T_obs)) / nperm}


def fp32_report(items, samples=None, max_events=None):
    """The float32 tier measured on the given samples (tp_probe_f32): how often its
    bound sends an event to the float64 recheck, its observed error against the
    float64 contraction (relative to the sum of the Laplace terms' magnitudes and
    to the value), and the raw float32 signs that are wrong, all of which must
    fall among the rechecked events."""
    import torch
    from paper_1612_04705_amd import tpasym
    U = 2.0 ** -53
    n_tot = rech = wrong = wrong_out = uncertain = 0
    rel_s, rel_v, ratio_max = [], [], 0.0
    for it in items:
        ds, ch = it[0], it[1]
        if max_events is not None and ds.n > max_events:
            ds = tpasym.DeviceSample([c[:max_events] for c in ds.comps], ds.tag[:max_events])
        d32, b32, d64, s64 = tpasym.probe_f32(ds, ch)
        d32 = d32.double()
        b32 = b32.double()
        err = (d32 - d64).abs()
        certified = d64.abs() > 10 * U * s64          # the float64 sign is certain
        rechecked = d32.abs() <= b32
        bad = certified & (torch.sign(d32) != torch.sign(d64))
        n_tot += ds.n
        rech += int(rechecked.sum())
        wrong += int(bad.sum())
        wrong_out += int((bad & ~rechecked).sum())
        uncertain += int((~certified).sum())
        pos = s64 > 0
        rel_s.append((err[pos] / s64[pos]).float())
        nz = d64 != 0
        rel_v.append((err[nz] / d64[nz].abs()).float())
        # the bound holds: |d32 - d64| <= bound32 + 8.1 u S
        ratio_max = max(ratio_max, float(((err - 8.1 * U * s64) / b32.clamp_min(1e-300)).max()))
    rs, rv = torch.cat(rel_s), torch.cat(rel_v)
    qs = torch.tensor([0.5, 0.99, 0.999], device=rs.device)

    def pct(t):
        # quantiles of a large tensor on a sorted sample (torch.quantile has a size cap)
        t = t.sort().values
        idx = (qs * (t.numel() - 1)).long()
        return [float(t[i]) for i in idx] + [float(t[-1])]
    return {"events": n_tot, "rechecked_frac": rech / n_tot,
            "err_over_term_sum": dict(zip(("p50", "p99", "p999", "max"), pct(rs))),
            "err_over_value": dict(zip(("p50", "p99", "p999", "max"), pct(rv))),
            "raw_fp32_wrong_signs": wrong, "wrong_signs_outside_recheck": wrong_out,
            "float64_sign_uncertain": uncertain, "max_err_over_bound": ratio_max}


def scp_report(items, reps):
    """Binned S_CP (eq. (1)) of every sample's counts in both splits of Sect. 5."""
    import numpy as np
    from paper_1612_04705_amd import tpasym
    rows = []
    for it in items:
        c = it[3].cpu().numpy().view(np.uint64)
        if not np.all(c % reps == 0):
            raise SystemExit("accumulated counts are not a whole number of passes")
        c = (c // reps).astype(np.int64)
        if c.size <= 8:
            continue
        r = []
        for mode in (0, 1):
            _, chi2, ndf, pv = tpasym.scp(c, mode)
            r += [round(float(chi2), 4), float(f"{pv:.4g}")]
        rows.append(r + [int(ndf)])
    return {"columns": ["chi2_P_even", "p_P_even", "chi2_P_odd", "p_P_odd", "ndf"], "per_sample": rows}


def single_leg(dev, workload, steps, warmup, chunk=0):
    """One large single-sample workload, resident in HBM, timed as a graphed
    pass (float32 storage, TP_PREC_F32_RECHECK requested: the float32 sign tier
    runs where no plane angle is binned, the first pass where one is).  With
    ``chunk`` > 0 the same events are also passed as consecutive chunks of that
    many events (one tp_bin call each, into the same counters), as a caller
    streaming them would, and the counts must be the same."""
    import numpy as np
    import torch
    from paper_1612_04705_amd import synth, tpasym
    t0 = time.time()
    spec = synth.workload_specs(workload)[0]
    smp = synth.make_sample(spec, device=dev)
    ds = tpasym.DeviceSample([smp.comps[a][b] for a in range(4) for b in range(4)], smp.tag)
    del smp
    n = ds.n
    bn = tpasym.Binning(spec.axes)
    ch = tpasym.channel(spec.channel.triple, spec.channel.planes)
    counts, stats = tpasym.new_counts(bn, dev)
    b = tpasym.Batch([(ds, ch, bn, counts, stats)])
    prec = tpasym.TP_PREC_F32_RECHECK
    torch.cuda.synchronize()
    log(f"{workload}: generated {n} events in {time.time() - t0:.1f}s")
    b.autotune(prec)
    for _ in range(warmup):
        b.run(prec, None, True)
    torch.cuda.synchronize()
    tpasym.timing_enable(True)
    tpasym.timing_reset()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        b.run(prec, None, True)
    e1.record()
    torch.cuda.synchronize()
    kern_ms, _ = tpasym.timing_read()
    tpasym.timing_enable(False)
    ms = e0.elapsed_time(e1) / steps
    b.check()
    reps = warmup + steps
    st = stats.cpu().numpy().view(np.uint64)
    c32 = counts.cpu().numpy().view(np.uint64)
    assert np.all(c32 % reps == 0)
    c32 = c32 // reps
    # the plain float64 request on the same events (one tp_bin per step): identical
    # counts; where no plane angle is binned this is the float32 tier against float64
    c64, s64 = tpasym.bin(ds, ch, bn, tpasym.TP_PREC_F64)
    same = bool(np.array_equal(c64.cpu().numpy().view(np.uint64), c32))
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        tpasym.bin(ds, ch, bn, tpasym.TP_PREC_F64, c64, s64, check=False)
    e1.record()
    torch.cuda.synchronize()
    ms64 = e0.elapsed_time(e1) / steps
    scp = []
    for mode in (0, 1):
        _, chi2, ndf, pv = tpasym.scp(c32.astype(np.int64), mode)
        scp.append({"split": "P-even" if mode == 0 else "P-odd", "chi2": float(chi2), "ndf": int(ndf),
                    "p": float(pv)})
    asym = tpasym.asym(c32.astype(np.int64))[0]
    achieved = n * BYTES_F32 / (kern_ms / 1e3) / 1e9
    log(f"{workload}: {ms:.3f} ms/step, {n / (ms / 1e3):.3e} events/s, {achieved:.0f} GB/s, "
        f"tier2 {int(st[4]) / reps / n:.2e}; float64 request {ms64:.3f} ms/step")
    phi = any(a.kind == synth.AXIS_ABSPHI for a in spec.axes)
    out = {"workload": workload, "events": n, "ms_per_step": ms, "value": n / (ms / 1e3),
           "unit": "events/s",
           "dtype": "f64 first pass and bins on f32 storage" if phi else "f32 sign tier, f64 recheck and bins",
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": achieved / HBM_PEAK_GBS, "bytes_per_event": BYTES_F32, "kernel_ms": kern_ms},
           "tiers": {"tier2_frac": int(st[4]) / reps / n, "tier3_per_step": int(st[5]) / reps,
                     "unresolved": int(st[6])},
           "counts_equal_f64_request": same,
           "f64_request": {"ms_per_step": ms64, "value": n / (ms64 / 1e3), "unit": "events/s",
                           "path": "tp_bin, TP_PREC_F64 (float64 sign and bins for every event)",
                           "speedup_of_leg": ms64 / ms},
           "scp": scp,
           "global": {"A_T": asym["A_T"][0], "Abar_T": asym["Abar_T"][0], "a_CP": asym["a_CP"][0],
                      "a_P": asym["a_P"][0]},
           "fp32": fp32_report([(ds, ch)], max_events=50_000_000)}
    if chunk > 0:
        # consecutive chunks of ``chunk`` events, one tp_bin call each
        parts = [tpasym.DeviceSample([c[k:k + chunk] for c in ds.comps], ds.tag[k:k + chunk])
                 for k in range(0, n, chunk)]
        cc, cs = tpasym.new_counts(bn, dev)
        for part in parts:
            tpasym.bin(part, ch, bn, prec, counts=cc, stats=cs, check=False)
        torch.cuda.synchronize()
        cc.zero_()
        cs.zero_()
        e0.record()
        for _ in range(steps):
            for part in parts:
                tpasym.bin(part, ch, bn, prec, counts=cc, stats=cs, check=False)
        e1.record()
        torch.cuda.synchronize()
        cms = e0.elapsed_time(e1) / steps
        cch = cc.cpu().numpy().view(np.uint64)
        out["chunked"] = {"chunk_events": chunk, "chunks": len(parts), "ms_per_step": cms,
                          "value": n / (cms / 1e3), "unit": "events/s",
                          "counts_equal_whole_pass": bool(np.all(cch % steps == 0)
                                                          and np.array_equal(cch // steps, c32))}
        log(f"{workload}: {len(parts)} chunks of {chunk} events: {cms:.3f} ms/step")
        del parts, cc, cs
    del ds, counts, stats, b, c64, s64
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lb_batch64_1e3to1e7",
                    help="named workload (paper_1612_04705_amd.synth.WORKLOADS)")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--precision", choices=["f32", "f64"], default="f32")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-events", type=float, default=2.5e7)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tuning", default=None,
                    help="fixed launch shape block,wg_per_cu,lds_copies,events_per_lane (skips the autotuner)")
    ap.add_argument("--no-f64-path", action="store_true",
                    help="skip the per-sample float64 comparison leg (profiling runs)")
    ap.add_argument("--energy-events", type=float, default=1e6,
                    help="events of the energy-test leg (0 skips it)")
    ap.add_argument("--energy-perms", type=int, default=1008,
                    help="permutations of the energy-test leg, 126 per launch of 128 columns")
    ap.add_argument("--no-ordered", action="store_true",
                    help="skip the leg that repeats the pass with the identical particles ordered on the fly")
    ap.add_argument("--energy-cpu-events", type=float, default=30000,
                    help="events of the bounded oracle timing beside the energy-test leg")
    ap.add_argument("--energy-bkg-perms", type=int, default=164,
                    help="permutations of the background-subtracted (eq. 3) leg, 41 per launch (0 skips it)")
    ap.add_argument("--no-pkpipi", action="store_true",
                    help="skip the 1e8-event Lambda_b -> p K- pi+ pi- leg (10 phi x 8 m(p pi-) bins, also in 16M-event chunks)")
    ap.add_argument("--no-d0", action="store_true",
                    help="skip the 5e8-event D0 -> K+ K- pi+ pi- leg (32 x 32 mass bins)")
    ap.add_argument("--no-fp32-report", action="store_true",
                    help="skip the measurement of the float32 tier's error on the workload")
    ap.add_argument("--copy-calib", action="store_true",
                    help="one extra untimed launch of the 1 GiB streaming reference (HBM byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the pass would shard by events and sum the uint64 histograms with one all-reduce)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1612_04705_amd import tpasym

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tpasym.load()
    prec = tpasym.TP_PREC_F32_RECHECK if args.precision == "f32" else tpasym.TP_PREC_F64
    specs, samples, items = make_workload(args.workload, dev, args.scale)
    nevents = sum(s.n for _, s in samples)
    f64_store = samples[0][1].comps[0][0].dtype == torch.float64
    bpe = BYTES_F64 if f64_store else BYTES_F32
    batch = tpasym.Batch(items)
    stream = torch.cuda.current_stream()

    tuning = None
    tuning_desc = "library defaults"
    if args.tuning:
        tuning = tpasym.Tuning(*[int(v) for v in args.tuning.split(",")])
        tuning_desc = tuning.as_dict()
    elif not args.no_autotune:
        t0 = time.time()
        largest = batch.autotune(prec)
        # runs without an explicit shape take each scheme group's tuned shape
        tuning_desc = {"per_scheme_autotuned": True, "largest_group": largest.as_dict()}
        if len({tuple(a.kind for a in sp.axes) for sp in specs}) > 1:     # several scheme groups
            tuning_desc["overlapping_groups"] = ("the largest launched at 16 workgroups per CU, the others "
                                                 "at most 4, whatever their tuned shapes")
        log(f"autotune: per scheme group, largest group {largest.as_dict()} in {time.time() - t0:.1f}s")
    graph = not args.no_graph
    for _ in range(args.warmup):
        batch.run(prec, tuning, graph)
    torch.cuda.synchronize()

    tpasym.timing_enable(True)
    tpasym.timing_reset()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(args.steps):
        batch.run(prec, tuning, graph)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    kern_ms, launches = tpasym.timing_read()
    tpasym.timing_enable(False)
    ms_per_step = total_ms / args.steps
    value = nevents / (ms_per_step / 1e3)
    log(f"{args.steps} steps: {ms_per_step:.4f} ms/step, kernel {kern_ms:.4f} ms over {launches} launches")

    # a plain streaming kernel for reference (and, under the profiler, the HBM
    # counter calibration): elementwise, reading 1 GiB and writing 1 GiB
    src = torch.empty(1 << 28, dtype=torch.int32, device=dev).fill_(7)
    dst = torch.empty_like(src)
    for _ in range(2 if args.copy_calib else 1):
        torch.bitwise_not(src, out=dst)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        torch.bitwise_not(src, out=dst)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * (1 << 30) / (c0.elapsed_time(c1) / 10 / 1e3) / 1e9
    del src, dst

    # statistics and parity-relevant totals (counts accumulate over warmup + steps)
    reps = args.warmup + args.steps
    st = np.stack([it[4].cpu().numpy().view(np.uint64) for it in items]).astype(np.float64).sum(axis=0)
    tier2, tier3, unres = st[4] / reps, st[5] / reps, st[6] / reps

    # plain all-float64 single-sample path, same inputs (non-persistent per-sample launches)
    f64_leg = None
    if not args.no_f64_path:
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        f64_items = [(ds, ch, bn, *tpasym.new_counts(bn, dev)) for ds, ch, bn, _, _ in items]
        for ds, ch, bn, c, s in f64_items:
            tpasym.bin(ds, ch, bn, tpasym.TP_PREC_F64, c, s, check=False)
        torch.cuda.synchronize()
        f64_steps = max(3, args.steps // 4)
        t0.record(stream)
        for _ in range(f64_steps):
            for ds, ch, bn, c, s in f64_items:
                tpasym.bin(ds, ch, bn, tpasym.TP_PREC_F64, c, s, check=False)
        t1.record(stream)
        torch.cuda.synchronize()
        f64_ms = t0.elapsed_time(t1) / f64_steps
        # both paths must agree bit for bit (whole numbers of passes on both sides)
        agree = True
        for a, b in zip(items, f64_items):
            ca, cb = a[3].cpu().numpy().view(np.uint64), b[3].cpu().numpy().view(np.uint64)
            agree = agree and bool(np.all(ca % reps == 0) and np.all(cb % (f64_steps + 1) == 0)
                                   and np.array_equal(ca // reps, cb // (f64_steps + 1)))
        f64_leg = {"value": nevents / (f64_ms / 1e3), "unit": "events/s", "ms_per_step": f64_ms,
                   "counts_equal_fast_path": bool(agree),
                   "path": "one tp_bin per sample with TP_PREC_F64, no graph: the plane-angle schemes evaluate "
                           "in float64 on both paths, so the ratio to the headline measures batching"}

    # the same pass with the identical particles (two pi- or two K-) ordered on
    # the fly by rest-frame energy: the stored order is then irrelevant
    ord_leg = None
    if not args.no_ordered:
        ord_items = [(ds, tpasym.channel(spec.channel.triple, spec.channel.planes, spec.channel.identical), bn,
                      *tpasym.new_counts(bn, dev)) for (ds, _, bn, _, _), (spec, _) in zip(items, samples)]
        nord = sum(1 for spec, _ in samples if spec.channel.identical is not None)
        ob = tpasym.Batch(ord_items)
        if tuning is None and not args.no_autotune:
            ob.autotune(prec)
        ob.run(prec, tuning, graph)
        torch.cuda.synchronize()
        osteps = max(5, args.steps // 4)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(osteps):
            ob.run(prec, tuning, graph)
        t1.record(stream)
        torch.cuda.synchronize()
        o_ms = t0.elapsed_time(t1) / osteps
        # the generator stored them in order (float64, before the boost): the
        # counts may differ only by events whose two energies tie to float32 rounding
        moved = sum(int(np.abs(a[3].cpu().numpy().view(np.uint64).astype(np.int64) // reps
                               - b[3].cpu().numpy().view(np.uint64).astype(np.int64) // (osteps + 1)).sum())
                    for a, b in zip(items, ord_items))
        ord_leg = {"value": nevents / (o_ms / 1e3), "unit": "events/s", "ms_per_step": o_ms,
                   "samples_with_identical_particles": nord, "count_changes_vs_stored_order": moved}
        log(f"ordered pass: {o_ms:.4f} ms/step ({nord} samples ordered on the fly), count changes {moved}")

    wl = args.workload
    if args.scale != 1.0:
        wl += f"_scale{args.scale:g}"
    achieved = nevents * bpe / (kern_ms / 1e3) / 1e9 if kern_ms > 0 else None
    traffic = traffic_from_profiles(wl)
    out = {
        "metric": "events/s for triple-product asymmetry pass; % of HBM peak; vs plain FP64 path",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # every binning scheme of the batched workload bins the plane angle, where the
        # pass decides the sign and the bins in float64 (first pass, then double-word
        # and exact integers) on the float32-stored events
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl, "samples": len(samples), "events": nevents,
                   "storage": "f64" if f64_store else "f32",
                   "path": ("persistent batched pass, one kernel per binning scheme on parallel branches, HIP graph"
                            if graph else "persistent batched pass, one kernel per binning scheme on parallel streams"),
                   "requested_precision": ("TP_PREC_F32_RECHECK" if args.precision == "f32" else "TP_PREC_F64"),
                   "arithmetic": "float64 certified tiers on float32 storage (plane-angle schemes: the float32 "
                                 "sign tier does not run), double-word and exact integers for deferred events",
                   "tuning": tuning_desc},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": traffic,
                     "streaming_reference_GBps": copy_gbs,
                     "bytes_per_event": bpe, "kernel_ms": kern_ms, "kernel_launches": launches},
        "fp64_single_sample": f64_leg,
        "ordered_identical": ord_leg,
        "tiers": {"tier2_per_step": tier2, "tier3_per_step": tier3, "unresolved_per_step": unres},
        "paper_context": "energy test (different algorithm): 1e6 events, one permutation ~30 min on "
                         "NVIDIA M2070 / K40c (Sect. 6); no timing is given for the triple-product pass",
    }
    out["scp"] = scp_report(items, reps)
    if not args.no_fp32_report:
        out["fp32_report"] = fp32_report(items)
        log(f"fp32 report: {out['fp32_report']['rechecked_frac']:.2e} rechecked, "
            f"{out['fp32_report']['raw_fp32_wrong_signs']} raw wrong signs, "
            f"{out['fp32_report']['wrong_signs_outside_recheck']} outside the recheck")
    batch.check()
    if not args.no_cpu:
        want = {}
        cpu, orc = cpu_baseline(samples, args.cpu_events, set(range(len(samples))))
        out["cpu_baseline"] = {k: v for k, v in cpu.items() if k != "seconds"}
        ok = True
        for i, r in orc.items():
            c = items[i][3].cpu().numpy().view(np.uint64)
            if not np.all(c % reps == 0):
                ok = False
                continue
            got = (c // reps).astype(np.int64).tolist()
            wantc = [v for row in r["counts"] for v in row]
            ok = ok and got == wantc
        out["parity_vs_oracle"] = {"samples_checked": len(orc), "counts_bit_exact": bool(ok)}
        log(f"cpu baseline {cpu['value']:.3e} events/s on {cpu['cores']} threads ({cpu['seconds']:.1f}s: "
            f"float64 pass {cpu['seconds_float64_pass']:.1f}s, serial exact stage {cpu['seconds_exact_serial']:.1f}s "
            f"for {cpu['flagged']} flagged events); one thread {cpu['single_thread']['value']:.3e} events/s")
    if not args.no_pkpipi:
        out["pkpipi_leg"] = single_leg(dev, "lb_pkpipi_1e8_phi10xm8", max(3, args.steps // 2), 2, chunk=1 << 24)
    if not args.no_d0:
        out["d0_leg"] = single_leg(dev, "d0_kkpipi_5e8_m32x32", max(3, args.steps // 2), 2)
    if args.energy_events > 0:
        out["energy_test"] = energy_leg(int(args.energy_events), args.energy_perms, dev,
                                        cpu_events=0 if args.no_cpu else args.energy_cpu_events)
        if args.energy_bkg_perms > 0:
            out["energy_test_background"] = energy_bkg_leg(int(args.energy_events), args.energy_bkg_perms, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
