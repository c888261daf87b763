"""The exact integer tier (csrc/tp_exact.h) compiled for the host, against the
oracle's exact-rational decisions (Fractions).  CPU only."""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import torch

import oracle
from oracle import exact
from paper_1612_04705_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "exact_harness.cpp")
OUT = os.path.join(ROOT, "tests", "_build", "libexact_harness.so")


@pytest.fixture(scope="module")
def hx():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC", "-I",
                    os.path.join(ROOT, "paper_1612_04705_amd", "csrc"), SRC, "-o", OUT], check=True)
    lib = ctypes.CDLL(OUT)
    lib.hx_decide.restype = ctypes.c_int
    return lib


def perm_sign(p):
    s = 1
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


def decide(hx, comps_slot, tag, triple, planes, axes, is_f32, dw=False):
    """Call the harness with the kernel-order layout (kernel slot t = channel slot planes[t]).

    dw: use the double-word tier (returns class 7 when it does not decide)."""
    inv = [0] * 4
    for t, s in enumerate(planes):
        inv[s] = t
    k = [comps_slot[planes[t]][c] for t in range(4) for c in range(4)]
    D = 6 - sum(triple)
    sigma = perm_sign([D, *triple]) * perm_sign(list(planes))
    kinds = (ctypes.c_int32 * 2)()
    nb = (ctypes.c_int32 * 2)()
    sl = (ctypes.c_int32 * 2)()
    eds = []
    for a, (kind, slots, edges) in enumerate(axes):
        kinds[a] = kind
        nb[a] = len(edges) - 1
        if kind == synth.AXIS_MASS:
            m = 0
            for s in range(4):
                if slots & (1 << s):
                    m |= 1 << inv[s]
            sl[a] = m
        elif kind == synth.AXIS_ABSCOS:
            sl[a] = inv[slots]
        eds.append((ctypes.c_double * len(edges))(*edges))
    while len(eds) < 2:
        eds.append(None)
    b = ctypes.c_int()
    if dw:
        c = hx.hx_decide_dw((ctypes.c_double * 16)(*k), int(tag), sigma, len(axes), kinds, nb, sl,
                            eds[0], eds[1], ctypes.byref(b))
    else:
        c = hx.hx_decide((ctypes.c_double * 16)(*k), int(is_f32), int(tag), sigma, len(axes), kinds, nb, sl,
                         eds[0], eds[1], ctypes.byref(b))
    return c, (b.value if axes and c < 4 else None)


def _check(hx, comps, tag, triple, planes, axes, is_f32, idx):
    """Both the exact integer tier and (where it decides) the double-word tier
    agree with the oracle's Fractions; returns how many the double-word tier left."""
    ax = [(a.kind, a.slots, list(map(float, a.edges))) for a in axes]
    undecided = 0
    for i in idx:
        ev = [[float(comps[s, c, i]) for c in range(4)] for s in range(4)]
        want = exact.exact_decision(ev, int(tag[i]), triple, planes, ax)
        got = decide(hx, ev, int(tag[i]), triple, planes, ax, is_f32)
        want = (want[0], want[1] if want[0] < 4 else None)
        assert got == want, (i, got, want)
        if all(np.isfinite(v) for row in ev for v in row):
            gdw = decide(hx, ev, int(tag[i]), triple, planes, ax, is_f32, dw=True)
            if gdw[0] == 7:
                undecided += 1
            else:
                assert gdw == want, ("double-word", i, gdw, want)
    return undecided


@pytest.mark.parametrize("chname,axes_fn,dtype", [
    ("Lb_pKpipi", lambda ch: [synth.absphi_axis(10), synth.lb_mass03_axis(ch)], torch.float32),
    ("Lb_ppipipi", lambda ch: [synth.absphi_axis(12)], torch.float64),
    ("Lb_ppiKK", lambda ch: [synth.abscos_axis(0, 5), synth.absphi_axis(10)], torch.float32),
    ("D0_KKpipi", lambda ch: [synth.mass_axis((0, 1), 987.354, 1585.7, 32),
                              synth.mass_axis((2, 3), 279.14, 877.486, 32)], torch.float32),
])
def test_exact_tier_random_events(hx, chname, axes_fn, dtype):
    ch = synth.CHANNELS[chname]
    s = synth.generate(ch, 150, 31, dtype=dtype)
    comps, tag = s.numpy()
    left = _check(hx, comps, tag, ch.triple, ch.planes, axes_fn(ch), dtype == torch.float32, range(150))
    assert left == 0        # random events never need the integer tier


@pytest.mark.parametrize("gamma", [1e3, 1e5])
def test_double_word_tier_extreme_boost(hx, gamma):
    ch = synth.CHANNELS["Lb_pKpipi"]
    s = synth.generate(ch, 60, 34, fixed_gamma=gamma)
    comps, tag = s.numpy()
    left = _check(hx, comps, tag, ch.triple, ch.planes, [synth.absphi_axis(10), synth.lb_mass03_axis(ch)],
                  True, range(60))
    assert left <= 3


def test_exact_tier_handbuilt(hx):
    from test_oracle_pins import _load_handbuilt, _as_sample
    rows = _load_handbuilt()
    comps, tag = _as_sample(rows)
    for axes in ([synth.absphi_axis(12)], [synth.absphi_axis(10)],
                 [synth.Axis(synth.AXIS_MASS, np.array([5.0, 6.0, 7.0]), 0b1001)],
                 [synth.Axis(synth.AXIS_MASS, np.array([4.0, 5.0, 6.0]), 0b1001)],
                 [synth.Axis(synth.AXIS_ABSCOS, np.linspace(0, 1, 6), 0)],
                 [synth.Axis(synth.AXIS_ABSCOS, np.array([0.0, 0.2, 0.4, 0.6, 0.8, 1.0]), 0)]):
        for planes in ((0, 1, 2, 3), (2, 3, 0, 1), (1, 0, 3, 2)):
            _check(hx, comps, tag, (0, 1, 2), planes, axes, True, range(len(rows)))
            _check(hx, comps, tag, (0, 2, 3), planes, axes, True, range(len(rows)))


def test_exact_tier_degenerate(hx):
    ch = synth.CHANNELS["Lb_pKpipi"]
    s = synth.generate(ch, 40, 32)
    comps, tag = s.numpy()
    c = comps.copy()
    c[:, 3, :20] = 0.0                     # coplanar: zero class
    c[1, 2, 21] = np.nan                   # invalid
    c[:, 0, 22] = 0.0                      # space-like P: invalid
    c[:, 1:, 23] = 0.0                     # all momenta zero
    c[2, :, 24] = c[1, :, 24]              # two identical daughters: zero
    tag = tag.copy()
    tag[25] = 3
    # tiny and huge components within the allowed exponent span
    c[0, 1, 26] = np.float32(1e-30)
    c[3, 2, 27] = np.float32(3e-25)
    ax = [synth.absphi_axis(10), synth.lb_mass03_axis(ch)]
    _check(hx, c, tag, ch.triple, ch.planes, ax, True, range(40))


def test_exact_tier_span_limit(hx):
    """An event whose components span more than 2^136 (float32) is reported unresolved."""
    ch = synth.CHANNELS["Lb_pKpipi"]
    s = synth.generate(ch, 2, 33)
    comps, tag = s.numpy()
    c = comps.copy()
    c[0, 1, 0] = np.float32(1e-40)      # subnormal next to ~1e4 values: span > 136
    ev = [[float(c[sl, k, 0]) for k in range(4)] for sl in range(4)]
    got = decide(hx, ev, int(tag[0]), ch.triple, ch.planes, [], True)
    assert got[0] == 6


def test_exact_tiers_under_sanitizers(hx, tmp_path):
    """The exact and double-word tiers built with the address and undefined-behaviour
    sanitizers (host build, g++) on random, extreme-boost, hand-built and degenerate
    events: no sanitizer report, and the same decisions as the plain build (which the
    tests above check against the oracle's Fractions)."""
    import struct
    exe = os.path.join(ROOT, "tests", "_build", "exact_san")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I",
                    os.path.join(ROOT, "paper_1612_04705_amd", "csrc"), "-I", os.path.join(ROOT, "tests", "host"),
                    os.path.join(ROOT, "tests", "host", "exact_sanitize_main.cpp"), "-o", exe], check=True)
    reqs, want = [], []

    def add(ev, tag, triple, planes, axes, is_f32):
        inv = [0] * 4
        for t, s in enumerate(planes):
            inv[s] = t
        k = [ev[planes[t]][c] for t in range(4) for c in range(4)]
        sigma = perm_sign([6 - sum(triple), *triple]) * perm_sign(list(planes))
        kinds, nb, sl, eds = [0, 0], [0, 0], [0, 0], []
        for a, (kind, slots, edges) in enumerate(axes):
            kinds[a], nb[a] = kind, len(edges) - 1
            sl[a] = sum(1 << inv[s] for s in range(4) if slots & (1 << s)) if kind == synth.AXIS_MASS else \
                (inv[slots] if kind == synth.AXIS_ABSCOS else 0)
            eds.append(edges)
        b = struct.pack("<16d10i", *k, int(is_f32), int(tag), sigma, len(axes), *kinds, *nb, *sl)
        for e in eds:
            b += struct.pack(f"<{len(e)}d", *e)
        reqs.append(b)
        c, bn = decide(hx, ev, tag, triple, planes, axes, is_f32)
        fin = all(np.isfinite(v) for row in ev for v in row)
        cd, bd = decide(hx, ev, tag, triple, planes, axes, is_f32, dw=True) if fin else (-1, None)
        want.append((c, bn, cd, bd))

    for chname, axes_fn, n, gamma in [
            ("Lb_pKpipi", lambda ch: [synth.absphi_axis(10), synth.lb_mass03_axis(ch)], 40, None),
            ("Lb_ppiKK", lambda ch: [synth.abscos_axis(0, 5), synth.absphi_axis(10)], 40, None),
            ("D0_KKpipi", lambda ch: [synth.mass_axis((0, 1), 987.354, 1585.7, 32),
                                      synth.mass_axis((2, 3), 279.14, 877.486, 32)], 30, None),
            ("Lb_pKpipi", lambda ch: [synth.absphi_axis(10), synth.lb_mass03_axis(ch)], 20, 1e5)]:
        ch = synth.CHANNELS[chname]
        s = synth.generate(ch, n, 35, fixed_gamma=gamma) if gamma else synth.generate(ch, n, 35)
        comps, tag = s.numpy()
        c = comps.copy()
        c[:, 3, :4] = 0.0                              # coplanar
        c[1, 2, 5] = np.nan                            # invalid
        c[:, 0, 6] = 0.0                               # space-like P
        c[0, 1, 7] = np.float32(1e-40)                 # beyond the exponent span
        ax = [(a.kind, a.slots, list(map(float, a.edges))) for a in axes_fn(ch)]
        for i in range(n):
            ev = [[float(c[sl_, k, i]) for k in range(4)] for sl_ in range(4)]
            add(ev, int(tag[i]), ch.triple, ch.planes, ax, True)
    from test_oracle_pins import _load_handbuilt, _as_sample
    comps, tag = _as_sample(_load_handbuilt())
    for axes in ([synth.absphi_axis(12)], [synth.Axis(synth.AXIS_MASS, np.array([5.0, 6.0, 7.0]), 0b1001)],
                 [synth.Axis(synth.AXIS_ABSCOS, np.array([0.0, 0.2, 0.4, 0.6, 0.8, 1.0]), 0)]):
        ax = [(a.kind, a.slots, list(map(float, a.edges))) for a in axes]
        for i in range(comps.shape[2]):
            ev = [[float(comps[sl_, k, i]) for k in range(4)] for sl_ in range(4)]
            add(ev, int(tag[i]), (0, 1, 2), (0, 1, 2, 3), ax, True)
    fin, fout = tmp_path / "req.bin", tmp_path / "res.bin"
    fin.write_bytes(struct.pack("<i", len(reqs)) + b"".join(reqs))
    r = subprocess.run([exe, str(fin), str(fout)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-2000:]
    res = np.frombuffer(fout.read_bytes(), dtype=np.int32).reshape(-1, 4)
    assert len(res) == len(want)
    for (c, bn, cd, bd), got in zip(want, res):
        assert got[0] == c and (bn is None or got[1] == bn)
        assert got[2] == cd and (bd is None or cd >= 4 or got[3] == bd)
