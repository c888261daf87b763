"""The allocation-free entry point tp_bin_noalloc against tp_bin, through the C-ABI:
identical counts and statistics on two calls in a row (the second smaller, with another
binning scheme), both precisions."""
import numpy as np
import pytest
import torch

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


def test_noalloc_matches_tp_bin_twice(tp):
    cases = [("Lb_pKpipi", 50021, [synth.abscos_axis(0, 5), synth.absphi_axis(10)], 51),
             ("Lb_ppipipi", 3001, [synth.absphi_axis(10), None], 52)]
    for name, n, axes, seed in cases:
        ch = synth.CHANNELS[name]
        if axes[-1] is None:
            axes = [axes[0], synth.lb_mass03_axis(ch)]
        s = synth.generate(ch, n, seed, inj=synth.INJ_SIN)
        ds = tp.DeviceSample.from_sample(s)
        bn = tp.Binning(axes)
        chan = tp.channel(ch.triple, ch.planes)
        for prec in (tp.TP_PREC_F32_RECHECK, tp.TP_PREC_F64):
            c1, s1 = tp.bin(ds, chan, bn, prec)
            c2, s2 = tp.bin_noalloc(ds, chan, bn, prec)
            print(f"[noalloc] {name} n={n} prec={prec} stats={u64(s2)}", flush=True)
            assert u64(c2) == u64(c1)
            assert u64(s2) == u64(s1)
            assert u64(s2)[0] == n and u64(s2)[6] == 0
