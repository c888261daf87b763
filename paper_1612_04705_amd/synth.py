"""Seeded synthetic four-body decay samples and the workload definitions.

This module produces INPUT DATA only: stored four-vectors, flavour tags, the
channel slot conventions and the bin-edge tables.  It holds none of the T-odd
method's arithmetic (no triple product, no class, no bin assignment, no
asymmetry); the CPU oracle and the HIP path each do that on their own.

Phase space.  A pseudo-scalar M decays to four particles, (a b)(c d).  The
phase-space density factorises into two-body steps (the same fact GENBOD,
F. James, CERN 68-15 (1968), is built on): M -> Q1 Q2 with Q1 -> a b and
Q2 -> c d, weight  p*(M; m12, m34) p*(m12; ma, mb) p*(m34; mc, md)  in
d m12 d m34, isotropic two-body decays.  The masses are drawn by accept-reject
against a numerical maximum of that weight; the angles are drawn directly.
The azimuth between the two decay planes is an explicit generated variable
(``phi_gen``), built so that the acoplanarity angle of the paper's Sect. 5
(signed angle from plane (a,b) to plane (c,d) about the (a b) direction in the
M rest frame) equals ``phi_gen``.  That is what lets an asymmetry be injected
by accept-reject in phi without this module measuring anything.

The parent is given |p| ~ Exp(mean 100 GeV) along an isotropic direction and
every daughter is boosted to the lab in float64; storage is then rounded to
float32 (or kept float64).  Identical particles (two pi- or two K-) are put in
canonical order: the one with the larger energy in the M rest frame goes to the
lower slot ("fast" first), which fixes the sign convention of C_T for those
channels (swapping identical particles would flip it).

Random numbers: torch.Generator seeded per sample (CPU and CUDA streams differ,
so a seed identifies a sample only together with the device it was drawn on).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

# ---------------------------------------------------------------- masses (MeV)
M_LB = 5619.6
M_D0 = 1864.84
M_P = 938.272
M_PI = 139.570
M_K = 493.677


@dataclass(frozen=True)
class Channel:
    """Slot layout of one decay channel.

    slots hold (E, px, py, pz) of the four final-state particles in this order;
    the conjugate decay stores the C-conjugate particles in the same slots.
    ``triple`` = slots (A, B, C) of C_T = p_A . (p_B x p_C) in the M rest frame
    (Sect. 5, eq. (4)); ``planes`` = (i, j, k, l): the acoplanarity angle is the
    angle between the (i, j) and (k, l) decay planes.  ``identical`` names two
    slots holding identical particles (ordered fast, slow) or is None.
    """
    name: str
    parent: float
    masses: tuple
    triple: tuple
    planes: tuple = (0, 1, 2, 3)
    identical: tuple | None = None


CHANNELS = {
    # Lambda_b0 -> p pi- pi+ pi-: p, pi-(fast), pi+, pi-(slow)
    "Lb_ppipipi": Channel("Lb_ppipipi", M_LB, (M_P, M_PI, M_PI, M_PI), (0, 1, 2), identical=(1, 3)),
    # Lambda_b0 -> p K- pi+ pi-
    "Lb_pKpipi": Channel("Lb_pKpipi", M_LB, (M_P, M_K, M_PI, M_PI), (0, 1, 2)),
    # Lambda_b0 -> p pi- K+ K-
    "Lb_ppiKK": Channel("Lb_ppiKK", M_LB, (M_P, M_PI, M_K, M_K), (0, 1, 2)),
    # Lambda_b0 -> p K- K+ K-: p, K-(fast), K+, K-(slow)
    "Lb_pKKK": Channel("Lb_pKKK", M_LB, (M_P, M_K, M_K, M_K), (0, 1, 2), identical=(1, 3)),
    # D0 -> K+ K- pi+ pi-, C_T = p_K+ . (p_pi+ x p_pi-)
    "D0_KKpipi": Channel("D0_KKpipi", M_D0, (M_K, M_K, M_PI, M_PI), (0, 2, 3)),
    # D0 -> pi+ pi- pi+ pi- (charge order), for the energy-test coordinates: the
    # labelling of the identical pions is left to the coordinates' own rule
    "D0_pipipipi": Channel("D0_pipipipi", M_D0, (M_PI, M_PI, M_PI, M_PI), (0, 1, 2)),
}

# axis kinds (same numbering as the C-ABI)
AXIS_ABSPHI, AXIS_MASS, AXIS_ABSCOS = 0, 1, 2


@dataclass
class Axis:
    """One binning axis.

    ABSPHI: folded acoplanarity |Phi| in [0, pi]; ``edges`` are the cosines
      c_0 = 1 > c_1 > ... > c_n = -1 of the angle edges; bin j holds
      c_{j+1} < cos|Phi| <= c_j (the last bin also holds cos|Phi| = -1).
    MASS: invariant mass of the slots in bit mask ``slots``; increasing edges
      e_0 >= 0; bin j holds e_j <= m < e_{j+1} (last bin closed); outside ->
      out of range.
    ABSCOS: |cos theta| of slot ``slots`` in the M rest frame against the M
      flight direction; edges 0 = e_0 < ... < e_n = 1; bin j holds
      e_j <= |cos| < e_{j+1} (last closed).
    """
    kind: int
    edges: np.ndarray
    slots: int = 0

    @property
    def nbins(self) -> int:
        return len(self.edges) - 1


def cos_edges(nfold: int) -> np.ndarray:
    """c_k = cos(k pi / nfold) correctly rounded to float64 (mpmath), k = 0..nfold.

    Exact 1, -1 at the ends and an exact 0 at pi/2 when nfold is even.
    """
    import mpmath
    mpmath.mp.prec = 200
    out = []
    for k in range(nfold + 1):
        if 2 * k == nfold:
            out.append(0.0)
            continue
        v = mpmath.cos(mpmath.pi * k / nfold)
        out.append(float(v))           # mpmath -> float rounds to nearest at 200 bits
    out[0], out[-1] = 1.0, -1.0
    return np.array(out, dtype=np.float64)


def absphi_axis(nphi_full: int) -> Axis:
    """|Phi| axis equivalent to ``nphi_full`` uniform phi bins in [0, 2 pi)."""
    if nphi_full % 2:
        raise ValueError("the folded |Phi| axis needs an even number of phi bins")
    return Axis(AXIS_ABSPHI, cos_edges(nphi_full // 2))


def mass_axis(slots: tuple, lo: float, hi: float, nbins: int) -> Axis:
    mask = 0
    for s in slots:
        mask |= 1 << s
    return Axis(AXIS_MASS, np.linspace(lo, hi, nbins + 1), mask)


def abscos_axis(slot: int, nbins: int) -> Axis:
    return Axis(AXIS_ABSCOS, np.linspace(0.0, 1.0, nbins + 1), slot)


# ------------------------------------------------------------------ kinematics
def _pstar(M, m1, m2):
    """Two-body breakup momentum of M -> m1 m2 (tensor or float)."""
    a = (M * M - (m1 + m2) ** 2) * (M * M - (m1 - m2) ** 2)
    if isinstance(a, torch.Tensor):
        return torch.sqrt(torch.clamp(a, min=0.0)) / (2 * M)
    return math.sqrt(max(a, 0.0)) / (2 * M)


def _weight_max(M, ma, mb, mc, md) -> float:
    """Maximum of the two-step phase-space weight, found on a fine grid, +3 %."""
    lo12, lo34 = ma + mb, mc + md
    g = np.linspace(0.0, 1.0, 801)
    m12 = lo12 + (M - lo34 - lo12) * g[:, None]
    m34 = lo34 + (M - lo12 - lo34) * g[None, :]
    ok = m12 + m34 <= M

    def ps(Mx, m1, m2):
        a = (Mx * Mx - (m1 + m2) ** 2) * (Mx * Mx - (m1 - m2) ** 2)
        return np.sqrt(np.clip(a, 0, None)) / (2 * Mx)
    w = ps(M, m12, m34) * ps(m12, ma, mb) * ps(m34, mc, md)
    return float(np.max(np.where(ok, w, 0.0))) * 1.03


def _boost_z(E, px, py, pz, beta, gamma):
    """Boost along +z with velocity beta (per-event tensors)."""
    return gamma * (E + beta * pz), px, py, gamma * (pz + beta * E)


def _boost(E, px, py, pz, bx, by, bz):
    """General pure boost by velocity (bx, by, bz): rest frame -> moving frame."""
    b2 = bx * bx + by * by + bz * bz
    gamma = 1.0 / torch.sqrt(1.0 - b2)
    bp = bx * px + by * py + bz * pz
    safe = torch.where(b2 > 0, b2, torch.ones_like(b2))
    k = torch.where(b2 > 0, (gamma - 1.0) * bp / safe, torch.zeros_like(b2)) + gamma * E
    return gamma * (E + bp), px + k * bx, py + k * by, pz + k * bz


@dataclass
class Injection:
    """Accept-reject weight 1 + eps_tag * f(phi_gen) per flavour.

    f = 'sin' (sin phi), 'sin2' (sin 2 phi) or 'sgn' (sign of sin phi).
    """
    f: str = "none"
    eps_m: float = 0.0
    eps_mbar: float = 0.0

    def weight(self, phi, tag):
        if self.f == "none":
            return torch.ones_like(phi)
        if self.f == "sin":
            g = torch.sin(phi)
        elif self.f == "sin2":
            g = torch.sin(2 * phi)
        elif self.f == "sgn":
            g = torch.sign(torch.sin(phi))
        else:
            raise ValueError(self.f)
        eps = torch.where(tag == 0, torch.full_like(phi, self.eps_m), torch.full_like(phi, self.eps_mbar))
        return 1.0 + eps * g

    @property
    def wmax(self) -> float:
        return 1.0 + max(abs(self.eps_m), abs(self.eps_mbar))


@dataclass
class Sample:
    """One stored sample: comps[slot][c] (c = E, px, py, pz), tag (int8: 0 = M, 1 = Mbar)."""
    channel: Channel
    comps: list            # 4 x 4 tensors of dtype float32/float64
    tag: torch.Tensor      # int8
    phi_gen: torch.Tensor | None = None   # generated plane angle (generation labelling), float64
    gamma: torch.Tensor | None = None      # parent Lorentz factor, float64
    m12: torch.Tensor | None = None        # generated pair masses (generation labelling), float64
    m34: torch.Tensor | None = None

    @property
    def n(self) -> int:
        return int(self.tag.numel())

    def arrays(self):
        """List of the 16 component arrays in slot-major order."""
        return [self.comps[s][c] for s in range(4) for c in range(4)]

    def numpy(self):
        a = np.stack([t.cpu().numpy() for t in self.arrays()])
        return a.reshape(4, 4, -1), self.tag.cpu().numpy()


def _candidates(ch: Channel, n: int, gen: torch.Generator, device, wmax_ps: float):
    """Draw ``n`` pure phase-space events in the M rest frame (float64)."""
    M = ch.parent
    ma, mb, mc, md = ch.masses
    lo12, lo34 = ma + mb, mc + md
    f64 = dict(dtype=torch.float64, device=device)
    out = []
    have = 0
    while have < n:
        k = max(4096, int((n - have) * 5))
        u = torch.rand(3, k, generator=gen, **f64)
        m12 = lo12 + (M - lo34 - lo12) * u[0]
        m34 = lo34 + (M - lo12 - lo34) * u[1]
        w = _pstar(M, m12, m34) * _pstar(m12, ma, mb) * _pstar(m34, mc, md)
        w = torch.where(m12 + m34 < M, w, torch.zeros_like(w))
        if bool((w > wmax_ps).any()):
            raise RuntimeError("phase-space weight above its maximum")
        keep = u[2] * wmax_ps < w
        out.append((m12[keep], m34[keep]))
        have += int(keep.sum())
    m12 = torch.cat([o[0] for o in out])[:n]
    m34 = torch.cat([o[1] for o in out])[:n]
    return m12, m34


def generate(ch: Channel, n: int, seed: int, *, frac_m: float = 0.5, inj: Injection | None = None,
             dtype=torch.float32, device="cpu", mean_p: float = 1.0e5,
             fixed_gamma: float | None = None) -> Sample:
    """Generate ``n`` stored events of channel ``ch``.

    frac_m: probability of flavour M (tag 0).  inj: accept-reject injection in
    phi_gen.  fixed_gamma: if given, every parent has this Lorentz factor
    (stress inputs); otherwise |p_parent| ~ Exp(mean_p).
    """
    inj = inj or Injection()
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f64 = dict(dtype=torch.float64, device=device)
    M = ch.parent
    ma, mb, mc, md = ch.masses
    wmax_ps = _weight_max(M, ma, mb, mc, md)

    parts = []
    have = 0
    while have < n:
        k = max(1024, int((n - have) * inj.wmax * 1.05) + 64)
        m12, m34 = _candidates(ch, k, gen, device, wmax_ps)
        u = torch.rand(11, k, generator=gen, **f64)
        tag = (u[0] >= frac_m).to(torch.int8)
        phi = 2 * math.pi * u[1]
        keep = u[2] * inj.wmax < inj.weight(phi, tag)
        parts.append(dict(m12=m12[keep], m34=m34[keep], tag=tag[keep], phi=phi[keep],
                          u=u[3:, keep]))
        have += int(keep.sum())
    cat = {key: torch.cat([p[key] for p in parts], dim=-1)[..., :n] for key in ("m12", "m34", "tag", "phi", "u")}
    m12, m34, tag, phi, u = cat["m12"], cat["m34"], cat["tag"], cat["phi"], cat["u"]

    # M rest frame, Q1 along +z
    q = _pstar(M, m12, m34)
    E1 = torch.sqrt(m12 * m12 + q * q)
    E2 = torch.sqrt(m34 * m34 + q * q)
    k1 = _pstar(m12, ma, mb)
    k2 = _pstar(m34, mc, md)
    c1 = 2 * u[0] - 1
    s1 = torch.sqrt(torch.clamp(1 - c1 * c1, min=0.0))
    c2 = 2 * u[1] - 1
    s2 = torch.sqrt(torch.clamp(1 - c2 * c2, min=0.0))
    chi1 = 2 * math.pi * u[2]
    # plane angle from (a,b) to (c,d) about +z equals phi when chi2 = chi1 + phi - pi
    chi2 = chi1 + phi - math.pi

    def two_body(k, m1, m2, ct, st, chi):
        e1 = torch.sqrt(m1 * m1 + k * k)
        e2 = torch.sqrt(m2 * m2 + k * k)
        px, py, pz = k * st * torch.cos(chi), k * st * torch.sin(chi), k * ct
        return (e1, px, py, pz), (e2, -px, -py, -pz)

    a, b = two_body(k1, ma, mb, c1, s1, chi1)
    c, d = two_body(k2, mc, md, c2, s2, chi2)
    be1, ga1 = q / E1, E1 / m12
    be2, ga2 = -q / E2, E2 / m34
    a = _boost_z(*a, be1, ga1)
    b = _boost_z(*b, be1, ga1)
    c = _boost_z(*c, be2, ga2)
    d = _boost_z(*d, be2, ga2)
    vecs = [list(a), list(b), list(c), list(d)]

    # isotropic orientation: rotate +z onto a random direction (azimuth already random via chi1)
    ct = 2 * u[3] - 1
    st = torch.sqrt(torch.clamp(1 - ct * ct, min=0.0))
    ph = 2 * math.pi * u[4]
    cp, sp = torch.cos(ph), torch.sin(ph)
    # rotation R = Rz(ph) Ry(theta)
    for v in vecs:
        x, y, z = v[1], v[2], v[3]
        x1 = ct * x + st * z
        z1 = -st * x + ct * z
        v[1], v[2], v[3] = cp * x1 - sp * y, sp * x1 + cp * y, z1

    # identical particles: fast (larger rest-frame energy) first
    if ch.identical is not None:
        i, j = ch.identical
        swap = vecs[j][0] > vecs[i][0]
        for cc in range(4):
            vi, vj = vecs[i][cc], vecs[j][cc]
            vecs[i][cc] = torch.where(swap, vj, vi)
            vecs[j][cc] = torch.where(swap, vi, vj)

    # parent momentum and lab boost
    if fixed_gamma is None:
        pmag = -mean_p * torch.log1p(-u[5])
    else:
        pmag = torch.full_like(u[5], M * math.sqrt(fixed_gamma * fixed_gamma - 1.0))
    pct = 2 * u[6] - 1
    pst = torch.sqrt(torch.clamp(1 - pct * pct, min=0.0))
    pph = 2 * math.pi * u[7]
    EP = torch.sqrt(M * M + pmag * pmag)
    bx = pmag * pst * torch.cos(pph) / EP
    by = pmag * pst * torch.sin(pph) / EP
    bz = pmag * pct / EP
    comps = []
    for v in vecs:
        E, px, py, pz = _boost(v[0], v[1], v[2], v[3], bx, by, bz)
        comps.append([t.to(dtype).contiguous() for t in (E, px, py, pz)])
    return Sample(ch, comps, tag.contiguous(), phi_gen=phi, gamma=EP / M, m12=m12, m34=m34)


# ------------------------------------------------------------ workload configs
@dataclass
class SampleSpec:
    channel: Channel
    n: int
    seed: int
    axes: list
    frac_m: float = 0.5
    inj: Injection = field(default_factory=Injection)
    dtype: torch.dtype = torch.float32


INJ_SIN = Injection("sin", 0.1, 0.05)       # w = 1 + 0.1 sin phi (M), 1 + 0.05 sin phi (Mbar)
INJ_SIN2 = Injection("sin2", 0.03, 0.0)     # w = 1 + 0.03 sin 2 phi on M only
INJ_SGN = Injection("sgn", 0.002, 0.002)    # w = 1 + 0.002 sgn(sin phi) for both flavours


def lb_mass03_axis(ch: Channel, nbins: int = 8) -> Axis:
    m = ch.masses
    return mass_axis((0, 3), m[0] + m[3], ch.parent - m[1] - m[2], nbins)


# Named workloads: channel, size, storage, binning, injection.
WORKLOADS = {
    "lb_ppipipi_f64_1e5": "Lambda_b -> p pi- pi+ pi-, 1e5 events, float64 storage, 5 |Phi| bins (10 phi)",
    "lb_ppipipi_1e7_phi12": "Lambda_b -> p pi- pi+ pi-, 1e7 events, 6 |Phi| bins (12 phi), sin(phi) injection",
    "lb_pkpipi_1e8_phi10xm8": "Lambda_b -> p K- pi+ pi-, 1e8 events, 5 |Phi| x 8 m(p pi-), sin(2 phi) on M",
    "lb_batch64_1e3to1e7": "64 Lambda_b samples (4 channels x 3 binnings), sizes log-uniform in [1e3, 1e7]",
    "d0_kkpipi_5e8_m32x32": "D0 -> K+ K- pi+ pi-, 5e8 events, 32 m(K+K-) x 32 m(pi+pi-), sgn(sin phi) injection",
}


def workload_specs(name: str, scale: float = 1.0, seed_offset: int = 0):
    """Sample specifications of a named workload (see WORKLOADS).

    scale < 1 shrinks every sample (same shapes, fewer events) for tests.
    """
    def N(x):
        return max(1, int(round(x * scale)))
    if name == "lb_ppipipi_f64_1e5":
        ch = CHANNELS["Lb_ppipipi"]
        return [SampleSpec(ch, N(1e5), 1 + seed_offset, [absphi_axis(10)], dtype=torch.float64)]
    if name == "lb_ppipipi_1e7_phi12":
        ch = CHANNELS["Lb_ppipipi"]
        return [SampleSpec(ch, N(1e7), 2 + seed_offset, [absphi_axis(12)], inj=INJ_SIN)]
    if name == "lb_pkpipi_1e8_phi10xm8":
        ch = CHANNELS["Lb_pKpipi"]
        return [SampleSpec(ch, N(1e8), 3 + seed_offset, [absphi_axis(10), lb_mass03_axis(ch)],
                           frac_m=0.52, inj=INJ_SIN2)]
    if name == "lb_batch64_1e3to1e7":
        rng = np.random.default_rng(4 + seed_offset)
        chans = ["Lb_ppipipi", "Lb_pKpipi", "Lb_ppiKK", "Lb_pKKK"]
        injs = {"Lb_ppipipi": INJ_SIN, "Lb_pKpipi": INJ_SIN2}
        specs = []
        U = rng.uniform(size=64)
        for i in range(64):
            combo = i % 12
            ch = CHANNELS[chans[combo // 3]]
            scheme = combo % 3
            if scheme == 0:
                axes = [absphi_axis(10)]
            elif scheme == 1:
                axes = [absphi_axis(10), lb_mass03_axis(ch)]
            else:
                axes = [abscos_axis(0, 5), absphi_axis(10)]
            n = N(round(10 ** (3 + 4 * U[i])))
            specs.append(SampleSpec(ch, n, 1000 * (4 + seed_offset) + i, axes,
                                    inj=injs.get(ch.name, Injection())))
        return specs
    if name == "d0_kkpipi_5e8_m32x32":
        ch = CHANNELS["D0_KKpipi"]
        return [SampleSpec(ch, N(5e8), 5 + seed_offset,
                           [mass_axis((0, 1), 2 * M_K, M_D0 - 2 * M_PI, 32),
                            mass_axis((2, 3), 2 * M_PI, M_D0 - 2 * M_K, 32)],
                           inj=INJ_SGN)]
    raise ValueError(f"unknown workload {name!r}; known: {sorted(WORKLOADS)}")


def make_sample(spec: SampleSpec, device="cpu", chunk: int = 1 << 22) -> Sample:
    """Generate one spec's sample, in chunks (child seeds) to bound memory."""
    if spec.n <= chunk:
        return generate(spec.channel, spec.n, spec.seed, frac_m=spec.frac_m, inj=spec.inj,
                        dtype=spec.dtype, device=device)
    parts = []
    left, k = spec.n, 0
    while left > 0:
        m = min(chunk, left)
        parts.append(generate(spec.channel, m, spec.seed * 1000003 + k, frac_m=spec.frac_m,
                              inj=spec.inj, dtype=spec.dtype, device=device))
        left -= m
        k += 1
    comps = [[torch.cat([p.comps[s][c] for p in parts]) for c in range(4)] for s in range(4)]
    return Sample(spec.channel, comps, torch.cat([p.tag for p in parts]),
                  torch.cat([p.phi_gen for p in parts]), torch.cat([p.gamma for p in parts]),
                  torch.cat([p.m12 for p in parts]), torch.cat([p.m34 for p in parts]))
