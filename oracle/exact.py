"""Exact rational decisions of the T-odd pass -- TEST INFRASTRUCTURE ONLY.

The stored components are binary floating-point numbers, so each is an exact
rational; every quantity below is a polynomial in them with rational
coefficients and is evaluated exactly with ``fractions.Fraction``.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark may use this
module.

Identities used (each pinned by a test against the textbook rest-frame
formulas of the float64 oracle, not by re-deriving them):

* Sign of C_T (Sect. 5, eq. (4)).  With P = sum of the four momenta and rows
  written as contravariant four-vectors (E, px, py, pz),
      det[P; p_A; p_B; p_C] = M * p*_A . (p*_B x p*_C),
  because in the rest frame P = (M, 0, 0, 0), and a proper Lorentz
  transformation has determinant +1.  M > 0, so the determinant has the sign
  of C_T.
* Rest-frame dot products from invariants: with G_ab = (P.p_a)(P.p_b) - M^2 (p_a.p_b),
  p*_a . p*_b = G_ab / M^2.
* Acoplanarity angle between planes (i,j) and (k,l): with n1 = p*_i x p*_j,
  n2 = p*_k x p*_l,
      X  = G_ik G_jl - G_il G_jk  = M^4 (n1 . n2),
      N1 = G_ii G_jj - G_ij^2     = M^4 |n1|^2,   N2 likewise,
  so cos Phi = X / sqrt(N1 N2).
* Angle of p*_s against the M flight direction:
      Nn = (P.p_s) E_P - M^2 E_s,  A = G_ss,  B = E_P^2 - M^2 = |P_lab|^2,
  |cos theta| = |Nn| / sqrt(A B).
* Invariant mass of a slot set S: m^2 = (sum_{s in S} p_s)^2.
* Rest-frame energy: E*_s = (P.p_s) / M, so of two identical particles the
  faster (larger E*) has the larger P.p_s.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction as F

CLS_I, CLS_II, CLS_III, CLS_IV, CLS_ZERO, CLS_INVALID = 0, 1, 2, 3, 4, 5
ABSPHI, MASS, ABSCOS = 0, 1, 2


def mdot(a, b):
    """Minkowski product, metric (+, -, -, -)."""
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def _perm_sign(perm):
    s = 1
    perm = list(perm)
    for i in range(len(perm)):
        for j in range(i + 1, len(perm)):
            if perm[i] > perm[j]:
                s = -s
    return s


_PERMS4 = [(p, _perm_sign(p)) for p in itertools.permutations(range(4))]


def det4(rows):
    """Leibniz determinant of a 4x4 matrix given as rows."""
    tot = 0
    for p, s in _PERMS4:
        tot += s * rows[0][p[0]] * rows[1][p[1]] * rows[2][p[2]] * rows[3][p[3]]
    return tot


def _sign(x):
    return (x > 0) - (x < 0)


def _sign_sqrt_diff(x, c, r2):
    """sign(x - c * sqrt(r2)) for rationals x, c and r2 >= 0."""
    if x >= 0 and c <= 0:
        return 0 if (x == 0 and (c == 0 or r2 == 0)) else 1
    if x <= 0 and c >= 0:
        return 0 if (x == 0 and (c == 0 or r2 == 0)) else -1
    d = x * x - c * c * r2
    return _sign(d) if x > 0 else -_sign(d)


class ExactEvent:
    """All exact quantities of one event."""

    def __init__(self, comps, tag):
        # comps: 4x4 python floats (exact promotion of the stored values)
        self.valid = all(math.isfinite(v) for row in comps for v in row) and tag in (0, 1)
        self.tag = tag
        self._G = {}
        self._planes = {}
        if not self.valid:
            return
        self.q = [[F(v) for v in row] for row in comps]
        self.P = [sum(self.q[s][c] for s in range(4)) for c in range(4)]
        self.M2 = mdot(self.P, self.P)
        self.valid = self.P[0] > 0 and self.M2 > 0
        if self.valid:
            self.PP = [mdot(self.P, self.q[s]) for s in range(4)]

    def G(self, a, b):
        key = (min(a, b), max(a, b))
        g = self._G.get(key)
        if g is None:
            g = self.PP[a] * self.PP[b] - self.M2 * mdot(self.q[a], self.q[b])
            self._G[key] = g
        return g

    def plane_terms(self, planes):
        """(X, N1 N2) of the acoplanarity angle between planes (i,j) and (k,l)."""
        got = self._planes.get(planes)
        if got is None:
            i, j, k, l = planes
            G = self.G
            X = G(i, k) * G(j, l) - G(i, l) * G(j, k)
            N1 = G(i, i) * G(j, j) - G(i, j) ** 2
            N2 = G(k, k) * G(l, l) - G(k, l) ** 2
            got = (X, N1 * N2)
            self._planes[planes] = got
        return got

    def det_triple(self, triple):
        A, B, C = triple
        return det4([self.P, self.q[A], self.q[B], self.q[C]])

    def cls(self, triple):
        if not self.valid:
            return CLS_INVALID
        s = _sign(self.det_triple(triple))
        if s == 0:
            return CLS_ZERO
        if self.tag == 0:
            return CLS_I if s > 0 else CLS_II
        return CLS_III if -s > 0 else CLS_IV

    # ---- coordinate comparisons: sign(value - edge)
    def cmp_cosphi(self, planes, c):
        X, R2 = self.plane_terms(tuple(planes))
        return _sign_sqrt_diff(X, F(c), R2)

    def cmp_mass(self, mask, e):
        S = [sum(self.q[s][c] for s in range(4) if mask & (1 << s)) for c in range(4)]
        m2 = mdot(S, S)
        return _sign(m2 - F(e) * F(e))

    def cmp_abscos(self, s, e):
        Nn = self.PP[s] * self.P[0] - self.M2 * self.q[s][0]
        A = self.G(s, s)
        B = self.P[0] ** 2 - self.M2
        return _sign(Nn * Nn - F(e) * F(e) * A * B)

    def axis_bin(self, planes, kind, slots, edges):
        """Bin index on one axis or -1 (out of range)."""
        n = len(edges) - 1
        if kind == ABSPHI:
            cmp = [self.cmp_cosphi(planes, c) for c in edges]
            # decreasing cos edges: bin j holds c_{j+1} < cos <= c_j; last bin closed
            if cmp[0] > 0 or cmp[n] < 0:
                return -1
            return sum(1 for k in range(1, n) if cmp[k] <= 0)
        if kind == MASS:
            cmp = [self.cmp_mass(slots, e) for e in edges]
        elif kind == ABSCOS:
            cmp = [self.cmp_abscos(slots, e) for e in edges]
        else:
            raise ValueError(kind)
        if cmp[0] < 0 or cmp[n] > 0:
            return -1
        return sum(1 for k in range(1, n) if cmp[k] >= 0)


def order_identical(comps, identical):
    """comps with the identical particles of slots (f, s) in canonical order:
    the larger rest-frame energy in slot f; an exact tie keeps the stored order.
    Events without a rest frame (or not finite) are returned unchanged."""
    f, s = identical
    if not all(math.isfinite(v) for row in comps for v in row):
        return comps
    q = [[F(v) for v in row] for row in comps]
    P = [sum(q[k][c] for k in range(4)) for c in range(4)]
    if not (P[0] > 0 and mdot(P, P) > 0):
        return comps
    if mdot(P, q[s]) > mdot(P, q[f]):
        comps = [list(row) for row in comps]
        comps[f], comps[s] = comps[s], comps[f]
    return comps


def exact_decision(comps, tag, triple, planes, axes, identical=None):
    """(class, combined bin or -1 out of range or None if not binned) of one event.

    axes: list of (kind, slots, edges); identical: None or (fast slot, slow slot).
    """
    if identical is not None:
        comps = order_identical(comps, identical)
    ev = ExactEvent(comps, tag)
    c = ev.cls(triple)
    if c >= CLS_ZERO or not axes:
        return c, None
    b = 0
    for kind, slots, edges in axes:
        j = ev.axis_bin(planes, kind, slots, edges)
        if j < 0:
            return c, -1
        b = b * (len(edges) - 1) + j
    return c, b


def accumulate(counts, stats, cls, b):
    """Add one decided event to counts (list of [4] rows) and stats [events, zero, invalid, oor]."""
    stats[0] += 1
    if cls == CLS_ZERO:
        stats[1] += 1
        return
    if cls == CLS_INVALID:
        stats[2] += 1
        return
    counts[0][cls] += 1
    if b is None:
        return
    if b < 0:
        stats[3] += 1
        return
    counts[1 + b][cls] += 1


# ------------------------------------------------------------------ asymmetries
def _ratio(num, den):
    return F(num, den) if den != 0 else None


def asym_row(n):
    """Exact asymmetries of one row of counts n = (N_I, N_II, N_III, N_IV).

    A_T = (N_I - N_II)/(N_I + N_II), Abar_T = (N_III - N_IV)/(N_III + N_IV),
    a_CP = (A_T - Abar_T)/2, a_P = (A_T + Abar_T)/2 (the usual T-odd quantities);
    eq. (5): A_CP(C_T>0) = (N_I - N_III)/(N_I + N_III),
             A_CP(C_T<0) = (N_II - N_IV)/(N_II + N_IV);
    eq. (6): A_CP^{P-even} = (A+ + A-)/2, A_CP^{P-odd} = (A+ - A-)/2.
    Binomial sigma of a two-count asymmetry over n events: sqrt((1 - A^2)/n);
    half-sums and half-differences of asymmetries of disjoint samples add the
    two sigmas in quadrature and halve.  A ratio with a zero denominator is None.
    Returns dict name -> (Fraction or None, float sigma or nan).
    """
    n1, n2, n3, n4 = (int(x) for x in n)

    def two(a, b):
        A = _ratio(a - b, a + b)
        if A is None:
            return None, math.nan
        return A, math.sqrt(max(0.0, float(1 - A * A)) / (a + b))

    AT, sAT = two(n1, n2)
    AbT, sAbT = two(n3, n4)
    Ap, sAp = two(n1, n3)
    Am, sAm = two(n2, n4)

    def half(a, sa, b, sb, sgn):
        if a is None or b is None:
            return None, math.nan
        return (a + sgn * b) / 2, 0.5 * math.sqrt(sa * sa + sb * sb)

    acp, sacp = half(AT, sAT, AbT, sAbT, -1)
    ap, sap = half(AT, sAT, AbT, sAbT, +1)
    ev, sev = half(Ap, sAp, Am, sAm, +1)
    od, sod = half(Ap, sAp, Am, sAm, -1)
    return {"A_T": (AT, sAT), "Abar_T": (AbT, sAbT), "a_CP": (acp, sacp), "a_P": (ap, sap),
            "A_plus": (Ap, sAp), "A_minus": (Am, sAm), "A_even": (ev, sev), "A_odd": (od, sod)}


def chi2_sf(x, k):
    """Survival function of the chi-square distribution, k degrees of freedom (scipy)."""
    from scipy.special import gammaincc
    if k <= 0:
        return math.nan
    return float(gammaincc(0.5 * k, 0.5 * x))


def scp(nx, nxbar):
    """Binned S_CP (eq. (1)) per bin and its chi^2, ndf = bins - 1, p-value.

    nx, nxbar: per-bin yields of the two compared samples.  alpha = N_tot(X)/N_tot(Xbar).
    S^i = (N^i(X) - alpha N^i(Xbar)) / sqrt(N^i(X) + alpha^2 N^i(Xbar)); empty bins give 0.
    """
    tx, txb = sum(nx), sum(nxbar)
    alpha = F(tx, txb) if txb else None
    s = []
    for a, b in zip(nx, nxbar):
        if alpha is None or (a + alpha * alpha * b) == 0:
            s.append(0.0)
            continue
        s.append(float(a - alpha * b) / math.sqrt(float(a + alpha * alpha * b)))
    chi2 = sum(v * v for v in s)
    ndf = len(s) - 1
    return s, chi2, ndf, chi2_sf(chi2, ndf)
