// Double-word tier of the T-odd pass: the same invariant quantities as the
// float64 tier, evaluated in double-word ("double-double", ~106-bit)
// arithmetic with a running absolute error bound on every intermediate.  It
// decides, in microseconds, the rare events whose float64 bounds were too
// wide (near-degenerate planes, near-edge values, extreme boosts); only what
// it cannot certify either goes on to exact integer arithmetic (tp_exact.h).
//
// Building blocks (Joldes, Muller & Popescu, "Tight and rigorous error bounds
// for basic building blocks of double-word arithmetic", ACM TOMS 44 (2017)):
//   2Sum, Fast2Sum, 2Prod (with FMA): exact error-free transformations;
//   AccurateDWPlusDW: relative error <= 3u^2/(1-4u);
//   DWTimesDW with FMA: relative error <= 5u^2.
// Every operation below is charged ETA = 2^-100 (> 64 u^2) relative error,
// plus the propagated input errors; bounds are formed in float64 and inflated
// by (1 + 2^-50) per step to cover their own rounding.  Valid while no
// intermediate underflows or overflows, which the entry check guarantees by
// admitting only events whose nonzero components lie in [2^-30, 2^40].
//
// Comparisons against bin edges use squared forms, so no square root is taken:
//   cos Phi <= c  from the signs of X, c and F = X^2 - c^2 N1 N2;
//   |cos theta| >= e  iff  Nn^2 - e^2 A B >= 0;   m >= e  iff  m^2 - e^2 >= 0.
//
// Requires -ffp-contract=off (the error-free transformations must not be fused).
#pragma once

#include <stdint.h>

#ifndef TP_HD
#define TP_HD
#endif

namespace tpw {

constexpr double ETA = 0x1p-100;
constexpr double INFL = 1.0 + 0x1p-50;

struct dw {
    double hi, lo;
};

TP_HD inline double aabs(double x) { return x < 0 ? -x : x; }

TP_HD inline dw two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return { s, e };
}

TP_HD inline dw fast_two_sum(double a, double b)
{
    const double s = a + b;
    const double e = b - (s - a);
    return { s, e };
}

TP_HD inline dw two_prod(double a, double b)
{
    const double p = a * b;
    const double e = __builtin_fma(a, b, -p);
    return { p, e };
}

TP_HD inline dw dw_add(dw x, dw y)
{
    const dw s = two_sum(x.hi, y.hi);
    const dw t = two_sum(x.lo, y.lo);
    const double c = s.lo + t.hi;
    const dw v = fast_two_sum(s.hi, c);
    const double w = t.lo + v.lo;
    return fast_two_sum(v.hi, w);
}

TP_HD inline dw dw_mul(dw x, dw y)
{
    const dw c = two_prod(x.hi, y.hi);
    const double tl0 = x.lo * y.lo;
    const double tl1 = __builtin_fma(x.hi, y.lo, tl0);
    const double cl2 = __builtin_fma(x.lo, y.hi, tl1);
    const double cl3 = c.lo + cl2;
    return fast_two_sum(c.hi, cl3);
}

// A double-word value with a bound on its distance to the exact quantity.
struct V {
    dw v;
    double e;
};

TP_HD inline double mag(const V &a) { return aabs(a.v.hi) * INFL + aabs(a.v.lo); }

TP_HD inline V exact(double x) { return { { x, 0.0 }, 0.0 }; }

TP_HD inline V add(const V &a, const V &b)
{
    V r;
    r.v = dw_add(a.v, b.v);
    r.e = ((a.e + b.e) + ETA * mag(r)) * INFL;
    return r;
}

TP_HD inline V neg(const V &a) { return { { -a.v.hi, -a.v.lo }, a.e }; }

TP_HD inline V sub(const V &a, const V &b) { return add(a, neg(b)); }

TP_HD inline V mul(const V &a, const V &b)
{
    V r;
    r.v = dw_mul(a.v, b.v);
    r.e = (((mag(a) + a.e) * b.e + mag(b) * a.e) + ETA * mag(r)) * INFL;
    return r;
}

// product of two stored values: exact as a double word
TP_HD inline V prod(double a, double b)
{
    V r;
    r.v = two_prod(a, b);
    r.e = 0.0;
    return r;
}

// certified sign: +1 / -1, or 0 when the bound does not decide
TP_HD inline int csign(const V &a)
{
    const double lo = aabs(a.v.hi) * (1.0 - 0x1p-50) - aabs(a.v.lo);
    if (!(lo > a.e * INFL)) return 0;
    return a.v.hi > 0 ? 1 : -1;
}

TP_HD inline V mink(const double a[4], const double b[4])
{
    V r = prod(a[0], b[0]);
    r = sub(r, prod(a[1], b[1]));
    r = sub(r, prod(a[2], b[2]));
    r = sub(r, prod(a[3], b[3]));
    return r;
}

enum { W_I = 0, W_II = 1, W_III = 2, W_IV = 3, W_ZERO = 4, W_INVALID = 5, W_UNRESOLVED = 6, W_UNCERTAIN = 7 };
enum { W_ABSPHI = 0, W_MASS = 1, W_ABSCOS = 2 };

// cos Phi <= c given the signs of X and of F = X^2 - c^2 D (D >= 0):
// 1 true, 0 false, -1 undecided
TP_HD inline int cos_le(int sX, int sF, double c)
{
    if (c > 0) {
        if (sX < 0 || sF < 0) return 1;
        if (sX > 0 && sF > 0) return 0;
        return -1;
    }
    if (c == 0) return sX < 0 ? 1 : (sX > 0 ? 0 : -1);
    if (sX < 0 && sF > 0) return 1;
    if (sX > 0 || sF < 0) return 0;
    return -1;
}

// Decide one event (components x in kernel slot order, float values exactly in
// double).  Same conventions as tpx::decide; returns W_UNCERTAIN when some
// decision is not certified here.
TP_HD inline int decide_dw(const double x[4][4], int tag, int sigma, int naxes, const int32_t kind[2],
                           const int32_t nbins[2], const int32_t slots[2], const double *const edges[2], int &bin)
{
    bin = -1;
    if (tag != 0 && tag != 1) return W_INVALID;
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 4; ++c) {
            const double a = aabs(x[s][c]);
            if (!(a == 0.0 || (a >= 0x1p-30 && a <= 0x1p40))) return W_UNCERTAIN;
        }
    V P[4];
    for (int c = 0; c < 4; ++c) {
        V t = add(exact(x[0][c]), exact(x[1][c]));
        t = add(t, exact(x[2][c]));
        P[c] = add(t, exact(x[3][c]));
    }
    V M2 = mul(P[0], P[0]);
    for (int c = 1; c < 4; ++c) M2 = sub(M2, mul(P[c], P[c]));
    const int sE = csign(P[0]), sM = csign(M2);
    if (sE < 0 || sM < 0) return W_INVALID;
    if (sE == 0 || sM == 0) return W_UNCERTAIN;

    // det[x0; x1; x2; x3] by Laplace on row pairs (0,1) | (2,3)
    const int pa[6] = { 0, 0, 0, 1, 1, 2 }, pb[6] = { 1, 2, 3, 2, 3, 3 };
    const int sg[6] = { 1, -1, 1, 1, -1, 1 };
    V det = exact(0.0);
    for (int k = 0; k < 6; ++k) {
        const int a = pa[k], b = pb[k], c = pa[5 - k], d = pb[5 - k];
        const V top = sub(prod(x[0][a], x[1][b]), prod(x[0][b], x[1][a]));
        const V bot = sub(prod(x[2][c], x[3][d]), prod(x[2][d], x[3][c]));
        const V t = mul(top, bot);
        det = sg[k] > 0 ? add(det, t) : sub(det, t);
    }
    const int sd = csign(det) * sigma;
    if (sd == 0) return W_UNCERTAIN;
    const int cls = tag == 0 ? (sd > 0 ? W_I : W_II) : (sd < 0 ? W_III : W_IV);
    if (naxes <= 0) return cls;

    V d[4][4], PP[4];
    for (int a = 0; a < 4; ++a)
        for (int b = a; b < 4; ++b) {
            d[a][b] = mink(x[a], x[b]);
            d[b][a] = d[a][b];
        }
    for (int a = 0; a < 4; ++a) PP[a] = add(add(d[a][0], d[a][1]), add(d[a][2], d[a][3]));
    auto G = [&](int a, int b) { return sub(mul(PP[a], PP[b]), mul(M2, d[a][b])); };

    int bsum = 0;
    bool oor = false;
    for (int ax = 0; ax < naxes; ++ax) {
        const int nb = nbins[ax];
        const double *e = edges[ax];
        int j = 0;
        if (kind[ax] == W_ABSPHI) {
            const V X = sub(mul(G(0, 2), G(1, 3)), mul(G(0, 3), G(1, 2)));
            const V G01 = G(0, 1), G23 = G(2, 3);
            const V N1 = sub(mul(G(0, 0), G(1, 1)), mul(G01, G01));
            const V N2 = sub(mul(G(2, 2), G(3, 3)), mul(G23, G23));
            const V D = mul(N1, N2);
            const V X2 = mul(X, X);
            const int sX = csign(X);
            for (int k = 1; k < nb; ++k) {
                const V F = sub(X2, mul(prod(e[k], e[k]), D));
                const int le = cos_le(sX, csign(F), e[k]);
                if (le < 0) return W_UNCERTAIN;
                j += le;
            }
        } else if (kind[ax] == W_ABSCOS) {
            const int s = slots[ax];
            const V Nn = sub(mul(PP[s], P[0]), mul(M2, exact(x[s][0])));
            const V A = G(s, s);
            const V B = sub(mul(P[0], P[0]), M2);
            const V AB = mul(A, B);
            const V Nn2 = mul(Nn, Nn);
            for (int k = 1; k < nb; ++k) {
                const int sF = csign(sub(Nn2, mul(prod(e[k], e[k]), AB)));
                if (sF == 0) return W_UNCERTAIN;
                j += sF > 0 ? 1 : 0;
            }
        } else {
            const int mask = slots[ax];
            V S[4];
            for (int c = 0; c < 4; ++c) {
                S[c] = exact(0.0);
                for (int t = 0; t < 4; ++t)
                    if (mask & (1 << t)) S[c] = add(S[c], exact(x[t][c]));
            }
            V m2 = mul(S[0], S[0]);
            for (int c = 1; c < 4; ++c) m2 = sub(m2, mul(S[c], S[c]));
            int cnt = 0, s0 = 0, sn = 0;
            for (int k = 0; k <= nb; ++k) {
                const int sF = csign(sub(m2, prod(e[k], e[k])));
                if (sF == 0) return W_UNCERTAIN;
                if (k == 0) s0 = sF;
                if (k == nb) sn = sF;
                if (k > 0 && k < nb && sF > 0) ++cnt;
            }
            j = (s0 < 0 || sn > 0) ? -1 : cnt;
        }
        if (j < 0) oor = true;
        bsum = bsum * nb + (j < 0 ? 0 : j);
    }
    bin = oor ? -1 : bsum;
    return cls;
}

}  // namespace tpw
