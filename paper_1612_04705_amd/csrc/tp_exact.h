// Exact tier of the T-odd pass: every decision evaluated in exact integer
// arithmetic on the stored components.
//
// Each stored component is a binary float x = m * 2^e (|m| < 2^53).  All the
// polynomials involved are homogeneous in the sixteen components, so the event
// is rescaled by 2^-emin (emin = smallest exponent among nonzero components),
// which makes every component an integer without changing any sign.  With the
// event's exponent span limited (float64 storage: 107, float32: 136) every
// scaled component is below 2^160 and the highest-degree quantity used
// (degree 16, the plane-angle comparison) fits in 88 limbs of 32 bits.
//
// Quantities (P = sum of the momenta, Minkowski metric (+,-,-,-)):
//   sign:       det[p0; p1; p2; p3] by Laplace expansion on row pairs
//   G_ab      = (P.p_a)(P.p_b) - M^2 (p_a.p_b)     (M^2 rest-frame dot products)
//   plane angle between (i,j) and (k,l):  X = G_ik G_jl - G_il G_jk,
//               R2 = (G_ii G_jj - G_ij^2)(G_kk G_ll - G_kl^2),  cos Phi = X / sqrt(R2)
//   helicity-type angle of slot s: Nn = (P.p_s) E_P - M^2 E_s, A = G_ss,
//               B = E_P^2 - M^2, |cos theta| = |Nn| / sqrt(A B)
//   mass of a slot set S: m^2 = (sum_{s in S} p_s)^2
// A comparison against an edge value y (a double) is the sign of a polynomial
// difference, e.g. sign(X - c sqrt(R2)) from the signs of X, c and X^2 - c^2 R2.
//
// This header is plain C++; TP_HD marks functions for both host and device so
// the arithmetic can also be unit-tested on the CPU.
#pragma once

#include <stdint.h>

#ifndef TP_HD
#define TP_HD
#endif

namespace tpx {

// ------------------------------------------------------------- sign-magnitude
template <int N>
struct Big {
    uint32_t w[N];   // magnitude, little-endian limbs
    int len;         // limbs in use (w[len..] are zero)
    int neg;         // 1 if negative (never set for zero)
};

template <int N>
TP_HD inline void big_zero(Big<N> &a)
{
    for (int i = 0; i < N; ++i) a.w[i] = 0;
    a.len = 0;
    a.neg = 0;
}

template <int N>
TP_HD inline void big_norm(Big<N> &a)
{
    while (a.len > 0 && a.w[a.len - 1] == 0) --a.len;
    if (a.len == 0) a.neg = 0;
}

template <int N>
TP_HD inline int big_sign(const Big<N> &a)
{
    return a.len == 0 ? 0 : (a.neg ? -1 : 1);
}

// |a| <=> |b|
template <int NA, int NB>
TP_HD inline int mag_cmp(const Big<NA> &a, const Big<NB> &b)
{
    if (a.len != b.len) return a.len < b.len ? -1 : 1;
    for (int i = a.len - 1; i >= 0; --i)
        if (a.w[i] != b.w[i]) return a.w[i] < b.w[i] ? -1 : 1;
    return 0;
}

// r = |a| + |b| (magnitudes), r must not alias
template <int NR, int NA, int NB>
TP_HD inline bool mag_add(Big<NR> &r, const Big<NA> &a, const Big<NB> &b)
{
    const int n = a.len > b.len ? a.len : b.len;
    uint64_t carry = 0;
    int i = 0;
    for (; i < n; ++i) {
        uint64_t s = carry;
        if (i < a.len) s += a.w[i];
        if (i < b.len) s += b.w[i];
        if (i >= NR) return false;
        r.w[i] = (uint32_t)s;
        carry = s >> 32;
    }
    r.len = n;
    if (carry) {
        if (n >= NR) return false;
        r.w[n] = (uint32_t)carry;
        r.len = n + 1;
    }
    for (int k = r.len; k < NR; ++k) r.w[k] = 0;
    return true;
}

// r = |a| - |b| with |a| >= |b|
template <int NR, int NA, int NB>
TP_HD inline bool mag_sub(Big<NR> &r, const Big<NA> &a, const Big<NB> &b)
{
    int64_t borrow = 0;
    if (a.len > NR) return false;
    for (int i = 0; i < a.len; ++i) {
        int64_t d = (int64_t)a.w[i] - borrow - (i < b.len ? (int64_t)b.w[i] : 0);
        borrow = d < 0 ? 1 : 0;
        r.w[i] = (uint32_t)(d + (borrow << 32));
    }
    for (int k = a.len; k < NR; ++k) r.w[k] = 0;
    r.len = a.len;
    big_norm(r);
    return true;
}

// r = a + sb * b, sb = +1 or -1 (r must not alias a or b)
template <int NR, int NA, int NB>
TP_HD inline bool big_addsub(Big<NR> &r, const Big<NA> &a, const Big<NB> &b, int sb)
{
    const int an = a.neg, bn = (b.len == 0) ? 0 : (b.neg ^ (sb < 0 ? 1 : 0));
    bool ok;
    if (an == bn) {
        ok = mag_add(r, a, b);
        r.neg = an;
    } else if (mag_cmp(a, b) >= 0) {
        ok = mag_sub(r, a, b);
        r.neg = an;
    } else {
        ok = mag_sub(r, b, a);
        r.neg = bn;
    }
    big_norm(r);
    return ok;
}

// r = a * b
template <int NR, int NA, int NB>
TP_HD inline bool big_mul(Big<NR> &r, const Big<NA> &a, const Big<NB> &b)
{
    for (int k = 0; k < NR; ++k) r.w[k] = 0;
    r.len = 0;
    r.neg = 0;
    if (a.len == 0 || b.len == 0) return true;
    if (a.len + b.len > NR) return false;
    for (int i = 0; i < a.len; ++i) {
        uint64_t carry = 0;
        const uint64_t ai = a.w[i];
        for (int j = 0; j < b.len; ++j) {
            uint64_t t = ai * b.w[j] + r.w[i + j] + carry;
            r.w[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        int k = i + b.len;
        while (carry) {
            uint64_t t = (uint64_t)r.w[k] + carry;
            r.w[k] = (uint32_t)t;
            carry = t >> 32;
            ++k;
        }
    }
    r.len = a.len + b.len;
    r.neg = a.neg ^ b.neg;
    big_norm(r);
    return true;
}

template <int NR, int NA>
TP_HD inline void big_copy(Big<NR> &r, const Big<NA> &a)
{
    for (int k = 0; k < NR; ++k) r.w[k] = k < a.len ? a.w[k] : 0;
    r.len = a.len;
    r.neg = a.neg;
}

// a * 2^s (s >= 0) into r
template <int NR, int NA>
TP_HD inline bool big_shl(Big<NR> &r, const Big<NA> &a, int s)
{
    for (int k = 0; k < NR; ++k) r.w[k] = 0;
    r.len = 0;
    r.neg = 0;
    if (a.len == 0) return true;
    const int q = s >> 5, b = s & 31;
    if (a.len + q + 1 > NR) return false;
    for (int i = 0; i < a.len; ++i) {
        uint64_t v = (uint64_t)a.w[i] << b;
        r.w[i + q] |= (uint32_t)v;
        r.w[i + q + 1] |= (uint32_t)(v >> 32);
    }
    r.len = a.len + q + 1;
    r.neg = a.neg;
    big_norm(r);
    return true;
}

template <int N>
TP_HD inline int big_bitlen(const Big<N> &a)
{
    if (a.len == 0) return 0;
    uint32_t top = a.w[a.len - 1];
    int b = 0;
    while (top) { ++b; top >>= 1; }
    return (a.len - 1) * 32 + b;
}

// sign(a * 2^sa - b * 2^sb) for non-negative a, b (sa, sb may be negative:
// the common power is factored out).  ok = false on capacity overflow.
template <int NA, int NB>
TP_HD inline int cmp_scaled(const Big<NA> &a, int sa, const Big<NB> &b, int sb, bool &ok)
{
    if (a.len == 0 && b.len == 0) return 0;
    if (a.len == 0) return -1;
    if (b.len == 0) return 1;
    const int la = big_bitlen(a) + sa, lb = big_bitlen(b) + sb;
    if (la > lb + 1) return 1;
    if (lb > la + 1) return -1;
    const int m = sa < sb ? sa : sb;
    Big<NA + 8> x;
    Big<NB + 8> y;
    ok = ok && big_shl(x, a, sa - m) && big_shl(y, b, sb - m);
    x.neg = 0;
    y.neg = 0;
    return mag_cmp(x, y);
}

// sign(x - y * sqrt(r2)) as cmp_sqrt, with x2 = x^2 precomputed.
template <int NX, int NX2, int NR>
TP_HD inline int cmp_sqrt_x2(const Big<NX> &x, const Big<NX2> &x2, const Big<NR> &r2, double y, bool &ok);

// ------------------------------------------------------------- float decoding
// x = mant * 2^exp exactly, mant an integer with |mant| < 2^53 (0 for zero)
TP_HD inline void decode_f64(double x, int64_t &mant, int &exp)
{
    union { double d; uint64_t u; } v;
    v.d = x;
    const uint64_t u = v.u;
    const int e = (int)((u >> 52) & 0x7ff);
    uint64_t m = u & ((1ull << 52) - 1);
    if (e == 0) {
        exp = -1074;
    } else {
        m |= 1ull << 52;
        exp = e - 1075;
    }
    mant = (u >> 63) ? -(int64_t)m : (int64_t)m;
    if (m == 0) exp = 0;
}

TP_HD inline void decode_f32(float x, int64_t &mant, int &exp)
{
    union { float f; uint32_t u; } v;
    v.f = x;
    const uint32_t u = v.u;
    const int e = (int)((u >> 23) & 0xff);
    uint32_t m = u & ((1u << 23) - 1);
    if (e == 0) {
        exp = -149;
    } else {
        m |= 1u << 23;
        exp = e - 150;
    }
    mant = (u >> 31) ? -(int64_t)m : (int64_t)m;
    if (m == 0) exp = 0;
}

template <int N>
TP_HD inline bool big_from_mant(Big<N> &r, int64_t mant, int shift)
{
    Big<3> t;
    big_zero(t);
    uint64_t m = mant < 0 ? (uint64_t)(-mant) : (uint64_t)mant;
    t.w[0] = (uint32_t)m;
    t.w[1] = (uint32_t)(m >> 32);
    t.len = 2;
    t.neg = mant < 0;
    big_norm(t);
    return big_shl(r, t, shift);
}

// ------------------------------------------------------------- event quantities
constexpr int L1 = 6;     // scaled components and their sums  (< 2^162)
constexpr int L2 = 12;    // dot products, M^2                  (< 2^326)
constexpr int L4 = 22;    // G_ab, determinant                  (< 2^651)
constexpr int L8 = 44;    // X, N1, N2, Nn^2 ...                (< 2^1301)
constexpr int L16 = 88;   // X^2, R2 = N1 N2                    (< 2^2600)

struct Event {
    Big<L1> q[4][4];   // scaled components (kernel slot order)
    Big<L1> P[4];
    Big<L2> M2;
    Big<L2> PP[4];     // P . p_s
    int shift;         // components were multiplied by 2^shift (shift = -emin)
    bool ok;           // arithmetic stayed within capacity
};

template <int NR, int NA, int NB>
TP_HD inline bool mdot(Big<NR> &r, const Big<NA> a[4], const Big<NB> b[4])
{
    Big<NR> t0, t1, acc;
    bool ok = big_mul(acc, a[0], b[0]);
    for (int c = 1; c < 4; ++c) {
        ok = ok && big_mul(t0, a[c], b[c]);
        ok = ok && big_addsub(t1, acc, t0, -1);
        big_copy(acc, t1);
    }
    big_copy(r, acc);
    return ok;
}

// Build the scaled integer event from 16 decoded components (mant[s][c], ex[s][c]).
// Returns false if the exponent span exceeds ``maxspan``.
TP_HD inline bool event_build(Event &ev, const int64_t mant[4][4], const int ex[4][4], int maxspan)
{
    int emin = 100000, emax = -100000;
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 4; ++c)
            if (mant[s][c] != 0) {
                if (ex[s][c] < emin) emin = ex[s][c];
                if (ex[s][c] > emax) emax = ex[s][c];
            }
    if (emin > emax) emin = emax = 0;
    if (emax - emin > maxspan) return false;
    ev.shift = -emin;
    ev.ok = true;
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 4; ++c) {
            if (mant[s][c] == 0) big_zero(ev.q[s][c]);
            else ev.ok = ev.ok && big_from_mant(ev.q[s][c], mant[s][c], ex[s][c] - emin);
        }
    for (int c = 0; c < 4; ++c) {
        Big<L1> t;
        big_copy(ev.P[c], ev.q[0][c]);
        for (int s = 1; s < 4; ++s) {
            ev.ok = ev.ok && big_addsub(t, ev.P[c], ev.q[s][c], 1);
            big_copy(ev.P[c], t);
        }
    }
    ev.ok = ev.ok && mdot(ev.M2, ev.P, ev.P);
    for (int s = 0; s < 4; ++s) ev.ok = ev.ok && mdot(ev.PP[s], ev.P, ev.q[s]);
    return true;
}

// Exact sign of P.p_a - P.p_b (the rest-frame energy order of slots a and b,
// M E*_s = P.p_s), or 2 if the event exceeds the arithmetic's capacity.
TP_HD inline int order_sign(const int64_t mant[4][4], const int ex[4][4], int span, int a, int b)
{
    Event ev;
    if (!event_build(ev, mant, ex, span)) return 2;
    Big<L2> d;
    ev.ok = ev.ok && big_addsub(d, ev.PP[a], ev.PP[b], -1);
    return ev.ok ? big_sign(d) : 2;
}

// Exact sign of m^2(a, b) - m^2(c, d), m^2(x, y) = (p_x + p_y)^2, or 2 if the
// event exceeds the arithmetic's capacity.
TP_HD inline int pair_mass2_cmp(const int64_t mant[4][4], const int ex[4][4], int span, int a, int b, int c, int d)
{
    Event ev;
    if (!event_build(ev, mant, ex, span)) return 2;
    Big<L1> S1[4], S2[4];
    for (int k = 0; k < 4; ++k) {
        ev.ok = ev.ok && big_addsub(S1[k], ev.q[a][k], ev.q[b][k], 1);
        ev.ok = ev.ok && big_addsub(S2[k], ev.q[c][k], ev.q[d][k], 1);
    }
    Big<L2> m1, m2, diff;
    ev.ok = ev.ok && mdot(m1, S1, S1) && mdot(m2, S2, S2) && big_addsub(diff, m1, m2, -1);
    return ev.ok ? big_sign(diff) : 2;
}

// E_P > 0 and M^2 > 0
TP_HD inline bool event_timelike(const Event &ev)
{
    return big_sign(ev.P[0]) > 0 && big_sign(ev.M2) > 0;
}

// det[q0; q1; q2; q3] (Laplace on row pairs (0,1) | (2,3))
TP_HD inline int event_det_sign(Event &ev)
{
    static const int pa[6] = { 0, 0, 0, 1, 1, 2 }, pb[6] = { 1, 2, 3, 2, 3, 3 };
    static const int sg[6] = { 1, -1, 1, 1, -1, 1 };
    Big<L4> acc, t, u;
    big_zero(acc);
    for (int k = 0; k < 6; ++k) {
        const int a = pa[k], b = pb[k], c = pa[5 - k], d = pb[5 - k];
        Big<L2> x1, x2, top, bot;
        ev.ok = ev.ok && big_mul(x1, ev.q[0][a], ev.q[1][b]);
        ev.ok = ev.ok && big_mul(x2, ev.q[0][b], ev.q[1][a]);
        ev.ok = ev.ok && big_addsub(top, x1, x2, -1);
        ev.ok = ev.ok && big_mul(x1, ev.q[2][c], ev.q[3][d]);
        ev.ok = ev.ok && big_mul(x2, ev.q[2][d], ev.q[3][c]);
        ev.ok = ev.ok && big_addsub(bot, x1, x2, -1);
        ev.ok = ev.ok && big_mul(t, top, bot);
        ev.ok = ev.ok && big_addsub(u, acc, t, sg[k]);
        big_copy(acc, u);
    }
    return big_sign(acc);
}

TP_HD inline bool event_G(Event &ev, int a, int b, Big<L4> &g)
{
    Big<L2> d;
    Big<L4> t1, t2;
    bool ok = mdot(d, ev.q[a], ev.q[b]);
    ok = ok && big_mul(t1, ev.PP[a], ev.PP[b]);
    ok = ok && big_mul(t2, ev.M2, d);
    ok = ok && big_addsub(g, t1, t2, -1);
    return ok;
}

// sign(x - y * sqrt(r2)) for an integer x, an integer r2 >= 0 and a double
// y = ym * 2^ye.  x and sqrt(r2) are homogeneous of the same degree in the
// components, so the event's scale cancels; y enters as y^2 = ym^2 * 2^(2 ye).
template <int NX, int NR>
TP_HD inline int cmp_sqrt(const Big<NX> &x, const Big<NR> &r2, double y, bool &ok)
{
    int64_t ym;
    int ye;
    decode_f64(y, ym, ye);
    const int sx = big_sign(x);
    const int sy = ym > 0 ? 1 : (ym < 0 ? -1 : 0);
    const int sr = big_sign(r2);
    if (sx >= 0 && (sy <= 0 || sr == 0)) return (sx == 0 && (sy == 0 || sr == 0)) ? 0 : 1;
    if (sx <= 0 && (sy >= 0 || sr == 0)) return (sx == 0 && (sy == 0 || sr == 0)) ? 0 : -1;
    // same strict sign: compare x^2 with y^2 r2
    Big<2 * NX> x2;
    ok = ok && big_mul(x2, x, x);
    return cmp_sqrt_x2(x, x2, r2, y, ok);
}

template <int NX, int NX2, int NR>
TP_HD inline int cmp_sqrt_x2(const Big<NX> &x, const Big<NX2> &x2in, const Big<NR> &r2, double y, bool &ok)
{
    int64_t ym;
    int ye;
    decode_f64(y, ym, ye);
    const int sx = big_sign(x);
    const int sy = ym > 0 ? 1 : (ym < 0 ? -1 : 0);
    const int sr = big_sign(r2);
    if (sx >= 0 && (sy <= 0 || sr == 0)) return (sx == 0 && (sy == 0 || sr == 0)) ? 0 : 1;
    if (sx <= 0 && (sy >= 0 || sr == 0)) return (sx == 0 && (sy == 0 || sr == 0)) ? 0 : -1;
    Big<NX2> x2;
    big_copy(x2, x2in);
    const uint64_t am = ym < 0 ? (uint64_t)(-ym) : (uint64_t)ym;
    // am^2 < 2^106: compute as 128-bit
    const uint64_t lo32 = am & 0xffffffffu, hi32 = am >> 32;
    const uint64_t ll = lo32 * lo32, lh = lo32 * hi32, hh = hi32 * hi32;
    uint64_t w0 = ll & 0xffffffffu;
    uint64_t mid = (ll >> 32) + 2 * (lh & 0xffffffffu);
    uint64_t w1 = mid & 0xffffffffu;
    uint64_t top = (mid >> 32) + 2 * (lh >> 32) + hh;
    Big<4> y2;
    big_zero(y2);
    y2.w[0] = (uint32_t)w0;
    y2.w[1] = (uint32_t)w1;
    y2.w[2] = (uint32_t)top;
    y2.w[3] = (uint32_t)(top >> 32);
    y2.len = 4;
    big_norm(y2);
    Big<NR + 4> yr;
    ok = ok && big_mul(yr, y2, r2);
    yr.neg = 0;
    x2.neg = 0;
    const int c = cmp_scaled(x2, 0, yr, 2 * ye, ok);   // sign(x^2 - y^2 r2)
    return sx > 0 ? c : -c;
}

// ------------------------------------------------------------- whole event
enum { X_I = 0, X_II = 1, X_III = 2, X_IV = 3, X_ZERO = 4, X_INVALID = 5, X_UNRESOLVED = 6 };
enum { X_ABSPHI = 0, X_MASS = 1, X_ABSCOS = 2 };

// Decide one event exactly.
//   mant/ex: decoded components in kernel slot order (kernel planes (0,1) | (2,3));
//   finite: every component finite; span: largest allowed exponent span;
//   sigma: C_T^inv = sigma * det[p0; p1; p2; p3];
//   axes: kind, nbins, slots (MASS: kernel-order bit mask; ABSCOS: kernel slot),
//   edges[a]: the nbins + 1 edge values (ABSPHI: decreasing cosines).
// Returns the class; *bin = combined bin or -1 (out of range / not binned).
TP_HD inline int decide(const int64_t mant[4][4], const int ex[4][4], bool finite, int tag, int span,
                        int sigma, int naxes, const int32_t kind[2], const int32_t nbins[2],
                        const int32_t slots[2], const double *const edges[2], int &bin)
{
    bin = -1;
    if (!finite || (tag != 0 && tag != 1)) return X_INVALID;
    Event ev;
    if (!event_build(ev, mant, ex, span)) return X_UNRESOLVED;
    if (!event_timelike(ev)) return ev.ok ? X_INVALID : X_UNRESOLVED;
    const int sd = event_det_sign(ev) * sigma;
    int cls;
    if (sd == 0) cls = X_ZERO;
    else cls = tag == 0 ? (sd > 0 ? X_I : X_II) : (sd < 0 ? X_III : X_IV);
    if (cls < 4 && naxes > 0) {
        int b = 0;
        bool oor = false;
        for (int a = 0; a < naxes; ++a) {
            const int nb = nbins[a];
            const double *ed = edges[a];
            int j = 0;
            if (kind[a] == X_ABSPHI) {
                // cos Phi <= c_k  <=>  sign(X - c_k sqrt(R2)) <= 0
                Big<L4> G00, G11, G01, G22, G33, G23, G02, G13, G03, G12;
                ev.ok = ev.ok && event_G(ev, 0, 0, G00) && event_G(ev, 1, 1, G11) &&
                        event_G(ev, 0, 1, G01) && event_G(ev, 2, 2, G22) && event_G(ev, 3, 3, G33) &&
                        event_G(ev, 2, 3, G23) && event_G(ev, 0, 2, G02) && event_G(ev, 1, 3, G13) &&
                        event_G(ev, 0, 3, G03) && event_G(ev, 1, 2, G12);
                Big<L8> t1, t2, X, N1, N2;
                ev.ok = ev.ok && big_mul(t1, G02, G13) && big_mul(t2, G03, G12) && big_addsub(X, t1, t2, -1);
                ev.ok = ev.ok && big_mul(t1, G00, G11) && big_mul(t2, G01, G01) && big_addsub(N1, t1, t2, -1);
                ev.ok = ev.ok && big_mul(t1, G22, G33) && big_mul(t2, G23, G23) && big_addsub(N2, t1, t2, -1);
                Big<L16> R2, X2;
                ev.ok = ev.ok && big_mul(R2, N1, N2) && big_mul(X2, X, X);
                for (int k = 1; k < nb; ++k)
                    if (cmp_sqrt_x2(X, X2, R2, ed[k], ev.ok) <= 0) ++j;
            } else if (kind[a] == X_ABSCOS) {
                // |cos theta| >= e_k  <=>  sign(|Nn| - e_k sqrt(A B)) >= 0
                const int sl = slots[a];
                Big<L4> Nn, A, t1, t2;
                Big<L2> Bv, dd;
                ev.ok = ev.ok && big_mul(t1, ev.PP[sl], ev.P[0]) && big_mul(t2, ev.M2, ev.q[sl][0]) &&
                        big_addsub(Nn, t1, t2, -1);
                ev.ok = ev.ok && event_G(ev, sl, sl, A);
                ev.ok = ev.ok && big_mul(dd, ev.P[0], ev.P[0]) && big_addsub(Bv, dd, ev.M2, -1);
                Big<L4 + L2> AB;
                Big<2 * L4> Nn2;
                ev.ok = ev.ok && big_mul(AB, A, Bv);
                Nn.neg = 0;
                ev.ok = ev.ok && big_mul(Nn2, Nn, Nn);
                for (int k = 1; k < nb; ++k)
                    if (cmp_sqrt_x2(Nn, Nn2, AB, ed[k], ev.ok) >= 0) ++j;
            } else {
                // m >= e_k  <=>  m^2 >= e_k^2 (e_k >= 0); m^2 < 0 lies below every edge
                const int mask = slots[a];
                Big<L1> Sm[4], t;
                for (int c = 0; c < 4; ++c) {
                    big_zero(Sm[c]);
                    for (int k = 0; k < 4; ++k)
                        if (mask & (1 << k)) {
                            ev.ok = ev.ok && big_addsub(t, Sm[c], ev.q[k][c], 1);
                            big_copy(Sm[c], t);
                        }
                }
                Big<L2> m2;
                ev.ok = ev.ok && mdot(m2, Sm, Sm);
                int c_lo = 0, c_hi = 0, cnt = 0;
                for (int k = 0; k <= nb; ++k) {
                    int c;
                    if (m2.neg) {
                        c = -1;
                    } else {
                        int64_t ym;
                        int ye;
                        decode_f64(ed[k], ym, ye);
                        Big<2> yb;
                        Big<4> y2;
                        big_zero(yb);
                        const uint64_t am = ym < 0 ? (uint64_t)(-ym) : (uint64_t)ym;
                        yb.w[0] = (uint32_t)am;
                        yb.w[1] = (uint32_t)(am >> 32);
                        yb.len = 2;
                        big_norm(yb);
                        ev.ok = ev.ok && big_mul(y2, yb, yb);
                        c = cmp_scaled(m2, -2 * ev.shift, y2, 2 * ye, ev.ok);
                    }
                    if (k == 0) c_lo = c;
                    if (k == nb) c_hi = c;
                    if (k > 0 && k < nb && c >= 0) ++cnt;
                }
                j = (c_lo < 0 || c_hi > 0) ? -1 : cnt;
            }
            if (j < 0) oor = true;
            b = b * nb + (j < 0 ? 0 : j);
        }
        bin = oor ? -1 : b;
    }
    if (!ev.ok) {
        bin = -1;
        return X_UNRESOLVED;
    }
    return cls;
}

}  // namespace tpx
