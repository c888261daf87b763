// Device kernels of the T-odd triple-product pass (gfx950).
//
// One persistent kernel walks a contiguous range of a virtual event space that
// concatenates every sample of a batch.  Per event:
//   1. tag check; validity (P future time-like) certified in float64;
//   2. sign of C_T^inv = det[P; p_A; p_B; p_C] (Sect. 5, evaluated as
//      sigma * det[p0;p1;p2;p3] in kernel slot order): float32 Kahan-FMA
//      minors with a running forward bound (TP_PREC_F32_RECHECK) rechecked in
//      float64 when the bound does not decide, or float64 directly;
//   3. class by eq. (4) from flavour and sign;
//   4. phase-space bins (plane angle, invariant mass, helicity-type angle) in
//      float64 with rigorous running error bounds against the bin edges;
//   5. counts: per-wave LDS histogram copies (ds_add_u32) for the bins, wave
//      ballot/popcount for the integrated class totals and the statistics,
//      flushed to the sample's uint64 counters when the workgroup leaves the
//      sample.
// Any decision the floating-point bounds do not settle sends the whole event
// to a work list that the exact integer kernel (tp_exact.hip) decides.
//
// Build: -O3 -ffp-contract=off (every fused multiply-add is written out: the
// error bounds below count one rounding per written operation).
#include <hip/hip_runtime.h>

#include "tp_kernel.h"

namespace tpk {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr double U64 = 0x1p-53;   // unit roundoff, float64
constexpr float U32 = 0x1p-24f;   // unit roundoff, float32

struct EvOut {
    int cls;      // CLS_* (CLS_DEFER: exact tier)
    int bin;      // combined bin, -1 out of range
    int t2;       // float64 recheck of the sign was needed
    int why;      // deferred at: 1 validity, 2 sign, 3 first axis, 4 second axis
    double ct;    // C_T^inv estimate
};

__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }

// a*d - b*c.  With float32 inputs promoted to float64 both products are exact,
// so one fused operation gives the correctly rounded minor; otherwise Kahan's
// algorithm (error <= 2u |minor|, Jeannerod, Louvet & Muller 2013).
template <bool EXACT_PRODUCTS>
__device__ __forceinline__ double minor64(double a, double b, double c, double d)
{
    if (EXACT_PRODUCTS) return fma(a, d, -(b * c));
    const double w = b * c;
    const double e = fma(-b, c, w);
    const double f = fma(a, d, -w);
    return f + e;
}

__device__ __forceinline__ float minor32(float a, float b, float c, float d)
{
    const float w = b * c;
    const float e = fmaf(-b, c, w);
    const float f = fmaf(a, d, -w);
    return f + e;
}

// 2x2 minors of two rows a, b: m[k] = a_i b_j - a_j b_i for the column pairs
// k = (0,1) (0,2) (0,3) (1,2) (1,3) (2,3) -- the six components of the bivector a^b.
template <bool EXACT_PRODUCTS>
__device__ __forceinline__ void minors_f64(const double (&a)[4], const double (&b)[4], double (&m)[6])
{
    m[0] = minor64<EXACT_PRODUCTS>(a[0], a[1], b[0], b[1]);
    m[1] = minor64<EXACT_PRODUCTS>(a[0], a[2], b[0], b[2]);
    m[2] = minor64<EXACT_PRODUCTS>(a[0], a[3], b[0], b[3]);
    m[3] = minor64<EXACT_PRODUCTS>(a[1], a[2], b[1], b[2]);
    m[4] = minor64<EXACT_PRODUCTS>(a[1], a[3], b[1], b[3]);
    m[5] = minor64<EXACT_PRODUCTS>(a[2], a[3], b[2], b[3]);
}

// Laplace expansion of det[x0; x1; x2; x3] on the row pairs (0,1) | (2,3) from
// the minors of both pairs: column pair k pairs with its complement 5 - k,
// signs + - + + - +.  With exact products each minor is correctly rounded and
// |s - det| <= 8.1 u S; with Kahan minors (float64 inputs) 10.1 u S plus
// underflow terms, S = sum |m01_k| |m23_(5-k)|.
template <bool EXACT_PRODUCTS>
__device__ __forceinline__ bool det_f64(const double (&m01)[6], const double (&m23)[6], double &det)
{
    double s = m01[0] * m23[5];
    s = fma(-m01[1], m23[4], s);
    s = fma(m01[2], m23[3], s);
    s = fma(m01[3], m23[2], s);
    s = fma(-m01[4], m23[1], s);
    s = fma(m01[5], m23[0], s);
    double S = dabs(m01[0]) * dabs(m23[5]);
#pragma unroll
    for (int k = 1; k < 6; ++k) S = fma(dabs(m01[k]), dabs(m23[5 - k]), S);
    const double bound = EXACT_PRODUCTS ? (10.0 * U64) * S : fma(12.0 * U64, S, 0x1p-160);
    det = s;
    return dabs(s) > bound;
}

__device__ __forceinline__ bool det_f32(const float x[4][4], float &det)
{
    float m01[6], m23[6];
#define TP_M(k, a, b)                                       \
    m01[k] = minor32(x[0][a], x[0][b], x[1][a], x[1][b]);   \
    m23[k] = minor32(x[2][a], x[2][b], x[3][a], x[3][b]);
    TP_M(0, 0, 1) TP_M(1, 0, 2) TP_M(2, 0, 3) TP_M(3, 1, 2) TP_M(4, 1, 3) TP_M(5, 2, 3)
#undef TP_M
    float s = m01[0] * m23[5];
    s = fmaf(-m01[1], m23[4], s);
    s = fmaf(m01[2], m23[3], s);
    s = fmaf(m01[3], m23[2], s);
    s = fmaf(-m01[4], m23[1], s);
    s = fmaf(m01[5], m23[0], s);
    float S = fabsf(m01[0]) * fabsf(m23[5]);
    float T = fabsf(m01[0]) + fabsf(m23[0]);
#pragma unroll
    for (int k = 1; k < 6; ++k) {
        S = fmaf(fabsf(m01[k]), fabsf(m23[5 - k]), S);
        T += fabsf(m01[k]) + fabsf(m23[k]);
    }
    // |s - det| <= 10.01 u S  + (subnormal / flush-to-zero terms) <= 2^-124 per minor
    const float bound = fmaf(10.5f * U32, S, fmaf(0x1p-120f, T, 0x1p-120f));
    det = s;
    return fabsf(s) > bound;
}

__device__ __forceinline__ double mink(const double a[4], const double b[4])
{
    return fma(-a[3], b[3], fma(-a[2], b[2], fma(-a[1], b[1], a[0] * b[0])));
}

// Absolute floor added to every float64 error bound: it covers the absolute
// (not relative) rounding errors of results that fall below the normal range,
// so a bound stays valid for inputs of any magnitude; events that small simply
// defer to the later tiers.
constexpr double TINY = 0x1p-1000;

// 1/sqrt(D), D > 0: hardware estimate r0, one Newton step, and the residual
// rho = 1 - D r0^2 of the estimate.  With |rho| <= 2^-10 the result satisfies
// |r sqrt(D) - 1| <= 0.5 rho^2 + 3u  (Newton's error is 1.5 delta^2 for an
// estimate error delta, and |rho| >= 1.9 |delta|).  ``rel`` receives that bound.
__device__ __forceinline__ double rsqrt_cert(double D, double &rel, bool &ok)
{
    const double r0 = __builtin_amdgcn_rsq(D);
    const double t = D * r0;
    const double rho = fma(-t, r0, 1.0);
    const double r = fma(0.5 * r0, rho, r0);
    ok = ok && (dabs(rho) <= 0x1p-10);
    rel = fma(0.5 * rho, rho, 3.0 * U64);
    return r;
}

// Error bound of v = Y * r against the true ratio Y / sqrt(D) when |Y| <= sqrt(D)
// holds exactly: eY, eD bound |Y^ - Y| and |D^ - D| (eD <= D^/4), rel bounds
// |r sqrt(D^) - 1|.  Includes the rounding of v and of the later v +- eps.
__device__ __forceinline__ double ratio_eps(double v, double r, double rel, double eY, double eD)
{
    return fma(1.01, fma(dabs(v), rel + U64, fma(eY, r, 0.54 * eD * r * r)), 3.0 * U64);
}

// Plane angle between kernel planes (0,1) and (2,3) from the bivectors
// B1 = p0^p1, B2 = p2^p3 (their minors m01, m23).  The covector C with
// det[c; P; a; b] = c.C for every c is, in the M rest frame, (0, +-M (p*_a x p*_b)),
// so with the Minkowski products
//   X = C1.C2 = -M^2 n1.n2,  S_i = C_i.C_i = -M^2 |n_i|^2,  cos Phi = -X / sqrt(S1 S2),
// n_i the rest-frame plane normals.  The minors are shared with the sign.
// Error bounds (W = L1 norm of all components, so |P_c| <= W):
//   |P^_c - P_c| <= 2.01 u W;  |m^ - m| <= k u |m^| (k = 1 correctly rounded
//   minors of float inputs, 2 Kahan minors of float64 inputs);
//   each C_mu is a three-term fused sum: |C^_mu - C_mu| <= (3.02 + 2.01 + k) u W sum|m^|
//   <= 7.2 u W sum|m^| = eC;
//   |X^ - X| <= eC2 A1 + eC1 A2 + 4 eC1 eC2 + 4.01 u A1 A2 (A = L1 norm of C^),
//   |S^ - S| <= 2 eC A + 4 eC^2 + 4.01 u A^2.
// S1, S2 < 0 certified, then D = S1 S2 and the ratio as for the other angles.
__device__ __forceinline__ void covector(const double (&P)[4], const double (&m)[6], double (&C)[4])
{
    C[0] = fma(P[3], m[3], fma(-P[2], m[4], P[1] * m[5]));
    C[1] = fma(-P[3], m[1], fma(P[2], m[2], -(P[0] * m[5])));
    C[2] = fma(P[3], m[0], fma(-P[1], m[2], P[0] * m[4]));
    C[3] = fma(-P[2], m[0], fma(P[1], m[1], -(P[0] * m[3])));
}

__device__ __forceinline__ int bin_absphi_bv(const double (&m01)[6], const double (&m23)[6], const double (&P)[4],
                                             double W, const double *edges, int n, bool &sure)
{
    double C1[4], C2[4];
    covector(P, m01, C1);
    covector(P, m23, C2);
    const double M1 = ((dabs(m01[0]) + dabs(m01[1])) + (dabs(m01[2]) + dabs(m01[3]))) + (dabs(m01[4]) + dabs(m01[5]));
    const double M2s = ((dabs(m23[0]) + dabs(m23[1])) + (dabs(m23[2]) + dabs(m23[3]))) + (dabs(m23[4]) + dabs(m23[5]));
    const double eabs = fma(TINY, W, TINY);
    const double eC1 = fma((7.2 * U64) * W, M1, eabs);
    const double eC2 = fma((7.2 * U64) * W, M2s, eabs);
    const double A1 = (dabs(C1[0]) + dabs(C1[1])) + (dabs(C1[2]) + dabs(C1[3]));
    const double A2 = (dabs(C2[0]) + dabs(C2[1])) + (dabs(C2[2]) + dabs(C2[3]));
    const double X = fma(-C1[3], C2[3], fma(-C1[2], C2[2], fma(-C1[1], C2[1], C1[0] * C2[0])));
    const double S1 = fma(-C1[3], C1[3], fma(-C1[2], C1[2], fma(-C1[1], C1[1], C1[0] * C1[0])));
    const double S2 = fma(-C2[3], C2[3], fma(-C2[2], C2[2], fma(-C2[1], C2[1], C2[0] * C2[0])));
    const double u4 = 4.02 * U64;
    const double eX = fma(eC2, A1, fma(eC1, A2, fma(4.0 * eC1, eC2, fma(u4 * A1, A2, TINY))));
    const double eS1 = fma(2.0 * eC1, A1, fma(4.0 * eC1, eC1, fma(u4 * A1, A1, TINY)));
    const double eS2 = fma(2.0 * eC2, A2, fma(4.0 * eC2, eC2, fma(u4 * A2, A2, TINY)));
    bool ok = (-S1 > eS1) && (-S2 > eS2);
    const double D = S1 * S2;
    const double eD = fma(dabs(S1) + eS1, eS2, fma(dabs(S2), eS1, fma(U64, D, TINY)));
    ok = ok && (eD <= 0.25 * D);
    double rel;
    const double r = rsqrt_cert(D, rel, ok);
    const double v = -X * r;
    const double eps = ratio_eps(v, r, rel, eX, eD);
    const double vhi = v + eps, vlo = v - eps;
    int bin = 0;
    for (int k = 1; k < n; ++k) {
        const double c = edges[k];
        const bool le = vhi <= c;
        bin += le ? 1 : 0;
        ok = ok && (le || vlo > c);
    }
    sure = sure && ok;
    return bin;
}

// |cos theta| of kernel slot s against the M flight direction:
// Nn = (P.p_s) E_P - M^2 E_s, A = G_ss, B = |P_lab|^2, |cos| = |Nn| / sqrt(A B).
// edges 0 = e_0 < ... < e_n = 1; returns #{k in 1..n-1 : |cos| >= e_k}.
__device__ __forceinline__ int bin_abscos(const double x[4][4], const double w[4], double W,
                                          const double P[4], double M2, double eM, double kdot,
                                          int s, const double *edges, int n, bool &sure)
{
    double xs[4];
    double ws = w[0];
#pragma unroll
    for (int c = 0; c < 4; ++c) xs[c] = x[0][c];
    if (s == 1) {
#pragma unroll
        for (int c = 0; c < 4; ++c) xs[c] = x[1][c];
        ws = w[1];
    } else if (s == 2) {
#pragma unroll
        for (int c = 0; c < 4; ++c) xs[c] = x[2][c];
        ws = w[2];
    } else if (s == 3) {
#pragma unroll
        for (int c = 0; c < 4; ++c) xs[c] = x[3][c];
        ws = w[3];
    }
    const double u2 = 2.01 * U64;
    const double PPs = mink(P, xs);
    const double ePP = (7.2 * U64) * W * ws;
    const double EP = P[0];
    const double eEP = (3.01 * U64) * W;
    const double Es = xs[0];
    const double dss = mink(xs, xs);
    const double eds = (kdot * U64) * ws * ws;
    const double Nn = fma(PPs, EP, -(M2 * Es));
    const double eNn = fma(dabs(PPs) + ePP, eEP, fma(dabs(EP), ePP,
                       fma(dabs(Es), eM, fma(u2, dabs(PPs * EP) + dabs(M2 * Es), TINY))));
    const double A = fma(PPs, PPs, -(M2 * dss));
    const double eA = fma(2.0 * dabs(PPs) + ePP, ePP, fma(dabs(M2) + eM, eds,
                      fma(dabs(dss), eM, fma(u2, PPs * PPs + dabs(M2 * dss), TINY))));
    const double B = fma(P[3], P[3], fma(P[2], P[2], P[1] * P[1]));
    const double eB = fma(6.1 * U64 * W, W, fma(3.1 * U64, B, TINY));
    bool ok = (A > eA) && (B > eB);
    const double D = A * B;
    const double eD = fma(A + eA, eB, fma(B, eA, fma(U64, D, TINY)));
    ok = ok && (eD <= 0.25 * D);
    double rel;
    const double r = rsqrt_cert(D, rel, ok);
    const double v = dabs(Nn) * r;
    const double eps = ratio_eps(v, r, rel, eNn, eD);
    const double vhi = v + eps, vlo = v - eps;
    int bin = 0;
    for (int k = 1; k < n; ++k) {
        const double e = edges[k];
        const bool ge = vlo >= e;
        bin += ge ? 1 : 0;
        ok = ok && (ge || vhi < e);
    }
    sure = sure && ok;
    return bin;
}

// Invariant mass of the kernel slots in ``mask``.  ed: [sq_lo(n+1) | sq_hi(n+1)]
// with sq_lo_k <= e_k^2 <= sq_hi_k.  Returns the bin or -1 (out of range).
__device__ __forceinline__ int bin_mass(const double x[4][4], const double w[4], int mask,
                                        const double *ed, int n, double glo, double ginv, bool &sure)
{
    double S[4] = { 0.0, 0.0, 0.0, 0.0 };
    double WS = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (mask & (1 << s)) {
#pragma unroll
            for (int c = 0; c < 4; ++c) S[c] += x[s][c];
            WS += w[s];
        }
    const double m2 = fma(-S[3], S[3], fma(-S[2], S[2], fma(-S[1], S[1], S[0] * S[0])));
    const double em = fma((12.4 * U64) * WS, WS, TINY);
    const double *sqlo = ed, *sqhi = ed + (n + 1);
    const double mlo = m2 - em, mhi = m2 + em;
    // guess on a uniform grid in m, then certify against the two neighbouring edges
    const float mg = sqrtf(fmaxf((float)m2, 0.0f));
    const float t = (float)(((double)mg - glo) * ginv);
    int j = 0;
    if (t >= (float)(n - 1)) j = n - 1;
    else if (t >= 0.0f) j = (int)t;
    if (mlo >= sqhi[j] && (j == n - 1 ? mhi <= sqlo[n] : mhi < sqlo[j + 1])) return j;
    // full scan
    if (mhi < sqlo[0] || mlo > sqhi[n]) return -1;          // certainly outside
    if (!(mlo >= sqhi[0] && mhi <= sqlo[n])) {               // not certainly inside
        sure = false;
        return -1;
    }
    int bin = 0;
    bool dec = true;
    for (int k = 1; k < n; ++k) {
        const bool ge = mlo >= sqhi[k];
        bin += ge ? 1 : 0;
        dec = dec && (ge || mhi < sqlo[k]);
    }
    sure = sure && dec;
    return bin;
}

struct Seg {
    int32_t sigma, nb0, nb1, slots0, slots1;
    double glo0, ginv0, glo1, ginv1;
    const double *e0, *e1;    // LDS edge data of each axis
};

// One axis of compile-time kind KIND: bin index, or -1 (out of range).
template <int KIND, bool EXACTP>
__device__ __forceinline__ int axis_bin(const double (&x)[4][4], const double (&w)[4], double W,
                                        const double (&m01)[6], const double (&m23)[6],
                                        const double (&P)[4], double M2, double eM, int nb, int sl,
                                        const double *ed, double glo, double ginv, bool &sure)
{
    constexpr double KDOT = EXACTP ? 3.02 : 4.02;
    if constexpr (KIND == AX_ABSPHI) return bin_absphi_bv(m01, m23, P, W, ed, nb, sure);
    else if constexpr (KIND == AX_MASS) return bin_mass(x, w, sl, ed, nb, glo, ginv, sure);
    else return bin_abscos(x, w, W, P, M2, eM, KDOT, sl, ed, nb, sure);
}

// Whole event, with the binning scheme (K0, K1; AX_NONE = absent) fixed at
// compile time.
template <typename Tin, int PREC, int K0, int K1>
__device__ __forceinline__ EvOut eval_event(const Tin (&q)[4][4], int tag, const Seg &g)
{
    constexpr bool EXACTP = sizeof(Tin) == 4;
    EvOut o;
    o.cls = CLS_DEFER;
    o.bin = -1;
    o.t2 = 0;
    o.why = 1;
    o.ct = 0.0;
    if (tag != 0 && tag != 1) {
        o.cls = CLS_INVALID;
        return o;
    }
    double x[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) x[s][c] = (double)q[s][c];

    // validity: E_P > 0 and M^2 > 0 (|M^2 computed - M^2| <= 10.1 u W^2 + underflow)
    double w[4], P[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) w[s] = (dabs(x[s][0]) + dabs(x[s][1])) + (dabs(x[s][2]) + dabs(x[s][3]));
    const double W = (w[0] + w[1]) + (w[2] + w[3]);
#pragma unroll
    for (int c = 0; c < 4; ++c) P[c] = (x[0][c] + x[1][c]) + (x[2][c] + x[3][c]);
    const double M2 = fma(-P[3], P[3], fma(-P[2], P[2], fma(-P[1], P[1], P[0] * P[0])));
    const double Emin = fmin(fmin(x[0][0], x[1][0]), fmin(x[2][0], x[3][0]));
    if (!(Emin >= 0.0 && P[0] > 0.0 && M2 > fma((11.0 * U64) * W, W, TINY))) return o;

    // Sign of the triple product.  The plane-angle bins need the float64
    // minors (the bivectors p0^p1, p2^p3) anyway, and the determinant from them
    // costs a dozen operations, less than the float32 contraction: so the
    // float32 sign with float64 recheck runs only when no plane angle is binned.
    constexpr bool NEED_BV = K0 == AX_ABSPHI || K1 == AX_ABSPHI;
    constexpr bool F32_SIGN = PREC == 1 && !NEED_BV;
    double m01[6], m23[6];
    double det;
    bool sure;
    if constexpr (F32_SIGN) {
        float det32;
        float qf[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 4; ++c) qf[s][c] = (float)q[s][c];
        sure = det_f32(qf, det32);
        det = (double)det32;
        if (!sure) {
            minors_f64<EXACTP>(x[0], x[1], m01);
            minors_f64<EXACTP>(x[2], x[3], m23);
            o.t2 = 1;
            sure = det_f64<EXACTP>(m01, m23, det);
        }
    } else {
        minors_f64<EXACTP>(x[0], x[1], m01);
        minors_f64<EXACTP>(x[2], x[3], m23);
        sure = det_f64<EXACTP>(m01, m23, det);
    }
    const double ct = g.sigma > 0 ? det : -det;
    o.ct = ct;
    o.why = 2;
    if (!sure) return o;
    const int cls = tag == 0 ? (ct > 0.0 ? CLS_I : CLS_II) : (ct < 0.0 ? CLS_III : CLS_IV);
    if constexpr (K0 == AX_NONE) {
        o.cls = cls;
        o.bin = 0;
        return o;
    } else {
        const double eM = (10.2 * U64) * W * W;
        bool bsure = true;
        o.why = 3;
        const int j0 = axis_bin<K0, EXACTP>(x, w, W, m01, m23, P, M2, eM, g.nb0, g.slots0, g.e0, g.glo0, g.ginv0,
                                            bsure);
        bool oor = j0 < 0;
        int bin = j0 < 0 ? 0 : j0;
        if constexpr (K1 != AX_NONE) {
            if (bsure) o.why = 4;
            const int j1 = axis_bin<K1, EXACTP>(x, w, W, m01, m23, P, M2, eM, g.nb1, g.slots1, g.e1, g.glo1,
                                                g.ginv1, bsure);
            oor = oor || j1 < 0;
            bin = bin * g.nb1 + (j1 < 0 ? 0 : j1);
        }
        if (!bsure) return o;
        o.cls = cls;
        o.bin = oor ? -1 : bin;
        return o;
    }
}

__device__ __forceinline__ uint32_t wave_count(bool p)
{
    return (uint32_t)__popcll(__ballot(p));
}

template <typename T>
__device__ __forceinline__ T ldnt(const void *p, int64_t i)
{
    typedef const T __attribute__((address_space(1))) *gptr;
    return __builtin_nontemporal_load((gptr)p + i);
}

// Load EPL consecutive events (EPL = 1, 2 or 4 per lane) starting at ``base``
// (a multiple of EPL) from the 16 component arrays and the tag array.
template <typename Tin, int EPL>
__device__ __forceinline__ void load_events(const void *const (&ptr)[16], const int8_t *tag, int64_t base,
                                            bool vec_ok, int64_t n_valid, Tin (&q)[EPL][4][4], int (&tg)[EPL])
{
    constexpr int BYTES = EPL * (int)sizeof(Tin);
    if (EPL > 1 && !(vec_ok && base + EPL <= n_valid)) {
#pragma unroll
        for (int e = 0; e < EPL; ++e) {
            const int64_t i = base + e;
            const bool in = i < n_valid;
#pragma unroll
            for (int k = 0; k < 16; ++k) q[e][k >> 2][k & 3] = in ? ldnt<Tin>(ptr[k], i) : (Tin)0;
            tg[e] = in ? (int)ldnt<int8_t>(tag, i) : -1;
        }
        return;
    }
    if constexpr (EPL == 1) {
        const bool in = base < n_valid;
#pragma unroll
        for (int k = 0; k < 16; ++k) q[0][k >> 2][k & 3] = in ? ldnt<Tin>(ptr[k], base) : (Tin)0;
        tg[0] = in ? (int)ldnt<int8_t>(tag, base) : -1;
    } else if constexpr (BYTES == 8) {
        typedef Tin v2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const v2 v = ldnt<v2>(ptr[k], base >> 1);
            q[0][k >> 2][k & 3] = v.x;
            q[1][k >> 2][k & 3] = v.y;
        }
        const uint16_t t = ldnt<uint16_t>(tag, base >> 1);
        tg[0] = (int)(int8_t)(t & 0xff);
        tg[1] = (int)(int8_t)(t >> 8);
    } else if constexpr (EPL == 4 && sizeof(Tin) == 4) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const f32x4 v = ldnt<f32x4>(ptr[k], base >> 2);
            q[0][k >> 2][k & 3] = v.x;
            q[1][k >> 2][k & 3] = v.y;
            q[2][k >> 2][k & 3] = v.z;
            q[3][k >> 2][k & 3] = v.w;
        }
        const uint32_t t = ldnt<uint32_t>(tag, base >> 2);
#pragma unroll
        for (int e = 0; e < 4; ++e) tg[e] = (int)(int8_t)(t >> (8 * e));
    } else {   // EPL == 2, double: 16-byte loads
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const f64x2 v = ldnt<f64x2>(ptr[k], base >> 1);
            q[0][k >> 2][k & 3] = v.x;
            q[1][k >> 2][k & 3] = v.y;
        }
        const uint16_t t = ldnt<uint16_t>(tag, base >> 1);
        tg[0] = (int)(int8_t)(t & 0xff);
        tg[1] = (int)(int8_t)(t >> 8);
    }
}

struct WaveCounts {
    uint32_t c0, c1, c2, c3, zero, inv, oor, t2, t3, un;
};

struct SegIO {
    const void *ptr[16];
    const int8_t *tag;
    int8_t *cls_out;
    double *ct_out;
    bool vec;
};

// One tile: EPL consecutive events per lane starting at ``base``.
template <typename Tin, int PREC, int MODE, int EPL, int K0, int K1>
__device__ __forceinline__ void process_tile(const KParams &kp, int s, const SegIO &io, const Seg &g,
                                             const Tin (&q)[EPL][4][4], const int (&tg)[EPL], int64_t base,
                                             int64_t ev1, uint32_t *myhist, WaveCounts &wc)
{
    constexpr bool BINNED = MODE == 0 && K0 != AX_NONE;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const int64_t i = base + e;
        const bool in = i < ev1;
        EvOut o;
        if (in) {
            o = eval_event<Tin, PREC, K0, K1>(q[e], tg[e], g);
        } else {
            o.cls = -1;
            o.bin = -1;
            o.t2 = 0;
            o.why = 0;
            o.ct = 0.0;
        }
        bool listed = false, unres = false;
        if (o.cls == CLS_DEFER) {
            const uint32_t slot = atomicAdd(kp.xcount, 1u);
            if (slot < kp.xcap) {
                kp.xlist[slot] = ((uint64_t)o.why << 60) | ((uint64_t)s << 40) | (uint64_t)i;
                listed = true;
            } else {
                unres = true;
            }
        }
        if (MODE == 1 && in) {
            io.cls_out[i] = (int8_t)(unres ? CLS_UNRESOLVED : o.cls);
            if (io.ct_out) io.ct_out[i] = o.ct;
        }
        const bool classified = o.cls >= 0 && o.cls < 4;
        if (BINNED && classified && o.bin >= 0) atomicAdd(&myhist[(1 + o.bin) * 4 + o.cls], 1u);
        if (MODE == 0) {
            wc.c0 += wave_count(o.cls == CLS_I);
            wc.c1 += wave_count(o.cls == CLS_II);
            wc.c2 += wave_count(o.cls == CLS_III);
            wc.c3 += wave_count(o.cls == CLS_IV);
        }
        // rare outcomes: one ballot decides whether the wave counts them
        const bool oor = BINNED && classified && o.bin < 0;
        const bool rare = (o.cls >= CLS_ZERO) || o.t2 || oor;
        if (__ballot(rare)) {
            wc.zero += wave_count(o.cls == CLS_ZERO);
            wc.inv += wave_count(o.cls == CLS_INVALID);
            wc.oor += wave_count(oor);
            wc.t2 += wave_count(o.t2 != 0);
            wc.t3 += wave_count(listed);
            wc.un += wave_count(unres);
        }
    }
}

// Whether the event loop keeps the next tile's inputs in flight in registers
// (two register sets used in turn).  Off where the second set would not fit
// the register budget of two waves per SIMD.
template <typename Tin, int EPL, int K0, int K1>
constexpr bool prefetch_tiles()
{
    return EPL * (int)sizeof(Tin) <= 8;
}

// The event loop of one segment (events [ev0, ev1) of sample s).
template <typename Tin, int PREC, int MODE, int EPL, int K0, int K1>
__device__ __forceinline__ void run_segment(const KParams &kp, int s, const SegIO &io, const Seg &g,
                                            int64_t ev0, int64_t ev1, uint32_t *myhist, WaveCounts &wc)
{
    const int64_t lane0 = (int64_t)EPL * threadIdx.x;
    const int64_t step = (int64_t)EPL * blockDim.x;
    if constexpr (prefetch_tiles<Tin, EPL, K0, K1>()) {
        // tile t is evaluated while tile t + 1 loads into the other register set
        Tin qa[EPL][4][4], qb[EPL][4][4];
        int ta[EPL], tb[EPL];
        int64_t t0 = ev0;
        if (t0 < ev1) load_events<Tin, EPL>(io.ptr, io.tag, t0 + lane0, io.vec, ev1, qa, ta);
        while (t0 < ev1) {
            const int64_t t1 = t0 + step;
            if (t1 < ev1) load_events<Tin, EPL>(io.ptr, io.tag, t1 + lane0, io.vec, ev1, qb, tb);
            process_tile<Tin, PREC, MODE, EPL, K0, K1>(kp, s, io, g, qa, ta, t0 + lane0, ev1, myhist, wc);
            if (t1 >= ev1) break;
            const int64_t t2 = t1 + step;
            if (t2 < ev1) load_events<Tin, EPL>(io.ptr, io.tag, t2 + lane0, io.vec, ev1, qa, ta);
            process_tile<Tin, PREC, MODE, EPL, K0, K1>(kp, s, io, g, qb, tb, t1 + lane0, ev1, myhist, wc);
            t0 = t2;
        }
    } else {
        for (int64_t t0 = ev0; t0 < ev1; t0 += step) {
            Tin q[EPL][4][4];
            int tg[EPL];
            load_events<Tin, EPL>(io.ptr, io.tag, t0 + lane0, io.vec, ev1, q, tg);
            process_tile<Tin, PREC, MODE, EPL, K0, K1>(kp, s, io, g, q, tg, t0 + lane0, ev1, myhist, wc);
        }
    }
}

// The pass over samples [kp.sbeg, kp.send), all of binning scheme (K0, K1):
// each workgroup takes a contiguous range of the virtual event space, splits
// it at sample boundaries, counts into LDS and flushes every segment.
template <typename Tin, int PREC, int MODE, int EPL, int K0, int K1>
__global__ __launch_bounds__(512) void tp_pass_kernel(const KParams kp)
{
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *hist = reinterpret_cast<uint32_t *>(smem);
    const int hist_words = kp.lds_copies * kp.hist_stride;
    double *ecache = reinterpret_cast<double *>(smem + ((hist_words * 4 + 15) & ~15));
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    uint32_t *myhist = hist + (wave % kp.lds_copies) * kp.hist_stride;

    int64_t vbeg = kp.vbeg + (int64_t)blockIdx.x * kp.range;
    const int64_t vend = vbeg + kp.range < kp.vend ? vbeg + kp.range : kp.vend;
    if (vbeg >= vend) return;
    int lo = kp.sbeg, hi = kp.send - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kp.samples[mid].vstart <= vbeg) lo = mid;
        else hi = mid - 1;
    }
    for (int s = lo; s < kp.send && vbeg < vend; ++s) {
        const KSample *S = kp.samples + s;
        const int64_t sv0 = S->vstart;
        const int64_t sv1 = s + 1 < kp.send ? kp.samples[s + 1].vstart : kp.vend;
        if (sv1 <= vbeg) continue;
        const int64_t segend = vend < sv1 ? vend : sv1;
        const int64_t n = S->n;
        const int64_t ev0 = vbeg - sv0;
        const int64_t ev1 = (segend - sv0) < n ? (segend - sv0) : n;
        vbeg = segend;
        if (ev1 <= ev0) continue;

        // everything the event loop needs, read once per segment
        SegIO io;
#pragma unroll
        for (int k = 0; k < 16; ++k) io.ptr[k] = S->p[k];
        io.tag = S->tag;
        io.vec = S->vec != 0;
        io.cls_out = S->cls_out;
        io.ct_out = S->ct_out;
        uint64_t *counts = S->counts;
        uint64_t *stats = S->stats;
        Seg g;
        g.sigma = S->sigma;
        g.nb0 = S->nbins[0];
        g.nb1 = S->nbins[1];
        g.slots0 = S->slots[0];
        g.slots1 = S->slots[1];
        g.glo0 = S->guess_lo[0];
        g.glo1 = S->guess_lo[1];
        g.ginv0 = S->guess_inv[0];
        g.ginv1 = S->guess_inv[1];
        const int nd0 = K0 != AX_NONE ? edge_doubles(K0, g.nb0) : 0;
        const int nd1 = K1 != AX_NONE ? edge_doubles(K1, g.nb1) : 0;
        const int eoff0 = S->eoff[0], eoff1 = S->eoff[1];
        const int nrow = (S->nbtot + 1) * 4;
        g.e0 = ecache;
        g.e1 = ecache + nd0;
        const int ncnt = nrow + NSTAT;
        for (int i = tid; i < hist_words; i += nthr) hist[i] = 0;
        for (int i = tid; i < nd0; i += nthr) ecache[i] = kp.edges[eoff0 + i];
        for (int i = tid; i < nd1; i += nthr) ecache[nd0 + i] = kp.edges[eoff1 + i];
        __syncthreads();

        WaveCounts wc = { 0, 0, 0, 0, 0, 0, 0, 0, 0, 0 };
        run_segment<Tin, PREC, MODE, EPL, K0, K1>(kp, s, io, g, ev0, ev1, myhist, wc);
        if (lane == 0) {
            if (MODE == 0) {
                atomicAdd(&myhist[0], wc.c0);
                atomicAdd(&myhist[1], wc.c1);
                atomicAdd(&myhist[2], wc.c2);
                atomicAdd(&myhist[3], wc.c3);
            }
            atomicAdd(&myhist[nrow + ST_ZERO], wc.zero);
            atomicAdd(&myhist[nrow + ST_INVALID], wc.inv);
            atomicAdd(&myhist[nrow + ST_OOR], wc.oor);
            atomicAdd(&myhist[nrow + ST_TIER2], wc.t2);
            atomicAdd(&myhist[nrow + ST_TIER3], wc.t3);
            atomicAdd(&myhist[nrow + ST_UNRESOLVED], wc.un);
        }
        __syncthreads();
        for (int i = tid; i < ncnt; i += nthr) {
            uint32_t v = 0;
            for (int k = 0; k < kp.lds_copies; ++k) v += hist[k * kp.hist_stride + i];
            if (i < nrow) {
                if (v && counts) atomicAdd((unsigned long long *)(counts + i), (unsigned long long)v);
            } else if (i - nrow == ST_EVENTS) {
                atomicAdd((unsigned long long *)(stats + ST_EVENTS), (unsigned long long)(ev1 - ev0));
            } else if (v) {
                atomicAdd((unsigned long long *)(stats + (i - nrow)), (unsigned long long)v);
            }
        }
        __syncthreads();
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers
namespace {
template <typename T, int P, int M, int EPL, int K0, int K1>
void launch_one(const KParams &kp, int grid, int block, size_t lds, hipStream_t st)
{
    // with a plane angle binned, the float32-sign variant is the float64 one
    constexpr int PE = (K0 == AX_ABSPHI || K1 == AX_ABSPHI) ? 0 : P;
    hipLaunchKernelGGL((tp_pass_kernel<T, PE, M, EPL, K0, K1>), dim3(grid), dim3(block), lds, st, kp);
}

template <typename T, int P, int M, int K0, int K1>
void launch_epl(int epl, const KParams &kp, int grid, int block, size_t lds, hipStream_t st)
{
    if constexpr (sizeof(T) == 4) {
        if (epl >= 4) {
            launch_one<T, P, M, 4, K0, K1>(kp, grid, block, lds, st);
            return;
        }
    }
    if (epl >= 2) launch_one<T, P, M, 2, K0, K1>(kp, grid, block, lds, st);
    else launch_one<T, P, M, 1, K0, K1>(kp, grid, block, lds, st);
}

template <typename T, int P, int M>
bool launch_scheme(int k0, int k1, int epl, const KParams &kp, int grid, int block, size_t lds, hipStream_t st)
{
    if constexpr (M == 1) {
        if (k0 != AX_NONE || k1 != AX_NONE) return false;
        launch_epl<T, P, M, AX_NONE, AX_NONE>(epl, kp, grid, block, lds, st);
        return true;
    } else {
#define TP_CASE(A, B)                                                          \
    case A * 4 + B: launch_epl<T, P, M, A, B>(epl, kp, grid, block, lds, st); return true;
        switch (k0 * 4 + k1) {
            TP_CASE(AX_NONE, AX_NONE)
            TP_CASE(AX_ABSPHI, AX_NONE)
            TP_CASE(AX_MASS, AX_NONE)
            TP_CASE(AX_ABSCOS, AX_NONE)
            TP_CASE(AX_ABSPHI, AX_MASS)
            TP_CASE(AX_ABSPHI, AX_ABSCOS)
            TP_CASE(AX_MASS, AX_ABSPHI)
            TP_CASE(AX_MASS, AX_MASS)
            TP_CASE(AX_MASS, AX_ABSCOS)
            TP_CASE(AX_ABSCOS, AX_ABSPHI)
            TP_CASE(AX_ABSCOS, AX_MASS)
            TP_CASE(AX_ABSCOS, AX_ABSCOS)
        default: return false;
        }
#undef TP_CASE
    }
}
}  // namespace

hipError_t launch_pass(int dtype, int prec, int mode, int epl, int k0, int k1, const KParams &kp, int grid,
                       int block, size_t lds, hipStream_t st)
{
    bool ok;
    if (dtype == 0) {
        if (prec == 1) {
            ok = mode == 0 ? launch_scheme<float, 1, 0>(k0, k1, epl, kp, grid, block, lds, st)
                           : launch_scheme<float, 1, 1>(k0, k1, epl, kp, grid, block, lds, st);
        } else {
            ok = mode == 0 ? launch_scheme<float, 0, 0>(k0, k1, epl, kp, grid, block, lds, st)
                           : launch_scheme<float, 0, 1>(k0, k1, epl, kp, grid, block, lds, st);
        }
    } else {
        ok = mode == 0 ? launch_scheme<double, 0, 0>(k0, k1, epl, kp, grid, block, lds, st)
                       : launch_scheme<double, 0, 1>(k0, k1, epl, kp, grid, block, lds, st);
    }
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace tpk
