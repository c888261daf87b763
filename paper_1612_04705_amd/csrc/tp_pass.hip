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

// Laplace expansion of det[x0; x1; x2; x3] on the row pairs (0,1) | (2,3):
// column pairs k = (0,1) (0,2) (0,3) (1,2) (1,3) (2,3), complement 5 - k,
// signs + - + + - +.
template <bool EXACT_PRODUCTS>
__device__ __forceinline__ bool det_f64(const double x[4][4], double &det)
{
    double m01[6], m23[6];
#define TP_M(k, a, b)                                                          \
    m01[k] = minor64<EXACT_PRODUCTS>(x[0][a], x[0][b], x[1][a], x[1][b]);      \
    m23[k] = minor64<EXACT_PRODUCTS>(x[2][a], x[2][b], x[3][a], x[3][b]);
    TP_M(0, 0, 1) TP_M(1, 0, 2) TP_M(2, 0, 3) TP_M(3, 1, 2) TP_M(4, 1, 3) TP_M(5, 2, 3)
#undef TP_M
    double s = m01[0] * m23[5];
    s = fma(-m01[1], m23[4], s);
    s = fma(m01[2], m23[3], s);
    s = fma(m01[3], m23[2], s);
    s = fma(-m01[4], m23[1], s);
    s = fma(m01[5], m23[0], s);
    double S = dabs(m01[0]) * dabs(m23[5]);
#pragma unroll
    for (int k = 1; k < 6; ++k) S = fma(dabs(m01[k]), dabs(m23[5 - k]), S);
    // |s - det| <= 8.1 u S (exact products) / 10.1 u S + underflow terms (Kahan minors)
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

__device__ __forceinline__ double dmax(double a, double b) { return __builtin_fmax(a, b); }

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

// Plane angle between kernel planes (0,1) and (2,3): cos Phi = X / sqrt(N1 N2).
// edges: c_0 = 1 > c_1 > ... > c_n = -1; returns #{k in 1..n-1 : cos Phi <= c_k}.
// Error bounds: |P.p_a^ - P.p_a| <= 7.2 u W w_a, |M^2^ - M^2| <= 10.2 u W^2,
// |d_ab^ - d_ab| <= kdot u w_a w_b (w_a = L1 norm of p_a, W = sum of w_a); one
// bound eG serves every G_ab, built from the largest |P.p_a|, |d_ab| and w_a.
__device__ __forceinline__ int bin_absphi(const double x[4][4], double W, double wmax, double M2,
                                          double kdot, const double *edges, int n, bool &sure)
{
    const double d00 = mink(x[0], x[0]), d11 = mink(x[1], x[1]), d22 = mink(x[2], x[2]), d33 = mink(x[3], x[3]);
    const double d01 = mink(x[0], x[1]), d02 = mink(x[0], x[2]), d03 = mink(x[0], x[3]);
    const double d12 = mink(x[1], x[2]), d13 = mink(x[1], x[3]), d23 = mink(x[2], x[3]);
    const double P0 = (d00 + d01) + (d02 + d03);
    const double P1 = (d01 + d11) + (d12 + d13);
    const double P2 = (d02 + d12) + (d22 + d23);
    const double P3 = (d03 + d13) + (d23 + d33);
#define TP_G(a, b, dab) fma(P##a, P##b, -(M2 * dab))
    const double G00 = TP_G(0, 0, d00), G11 = TP_G(1, 1, d11), G22 = TP_G(2, 2, d22), G33 = TP_G(3, 3, d33);
    const double G01 = TP_G(0, 1, d01), G23 = TP_G(2, 3, d23);
    const double G02 = TP_G(0, 2, d02), G13 = TP_G(1, 3, d13), G03 = TP_G(0, 3, d03), G12 = TP_G(1, 2, d12);
#undef TP_G
    const double PPm = dmax(dmax(dabs(P0), dabs(P1)), dmax(dabs(P2), dabs(P3)));
    const double dm = dmax(dmax(dmax(dabs(d00), dabs(d11)), dmax(dabs(d22), dabs(d33))),
                           dmax(dmax(dmax(dabs(d01), dabs(d02)), dmax(dabs(d03), dabs(d12))),
                                dmax(dabs(d13), dabs(d23))));
    const double aM = dabs(M2);
    const double uWW = U64 * W * W;
    // eG >= |G^ - G| for every pair (first-order terms, second-order 94 u^2 W^4, roundings)
    const double eG = fma(U64, fma((14.4 * W) * wmax, PPm, fma(10.2 * W * W, dm,
                          fma((kdot * wmax) * wmax, aM, 2.01 * fma(PPm, PPm, aM * dm)))),
                          94.0 * uWW * uWW);
    const double u2 = 2.01 * U64;
    const double p1 = G03 * G12;
    const double X = fma(G02, G13, -p1);
    const double eX = fma(eG, ((dabs(G02) + dabs(G13)) + (dabs(G03) + dabs(G12))) + 2.0 * eG,
                          u2 * fma(dabs(G02), dabs(G13), dabs(p1)));
    const double q1 = G01 * G01;
    const double N1 = fma(G00, G11, -q1);
    const double eN1 = fma(eG, (dabs(G00) + dabs(G11)) + (2.0 * dabs(G01) + 2.0 * eG),
                           u2 * fma(dabs(G00), dabs(G11), q1));
    const double q2 = G23 * G23;
    const double N2 = fma(G22, G33, -q2);
    const double eN2 = fma(eG, (dabs(G22) + dabs(G33)) + (2.0 * dabs(G23) + 2.0 * eG),
                           u2 * fma(dabs(G22), dabs(G33), q2));
    bool ok = (N1 > eN1) && (N2 > eN2);
    const double D = N1 * N2;
    const double eD = fma(N1 + eN1, eN2, fma(N2, eN1, U64 * D));
    ok = ok && (eD <= 0.25 * D);
    double rel;
    const double r = rsqrt_cert(D, rel, ok);
    const double v = X * r;
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
                       fma(dabs(Es), eM, u2 * (dabs(PPs * EP) + dabs(M2 * Es)))));
    const double A = fma(PPs, PPs, -(M2 * dss));
    const double eA = fma(2.0 * dabs(PPs) + ePP, ePP, fma(dabs(M2) + eM, eds,
                      fma(dabs(dss), eM, u2 * (PPs * PPs + dabs(M2 * dss)))));
    const double B = fma(P[3], P[3], fma(P[2], P[2], P[1] * P[1]));
    const double eB = fma(6.1 * U64 * W, W, (3.1 * U64) * B);
    bool ok = (A > eA) && (B > eB);
    const double D = A * B;
    const double eD = fma(A + eA, eB, fma(B, eA, U64 * D));
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
    const double em = (12.4 * U64) * WS * WS;
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
__device__ __forceinline__ int axis_bin(const double (&x)[4][4], const double (&w)[4], double W, double wmax,
                                        const double (&P)[4], double M2, double eM, int nb, int sl,
                                        const double *ed, double glo, double ginv, bool &sure)
{
    constexpr double KDOT = EXACTP ? 3.02 : 4.02;
    if constexpr (KIND == AX_ABSPHI) return bin_absphi(x, W, wmax, M2, KDOT, ed, nb, sure);
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

    // validity: E_P > 0 and M^2 > 0 (|M^2 computed - M^2| <= 10.1 u W^2)
    double w[4], P[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) w[s] = (dabs(x[s][0]) + dabs(x[s][1])) + (dabs(x[s][2]) + dabs(x[s][3]));
    const double W = (w[0] + w[1]) + (w[2] + w[3]);
#pragma unroll
    for (int c = 0; c < 4; ++c) P[c] = (x[0][c] + x[1][c]) + (x[2][c] + x[3][c]);
    const double M2 = fma(-P[3], P[3], fma(-P[2], P[2], fma(-P[1], P[1], P[0] * P[0])));
    const double Emin = fmin(fmin(x[0][0], x[1][0]), fmin(x[2][0], x[3][0]));
    if (!(Emin >= 0.0 && P[0] > 0.0 && M2 > (11.0 * U64) * W * W)) return o;

    // sign of the triple product
    double det;
    bool sure;
    if constexpr (PREC == 1) {
        float det32;
        float qf[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 4; ++c) qf[s][c] = (float)q[s][c];
        sure = det_f32(qf, det32);
        det = (double)det32;
        if (!sure) {
            o.t2 = 1;
            sure = det_f64<EXACTP>(x, det);
        }
    } else {
        sure = det_f64<EXACTP>(x, det);
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
        double wmax = 0.0;
        if constexpr (K0 == AX_ABSPHI || K1 == AX_ABSPHI) wmax = dmax(dmax(w[0], w[1]), dmax(w[2], w[3]));
        bool bsure = true;
        o.why = 3;
        const int j0 = axis_bin<K0, EXACTP>(x, w, W, wmax, P, M2, eM, g.nb0, g.slots0, g.e0, g.glo0, g.ginv0, bsure);
        bool oor = j0 < 0;
        int bin = j0 < 0 ? 0 : j0;
        if constexpr (K1 != AX_NONE) {
            if (bsure) o.why = 4;
            const int j1 = axis_bin<K1, EXACTP>(x, w, W, wmax, P, M2, eM, g.nb1, g.slots1, g.e1, g.glo1,
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

// The event loop of one segment (events [ev0, ev1) of sample s) for one
// binning scheme.
template <typename Tin, int PREC, int MODE, int EPL, int K0, int K1>
__device__ __forceinline__ void run_segment(const KParams &kp, int s, const SegIO &io, const Seg &g,
                                            int64_t ev0, int64_t ev1, uint32_t *myhist, WaveCounts &wc)
{
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    constexpr bool BINNED = MODE == 0 && K0 != AX_NONE;
    // Register double buffer: the next tile's inputs are requested before the
    // current tile is evaluated, so every wave keeps loads in flight.
    constexpr bool PF = EPL <= 2;
    const int64_t step = (int64_t)EPL * nthr;
    Tin qn[EPL][4][4];
    int tgn[EPL];
    if (PF && ev0 < ev1) load_events<Tin, EPL>(io.ptr, io.tag, ev0 + (int64_t)EPL * tid, io.vec, ev1, qn, tgn);
    for (int64_t t0 = ev0; t0 < ev1; t0 += step) {
        const int64_t base = t0 + (int64_t)EPL * tid;
        Tin q[EPL][4][4];
        int tg[EPL];
        if constexpr (PF) {
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                tg[e] = tgn[e];
#pragma unroll
                for (int k = 0; k < 16; ++k) q[e][k >> 2][k & 3] = qn[e][k >> 2][k & 3];
            }
            if (t0 + step < ev1) load_events<Tin, EPL>(io.ptr, io.tag, base + step, io.vec, ev1, qn, tgn);
        } else {
            load_events<Tin, EPL>(io.ptr, io.tag, base, io.vec, ev1, q, tg);
        }
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
}

template <typename Tin, int PREC, int MODE, int EPL>
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

    int64_t vbeg = (int64_t)blockIdx.x * kp.range;
    const int64_t vend = vbeg + kp.range < kp.vtotal ? vbeg + kp.range : kp.vtotal;
    if (vbeg >= vend) return;
    int lo = 0, hi = kp.nsamples - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (kp.samples[mid].vstart <= vbeg) lo = mid;
        else hi = mid - 1;
    }
    for (int s = lo; s < kp.nsamples && vbeg < vend; ++s) {
        const KSample *S = kp.samples + s;
        const int64_t sv0 = S->vstart;
        const int64_t sv1 = s + 1 < kp.nsamples ? kp.samples[s + 1].vstart : kp.vtotal;
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
        const int naxes = MODE == 0 ? S->naxes : 0;
        const int kind0 = naxes > 0 ? S->kind[0] : AX_NONE;
        const int kind1 = naxes > 1 ? S->kind[1] : AX_NONE;
        g.nb0 = S->nbins[0];
        g.nb1 = S->nbins[1];
        g.slots0 = S->slots[0];
        g.slots1 = S->slots[1];
        g.glo0 = S->guess_lo[0];
        g.glo1 = S->guess_lo[1];
        g.ginv0 = S->guess_inv[0];
        g.ginv1 = S->guess_inv[1];
        const int nd0 = naxes > 0 ? edge_doubles(kind0, g.nb0) : 0;
        const int nd1 = naxes > 1 ? edge_doubles(kind1, g.nb1) : 0;
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
#define TP_SEG(A, B) run_segment<Tin, PREC, MODE, EPL, A, B>(kp, s, io, g, ev0, ev1, myhist, wc)
        if constexpr (MODE == 1) {
            TP_SEG(AX_NONE, AX_NONE);
        } else {
            switch (kind0 * 4 + kind1) {
            case AX_ABSPHI * 4 + AX_NONE: TP_SEG(AX_ABSPHI, AX_NONE); break;
            case AX_MASS * 4 + AX_NONE: TP_SEG(AX_MASS, AX_NONE); break;
            case AX_ABSCOS * 4 + AX_NONE: TP_SEG(AX_ABSCOS, AX_NONE); break;
            case AX_ABSPHI * 4 + AX_MASS: TP_SEG(AX_ABSPHI, AX_MASS); break;
            case AX_ABSPHI * 4 + AX_ABSCOS: TP_SEG(AX_ABSPHI, AX_ABSCOS); break;
            case AX_MASS * 4 + AX_ABSPHI: TP_SEG(AX_MASS, AX_ABSPHI); break;
            case AX_MASS * 4 + AX_MASS: TP_SEG(AX_MASS, AX_MASS); break;
            case AX_MASS * 4 + AX_ABSCOS: TP_SEG(AX_MASS, AX_ABSCOS); break;
            case AX_ABSCOS * 4 + AX_ABSPHI: TP_SEG(AX_ABSCOS, AX_ABSPHI); break;
            case AX_ABSCOS * 4 + AX_MASS: TP_SEG(AX_ABSCOS, AX_MASS); break;
            case AX_ABSCOS * 4 + AX_ABSCOS: TP_SEG(AX_ABSCOS, AX_ABSCOS); break;
            default: TP_SEG(AX_NONE, AX_NONE); break;
            }
        }
#undef TP_SEG
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
template <typename T, int P, int M>
void launch_epl(int epl, const KParams &kp, int grid, int block, size_t lds, hipStream_t st)
{
    if constexpr (sizeof(T) == 4) {
        if (epl >= 4) {
            hipLaunchKernelGGL((tp_pass_kernel<T, P, M, 4>), dim3(grid), dim3(block), lds, st, kp);
            return;
        }
    }
    if (epl >= 2) hipLaunchKernelGGL((tp_pass_kernel<T, P, M, 2>), dim3(grid), dim3(block), lds, st, kp);
    else hipLaunchKernelGGL((tp_pass_kernel<T, P, M, 1>), dim3(grid), dim3(block), lds, st, kp);
}
}  // namespace

hipError_t launch_pass(int dtype, int prec, int mode, int epl, const KParams &kp, int grid, int block,
                       size_t lds, hipStream_t st)
{
    if (dtype == 0) {
        if (prec == 1) {
            if (mode == 0) launch_epl<float, 1, 0>(epl, kp, grid, block, lds, st);
            else launch_epl<float, 1, 1>(epl, kp, grid, block, lds, st);
        } else {
            if (mode == 0) launch_epl<float, 0, 0>(epl, kp, grid, block, lds, st);
            else launch_epl<float, 0, 1>(epl, kp, grid, block, lds, st);
        }
    } else {
        if (mode == 0) launch_epl<double, 0, 0>(epl, kp, grid, block, lds, st);
        else launch_epl<double, 0, 1>(epl, kp, grid, block, lds, st);
    }
    return hipGetLastError();
}

}  // namespace tpk
