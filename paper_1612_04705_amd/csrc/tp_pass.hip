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
    int why;      // deferred at: 1 validity, 2 sign, 3 first axis, 4 second axis, 5 order,
                  // 6 first pass (eval_lean)
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
// Sm > 0: a bound S <= Sm supplied by the caller (the product of the two
// minors' L1 norms bounds S); otherwise S is formed here.
template <bool EXACT_PRODUCTS>
__device__ __forceinline__ bool det_f64(const double (&m01)[6], const double (&m23)[6], double &det,
                                        double Sm = 0.0)
{
    double s = m01[0] * m23[5];
    s = fma(-m01[1], m23[4], s);
    s = fma(m01[2], m23[3], s);
    s = fma(m01[3], m23[2], s);
    s = fma(-m01[4], m23[1], s);
    s = fma(m01[5], m23[0], s);
    double S = Sm;
    if (!(Sm > 0.0)) {
        S = dabs(m01[0]) * dabs(m23[5]);
#pragma unroll
        for (int k = 1; k < 6; ++k) S = fma(dabs(m01[k]), dabs(m23[5 - k]), S);
    }
    const double bound = EXACT_PRODUCTS ? (10.0 * U64) * S : fma(12.0 * U64, S, 0x1p-160);
    det = s;
    return dabs(s) > bound;
}

__device__ __forceinline__ bool det_f32(const float x[4][4], float &det, float *bound_out = nullptr)
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
    if (bound_out) *bound_out = bound;
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

// Counts over the inner edges e[1..n-1] (LDS) for the two ends of an
// interval, in one pass: LE = true counts x <= e[k], LE = false counts
// e[k] <= x.  A bin is certified when both ends give the same count (no edge
// falls inside the interval).  Branch-free body, unrolled by four.
template <bool LE>
__device__ __forceinline__ void count_edges(double xa, double xb, const double *e, int n, int &ca, int &cb)
{
    int a = 0, b = 0;
    int k = 1;
    for (; k + 3 < n; k += 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double c = e[k + i];
            a += LE ? (xa <= c) : (c <= xa);
            b += LE ? (xb <= c) : (c <= xb);
        }
    }
    for (; k < n; ++k) {
        const double c = e[k];
        a += LE ? (xa <= c) : (c <= xa);
        b += LE ? (xb <= c) : (c <= xb);
    }
    ca = a;
    cb = b;
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

__device__ __forceinline__ double l1norm6(const double (&m)[6])
{
    return ((dabs(m[0]) + dabs(m[1])) + (dabs(m[2]) + dabs(m[3]))) + (dabs(m[4]) + dabs(m[5]));
}

// M1, M2s: L1 norms of m01, m23
__device__ __forceinline__ int bin_absphi_bv(const double (&m01)[6], const double (&m23)[6], double M1, double M2s,
                                             const double (&P)[4], double W, const double *edges, int n, bool &sure)
{
    double C1[4], C2[4];
    covector(P, m01, C1);
    covector(P, m23, C2);
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
    // bin = #{k : cos Phi <= c_k}: certified when vhi and vlo pass the same edges
    int bin, blo;
    count_edges<true>(v + eps, v - eps, edges, n, bin, blo);
    sure = sure && ok && bin == blo;
    return bin;
}

// |cos theta| of kernel slot s against the M flight direction:
// Nn = (P.p_s) E_P - M^2 E_s, A = G_ss, B = |P_lab|^2, |cos| = |Nn| / sqrt(A B).
// edges 0 = e_0 < ... < e_n = 1; returns #{k in 1..n-1 : |cos| >= e_k}.
// SLOT0: the slot is kernel slot 0 (the host relabels the slots so), else s.
template <bool SLOT0>
__device__ __forceinline__ int bin_abscos(const double x[4][4], const double w[4], double W,
                                          const double P[4], double M2, int s, const double *edges, int n,
                                          bool &sure)
{
    double xs[4];
    double ws = w[0];
#pragma unroll
    for (int c = 0; c < 4; ++c) xs[c] = x[0][c];
    if (!SLOT0) {
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
    }
    // Bounds from magnitudes (W = L1 norm of all components, w_s of slot s;
    // |P_c| <= W, |P.p_s| <= W w_s, |M^2| <= W^2, |p_s.p_s| <= w_s^2):
    //   |P.p_s^ - P.p_s| <= (4.01 + 2.01) u W w_s (four roundings, P's error),
    //   |E_P^ - E_P| <= 2.01 u W, |M^2^ - M^2| <= 10.2 u W^2,
    //   |d_ss^ - d_ss| <= 4.02 u w_s^2, so with the roundings of the fused steps
    //   |Nn^ - Nn| <= (2.01 + 6.02 + 10.2 + 3) u W^2 w_s   <= 24 u W^2 w_s,
    //   |A^ - A|   <= (12.04 + 4.02 + 10.2 + 3) u W^2 w_s^2 <= 32 u W^2 w_s^2,
    //   |B^ - B|   <= (4.02 + 3.01) u W^2 (+ slack)         <= 10 u W^2.
    const double PPs = mink(P, xs);
    const double Es = xs[0];
    const double dss = mink(xs, xs);
    const double Nn = fma(PPs, P[0], -(M2 * Es));
    const double A = fma(PPs, PPs, -(M2 * dss));
    const double B = fma(P[3], P[3], fma(P[2], P[2], P[1] * P[1]));
    const double WW = W * W;
    const double Q = WW * ws;
    const double eNn = fma(24.0 * U64, Q, TINY);
    const double eA = fma((32.0 * U64) * Q, ws, TINY);
    const double eB = fma(10.0 * U64, WW, TINY);
    bool ok = (A > eA) && (B > eB);
    const double D = A * B;
    const double eD = fma(A + eA, eB, fma(B, eA, fma(U64, D, TINY)));
    ok = ok && (eD <= 0.25 * D);
    double rel;
    const double r = rsqrt_cert(D, rel, ok);
    const double v = dabs(Nn) * r;
    const double eps = ratio_eps(v, r, rel, eNn, eD);
    // bin = #{k : |cos| >= e_k}: certified when vlo and vhi pass the same edges
    int bin, bhi;
    count_edges<false>(v - eps, v + eps, edges, n, bin, bhi);
    sure = sure && ok && bin == bhi;
    return bin;
}

// Invariant mass of the kernel slots in ``mask``.  ed: [sq_lo(n+1) | sq_hi(n+1)]
// with sq_lo_k <= e_k^2 <= sq_hi_k.  Returns the bin or -1 (out of range).
__device__ __forceinline__ int bin_mass(const double x[4][4], const double w[4], int mask,
                                        const double *ed, int n, double glo, double ginv, bool &sure)
{
    // sum of the slots in the mask with 0/1 weights: b x is exact, so every
    // fused step rounds at most once and only where a slot is added
    const double b0 = (mask & 1) ? 1.0 : 0.0, b1 = (mask & 2) ? 1.0 : 0.0;
    const double b2 = (mask & 4) ? 1.0 : 0.0, b3 = (mask & 8) ? 1.0 : 0.0;
    double S[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) S[c] = fma(b3, x[3][c], fma(b2, x[2][c], fma(b1, x[1][c], b0 * x[0][c])));
    const double WS = fma(b3, w[3], fma(b2, w[2], fma(b1, w[1], b0 * w[0])));
    const double m2 = fma(-S[3], S[3], fma(-S[2], S[2], fma(-S[1], S[1], S[0] * S[0])));
    const double em = fma((12.4 * U64) * WS, WS, TINY);
    const double *sqlo = ed, *sqhi = ed + (n + 1);
    const double mlo = m2 - em, mhi = m2 + em;
    // guess on a uniform grid in m (hardware square root: only a guess), then
    // certify against the two neighbouring edges
    const float mg = __builtin_amdgcn_sqrtf(fmaxf((float)m2, 0.0f));
    const float t = (mg - (float)glo) * (float)ginv;
    const int j = (int)fminf(fmaxf(t, 0.0f), (float)(n - 1));
    // bin j when e_j^2 <= m^2 and m^2 < e_(j+1)^2 (<= for the last, closed bin)
    const double ehi = sqlo[j + 1];
    if (mlo >= sqhi[j] && (mhi < ehi || (j == n - 1 && mhi <= ehi))) return j;
    // full scan
    if (mhi < sqlo[0] || mlo > sqhi[n]) return -1;          // certainly outside
    if (!(mlo >= sqhi[0] && mhi <= sqlo[n])) {               // not certainly inside
        sure = false;
        return -1;
    }
    // bin = #{k : m^2 >= e_k^2}: certified when mlo and mhi pass the same edges
    int bin = 0, bhi = 0;
    for (int k = 1; k < n; ++k) {
        bin += mlo >= sqhi[k];
        bhi += mhi >= sqlo[k];
    }
    sure = sure && bin == bhi;
    return bin;
}

struct Seg {
    int32_t sigma, nb0, nb1, nbtot, slots0, slots1, olo, odir;
    double glo0, ginv0, glo1, ginv1;
    const double *e0, *e1;    // LDS edge data of each axis
};

// One axis of compile-time kind KIND: bin index, or -1 (out of range).
template <int KIND, bool EXACTP, bool SLOT0>
__device__ __forceinline__ int axis_bin(const double (&x)[4][4], const double (&w)[4], double W,
                                        const double (&m01)[6], const double (&m23)[6], double M1, double M2s,
                                        const double (&P)[4], double M2, int nb, int sl,
                                        const double *ed, double glo, double ginv, bool &sure)
{
    if constexpr (KIND == AX_ABSPHI) return bin_absphi_bv(m01, m23, M1, M2s, P, W, ed, nb, sure);
    else if constexpr (KIND == AX_MASS) return bin_mass(x, w, sl, ed, nb, glo, ginv, sure);
    else return bin_abscos<SLOT0>(x, w, W, P, M2, sl, ed, nb, sure);
}

// Canonical order of two identical particles in kernel slots LO and LO + 2:
// the one with the larger energy in the M rest frame, i.e. the larger P.p
// (= M E*), belongs in the channel's "fast" slot (dir = +1: slot LO).  With
// d = p_LO - p_HI and s = P.d (Minkowski), every rounding is bounded on
// magnitudes: P_c sums four components (2u of sum_s |x_sc|), d_c one
// difference (u |d_c|), the four-term product 4u; in all
// |s_computed - s| <= 8u sum_c (sum_s |x_sc|)(|x_LO,c| + |x_HI,c|)
//                   <= 8u W (w_LO + w_HI),
// taken as 8.1u with the bound's own roundings.  A decided event has its rows
// (and row norms) exchanged when the slow one is stored first; an undecided
// one -- including an exact tie, which keeps the stored order -- goes to the
// exact tier.
template <int LO>
__device__ __forceinline__ bool order_pair(double (&x)[4][4], double (&w)[4], const double (&P)[4], double W, int dir)
{
    constexpr int HI = LO + 2;
    double d[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) d[c] = x[LO][c] - x[HI][c];
    const double s = fma(-P[3], d[3], fma(-P[2], d[2], fma(-P[1], d[1], P[0] * d[0])));
    const double bound = fma((8.1 * U64) * W, w[LO] + w[HI], TINY);
    if (!(dabs(s) > bound)) return false;
    const bool sw = (dir > 0) ? (s < 0.0) : (s > 0.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double a = x[LO][c], b = x[HI][c];
        x[LO][c] = sw ? b : a;
        x[HI][c] = sw ? a : b;
    }
    const double a = w[LO], b = w[HI];
    w[LO] = sw ? b : a;
    w[HI] = sw ? a : b;
    return true;
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

    if (g.olo >= 0) {   // uniform: identical particles to be ordered
        o.why = 5;
        const bool ok = g.olo == 0 ? order_pair<0>(x, w, P, W, g.odir) : order_pair<1>(x, w, P, W, g.odir);
        if (!ok) return o;
    }

    // Sign of the triple product.  The plane-angle bins need the float64
    // minors (the bivectors p0^p1, p2^p3) anyway, and the determinant from them
    // costs a dozen operations, less than the float32 contraction: so the
    // float32 sign with float64 recheck runs only when no plane angle is binned.
    constexpr bool NEED_BV = K0 == AX_ABSPHI || K1 == AX_ABSPHI;
    constexpr bool F32_SIGN = PREC == 1 && !NEED_BV;
    double m01[6], m23[6];
    double M1 = 0.0, M2s = 0.0;
    double det;
    bool sure;
    if constexpr (F32_SIGN) {
        float det32;
        float qf[4][4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 4; ++c) qf[s][c] = (float)x[s][c];   // x holds q exactly (rows possibly ordered)
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
        if constexpr (NEED_BV) {
            M1 = l1norm6(m01);
            M2s = l1norm6(m23);
            sure = det_f64<EXACTP>(m01, m23, det, M1 * M2s);
        } else {
            sure = det_f64<EXACTP>(m01, m23, det);
        }
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
        bool bsure = true;
        o.why = 3;
        // the first |cos theta| axis reads kernel slot 0 (host relabelling)
        const int j0 = axis_bin<K0, EXACTP, true>(x, w, W, m01, m23, M1, M2s, P, M2, g.nb0, g.slots0, g.e0, g.glo0, g.ginv0,
                                            bsure);
        bool oor = j0 < 0;
        int bin = j0 < 0 ? 0 : j0;
        if constexpr (K1 != AX_NONE) {
            if (bsure) o.why = 4;
            const int j1 = axis_bin<K1, EXACTP, K0 != AX_ABSCOS>(x, w, W, m01, m23, M1, M2s, P, M2, g.nb1, g.slots1, g.e1, g.glo1,
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

// ------------------------------------------------------------ first pass
// A lean evaluation of one event for float32 storage and a binning scheme
// with a plane angle: the same quantities as eval_event (validity, minors,
// sign, covectors, |cos theta| invariants, mass), computed branch-free, with
// the error of each angle bounded by one combined expression.  Every
// decision it returns is certified; ``ok`` is false where a bound does not
// settle one, or where an input lies outside the ranges the bounds assume,
// and the event then goes to the later tiers (double-word, exact integers).
//
// Ranges: with float32 inputs every exact intermediate of degree k in the
// components is a multiple of 2^(-149 k), so nothing below degree 7 falls into
// the subnormal range; W <= 2^64 keeps every intermediate finite, and the
// degree-12 product D of the plane angle is required to be >= 2^-1000.  The
// factor (1 +- eps_1)(1 +- eps_2) of D is taken to first order with the
// constant 0.574 = (1 - sqrt(3/4)) / (1/4) * 1.07, valid for eps_1 + eps_2 <= 1/8.
//
// Plane angle (notation of bin_absphi_bv): with the term-by-term bounds eX,
// eS_i of the full evaluation, eps_i = eS_i/|S_i^| with eps_1 + eps_2 <= 1/8
// (so |sqrt(S1 S2 / D^) - 1| <= 0.574 (eps_1 + eps_2) + u) and the certified
// reciprocal square root r (|r sqrt(D^) - 1| <= rel), the true
// cos Phi = -X / sqrt(S1 S2) (|cos Phi| <= 1: the C_i lie in the space-like
// complement of P) satisfies
//   |v^ - cos Phi| <= eX r + rel + 0.575 (eps_1 + eps_2) + 1.6 u,
// and eps_1 + eps_2 <= 1.0001 r^2 (eS1 |S2^| + eS2 |S1^|); evaluated with the
// constant 0.58 and 4 u (roundings of the bound itself and of v^ +- eps), and
// required to be at most 1/16 (which keeps eps_1 + eps_2 below 1/8).  This
// replaces the separate bound on D and the ratio's error terms of the full
// evaluation by one expression.
//
// |cos theta|: with the magnitude bounds of bin_abscos (24, 32, 10 u W^2 ...)
// and the same steps, using 24 w_s/sqrt(A B) <= 0.672 (32 w_s^2/A + 10/B),
//   |v^ - |cos theta|| <= 1.246 u W^2 (32 w_s^2 B + 10 A) r^2 + rel + 1.6 u,
// evaluated as u W^2 (40 w_s^2 B + 13 A) r^2 + rel + 4 u, at most 1/16.
//
// A bin is certified when v^ - eps and v^ + eps pass the same edges.
__device__ __forceinline__ double rsqrt_lean(double D, double &rel, bool &ok)
{
    const double r0 = __builtin_amdgcn_rsq(D);
    const double t = D * r0;
    const double rho = fma(-t, r0, 1.0);
    const double r = fma(0.5 * r0, rho, r0);
    ok = ok && (dabs(rho) <= 0x1p-10) && (D >= 0x1p-1000);
    rel = fma(0.5 * rho, rho, 3.0 * U64);
    return r;
}

// cos|Phi| bin: #{k in 1..n-1 : cos Phi <= c_k}
__device__ __forceinline__ int absphi_lean(const double (&m01)[6], const double (&m23)[6], double M1, double M2s,
                                           const double (&P)[4], double W, const double *e, int n, bool &ok)
{
    double C1[4], C2[4];
    covector(P, m01, C1);
    covector(P, m23, C2);
    const double X = fma(-C1[3], C2[3], fma(-C1[2], C2[2], fma(-C1[1], C2[1], C1[0] * C2[0])));
    const double S1 = fma(-C1[3], C1[3], fma(-C1[2], C1[2], fma(-C1[1], C1[1], C1[0] * C1[0])));
    const double S2 = fma(-C2[3], C2[3], fma(-C2[2], C2[2], fma(-C2[1], C2[1], C2[0] * C2[0])));
    const double D = S1 * S2;
    double rel;
    bool good = (S1 < 0.0) && (S2 < 0.0);
    const double r = rsqrt_lean(D, rel, good);
    const double v = -X * r;
    // term-by-term bounds of bin_absphi_bv
    const double A1 = (dabs(C1[0]) + dabs(C1[1])) + (dabs(C1[2]) + dabs(C1[3]));
    const double A2 = (dabs(C2[0]) + dabs(C2[1])) + (dabs(C2[2]) + dabs(C2[3]));
    const double k = (7.2 * U64) * W;
    const double eC1 = fma(k, M1, TINY), eC2 = fma(k, M2s, TINY);
    const double uA1 = (4.02 * U64) * A1, uA2 = (4.02 * U64) * A2;
    const double eX = fma(eC2, A1, fma(eC1, A2, fma(4.0 * eC1, eC2, uA1 * A2)));
    const double eS1 = fma(2.0 * eC1, A1, fma(4.0 * eC1, eC1, uA1 * A1));
    const double eS2 = fma(2.0 * eC2, A2, fma(4.0 * eC2, eC2, uA2 * A2));
    // eps_1 + eps_2 = eS1/|S1| + eS2/|S2| <= 1.0001 r^2 (eS1 |S2| + eS2 |S1|)
    const double q = fma(eS1, -S2, eS2 * -S1);
    const double eps = fma(eX, r, fma(0.58 * (r * r), q, rel + 4.0 * U64));
    good = good && (eps <= 0.0625);
    // bin = #{k : cos Phi <= c_k}: certified when both ends pass the same edges
    int j, jlo;
    count_edges<true>(v + eps, v - eps, e, n, j, jlo);
    ok = ok && good && j == jlo;
    return j;
}

// |cos theta| bin of kernel slot 0: #{k in 1..n-1 : |cos| >= e_k}
__device__ __forceinline__ int abscos_lean(const double (&x)[4][4], double w0, const double (&P)[4], double M2,
                                           double WW, const double *e, int n, bool &ok)
{
    const double PPs = mink(P, x[0]);
    const double dss = mink(x[0], x[0]);
    const double Nn = fma(PPs, P[0], -(M2 * x[0][0]));
    const double A = fma(PPs, PPs, -(M2 * dss));
    const double B = fma(P[3], P[3], fma(P[2], P[2], P[1] * P[1]));
    bool good = (A > 0.0) && (B > 0.0);
    double rel;
    const double r = rsqrt_lean(A * B, rel, good);
    const double v = dabs(Nn) * r;
    const double T = (r * r) * fma((40.0 * w0) * w0, B, 13.0 * A);
    const double eps = fma(U64 * WW, T, rel + 4.0 * U64);
    good = good && (eps <= 0.0625);
    // bin = #{k : |cos| >= e_k}: certified when both ends pass the same edges
    int j, jhi;
    count_edges<false>(v - eps, v + eps, e, n, j, jhi);
    ok = ok && good && j == jhi;
    return j;
}

template <int KIND>
__device__ __forceinline__ int axis_lean(const double (&x)[4][4], const double (&w)[4], double WW,
                                         const double *, const double *, double, double, const double (&P)[4],
                                         double M2, int nb, int sl, const double *ed, double glo, double ginv,
                                         bool &ok)
{
    static_assert(KIND == AX_MASS, "mass axis only");
    (void)WW;
    (void)P;
    (void)M2;
    bool sure = true;
    const int j = bin_mass(x, w, sl, ed, nb, glo, ginv, sure);
    ok = ok && sure;
    return j;
}

// The first pass over one float32 event.  On ok: cls (CLS_I .. CLS_IV) and
// bin (-1: outside the binned range).  The axes that read the components
// (mass, |cos theta|) are evaluated before the minors so that the components
// are no longer live during the plane angle.
template <int K0, int K1, bool ORD>
__device__ __forceinline__ void eval_lean(const float (&q)[4][4], int tag, const Seg &g, int &cls, int &bin,
                                          bool &ok)
{
    double x[4][4];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 4; ++c) x[s][c] = (double)q[s][c];
    double w[4], P[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) w[s] = (dabs(x[s][0]) + dabs(x[s][1])) + (dabs(x[s][2]) + dabs(x[s][3]));
    const double W = (w[0] + w[1]) + (w[2] + w[3]);
#pragma unroll
    for (int c = 0; c < 4; ++c) P[c] = (x[0][c] + x[1][c]) + (x[2][c] + x[3][c]);
    const double M2 = fma(-P[3], P[3], fma(-P[2], P[2], fma(-P[1], P[1], P[0] * P[0])));
    const double WW = W * W;
    // validity as in eval_event, and the range the bounds assume
    const bool epos = (x[0][0] >= 0.0) & (x[1][0] >= 0.0) & (x[2][0] >= 0.0) & (x[3][0] >= 0.0);
    ok = (tag == 0 || tag == 1) && epos && P[0] > 0.0 && M2 > fma(11.0 * U64, WW, TINY) && W <= 0x1p64;
    if constexpr (ORD) {   // identical particles to be ordered (every sample of the launch)
        const bool o = g.olo == 0 ? order_pair<0>(x, w, P, W, g.odir) : order_pair<1>(x, w, P, W, g.odir);
        ok = ok && o;
    }
    int j0 = 0, j1 = 0;
    if constexpr (K0 == AX_MASS) j0 = axis_lean<K0>(x, w, WW, nullptr, nullptr, 0, 0, P, M2, g.nb0, g.slots0, g.e0,
                                                    g.glo0, g.ginv0, ok);
    if constexpr (K1 == AX_MASS) j1 = axis_lean<K1>(x, w, WW, nullptr, nullptr, 0, 0, P, M2, g.nb1, g.slots1, g.e1,
                                                    g.glo1, g.ginv1, ok);
    if constexpr (K0 == AX_ABSCOS) j0 = abscos_lean(x, w[0], P, M2, WW, g.e0, g.nb0, ok);
    if constexpr (K1 == AX_ABSCOS) j1 = abscos_lean(x, w[0], P, M2, WW, g.e1, g.nb1, ok);
    double m01[6], m23[6];
    minors_f64<true>(x[0], x[1], m01);
    minors_f64<true>(x[2], x[3], m23);
    const double M1 = l1norm6(m01), M2s = l1norm6(m23);
    // Laplace sum of det_f64 with its bound from the product of the minors' norms
    double det = m01[0] * m23[5];
    det = fma(-m01[1], m23[4], det);
    det = fma(m01[2], m23[3], det);
    det = fma(m01[3], m23[2], det);
    det = fma(-m01[4], m23[1], det);
    det = fma(m01[5], m23[0], det);
    ok = ok && (dabs(det) > (10.0 * U64) * (M1 * M2s));
    const double ct = g.sigma > 0 ? det : -det;
    cls = tag == 0 ? (ct > 0.0 ? CLS_I : CLS_II) : (ct < 0.0 ? CLS_III : CLS_IV);
    if constexpr (K0 == AX_ABSPHI) j0 = absphi_lean(m01, m23, M1, M2s, P, W, g.e0, g.nb0, ok);
    if constexpr (K1 == AX_ABSPHI) j1 = absphi_lean(m01, m23, M1, M2s, P, W, g.e1, g.nb1, ok);
    bool oor = j0 < 0;
    int b = j0 < 0 ? 0 : j0;
    if constexpr (K1 != AX_NONE) {
        oor = oor || j1 < 0;
        b = b * g.nb1 + (j1 < 0 ? 0 : j1);
    }
    bin = oor ? -1 : b;
}

__device__ __forceinline__ uint32_t wave_count(bool p)
{
    return (uint32_t)__popcll(__ballot(p));
}

// Nontemporal load of element i (32-bit index) from a uniform base pointer:
// the byte offset is formed in 32 bits so the load takes the scalar-base +
// vector-offset addressing form.
template <typename T>
__device__ __forceinline__ T ldnt(const void *base, uint32_t i)
{
    typedef const T __attribute__((address_space(1))) *gptr;
    const uint32_t byte = i * (uint32_t)sizeof(T);
    return __builtin_nontemporal_load((gptr)((const char *)base + byte));
}

typedef const __attribute__((address_space(4))) KSample *ctab;

// Load EPL consecutive events per lane, the lane's first at segment offset
// ``off``, from the 16 component arrays and the tag array.  Every offset is
// clamped to ``last`` (the segment's last event), so every load stays in
// bounds and none is predicated.
template <typename Tin, int EPL>
__device__ __forceinline__ void load_scalar(ctab S, int64_t ev0, uint32_t off, uint32_t last,
                                            Tin (&q)[EPL][4][4], int (&tg)[EPL])
{
    // The table pointer is passed through an empty asm, so the compiler cannot
    // hoist the scalar loads of the 16 array pointers out of the tile loop:
    // they are re-read (scalar cache) per tile and occupy SGPRs only while the
    // tile's loads issue.
    asm volatile("" : "+s"(S));
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        // index from the array base: below 2^32 bytes (the host splits larger samples)
        const uint32_t o = (uint32_t)ev0 + (off + e < last ? off + e : last);
#pragma unroll
        for (int k = 0; k < 16; ++k) q[e][k >> 2][k & 3] = ldnt<Tin>(S->p[k], o);
        tg[e] = (int)ldnt<int8_t>(S->tag, o);
    }
}

// The same for a tile lying wholly inside the segment, with 8- or 16-byte
// vector loads (arrays 16-byte aligned, ``off`` a multiple of EPL).
template <typename Tin, int EPL>
__device__ __forceinline__ void load_vector(ctab S, int64_t ev0, uint32_t off, Tin (&q)[EPL][4][4],
                                            int (&tg)[EPL])
{
    constexpr int BYTES = EPL * (int)sizeof(Tin);
    asm volatile("" : "+s"(S));
    const void *tag = S->tag;
    off += (uint32_t)ev0;   // from the array base (ev0 is a multiple of 256)
    if constexpr (BYTES == 8) {
        typedef Tin v2 __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const v2 v = ldnt<v2>(S->p[k], off >> 1);
            q[0][k >> 2][k & 3] = v.x;
            q[1][k >> 2][k & 3] = v.y;
        }
        const uint16_t t = ldnt<uint16_t>(tag, off >> 1);
        tg[0] = (int)(int8_t)(t & 0xff);
        tg[1] = (int)(int8_t)(t >> 8);
    } else if constexpr (EPL == 4 && sizeof(Tin) == 4) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const f32x4 v = ldnt<f32x4>(S->p[k], off >> 2);
            q[0][k >> 2][k & 3] = v.x;
            q[1][k >> 2][k & 3] = v.y;
            q[2][k >> 2][k & 3] = v.z;
            q[3][k >> 2][k & 3] = v.w;
        }
        const uint32_t t = ldnt<uint32_t>(tag, off >> 2);
#pragma unroll
        for (int e = 0; e < 4; ++e) tg[e] = (int)(int8_t)(t >> (8 * e));
    } else if constexpr (EPL == 2) {   // double: 16-byte loads
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const f64x2 v = ldnt<f64x2>(S->p[k], off >> 1);
            q[0][k >> 2][k & 3] = v.x;
            q[1][k >> 2][k & 3] = v.y;
        }
        const uint16_t t = ldnt<uint16_t>(tag, off >> 1);
        tg[0] = (int)(int8_t)(t & 0xff);
        tg[1] = (int)(int8_t)(t >> 8);
    }
}

// Class totals of a wave's events, for the schemes without bins (binned
// schemes derive them from the histogram).
struct WaveCounts {
    uint32_t c0, c1, c2, c3;
};

struct SegIO {
    ctab S;                   // this sample's table entry
    int8_t *cls_out;
    double *ct_out;
    bool vec;
};

// LDS layout of one histogram copy: rows 0 .. nbtot + 1 of four class
// counters (row 0 class totals, rows 1 .. nbtot the bins, row nbtot + 1 the
// events outside every bin), then NSTAT statistics words.
__device__ __forceinline__ int lds_stats(int nbtot) { return (nbtot + 2) * 4; }

// Whether binned float32 passes with a plane angle take the first pass
// (eval_lean) before the full evaluation.
template <typename Tin, int MODE, int K0, int K1>
constexpr bool lean_pass()
{
    return MODE == 0 && sizeof(Tin) == 4 && (K0 == AX_ABSPHI || K1 == AX_ABSPHI);
}

// One tile: EPL consecutive events per lane, the lane's first at segment
// offset ``loc``; ``len`` events in the segment, which starts at event ev0.
template <typename Tin, int PREC, int MODE, int EPL, int K0, int K1, bool ORD>
__device__ __forceinline__ void process_tile(const KParams &kp, int s, const SegIO &io, const Seg &g,
                                             const Tin (&q)[EPL][4][4], const int (&tg)[EPL], uint32_t loc,
                                             uint32_t len, int64_t ev0, uint32_t *myhist, int srow,
                                             WaveCounts &wc)
{
    constexpr bool BINNED = MODE == 0 && K0 != AX_NONE;
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
        const uint32_t li = loc + e;
        const bool in = li < len;
        EvOut o;
        bool done = false;
        if constexpr (lean_pass<Tin, MODE, K0, K1>()) {
            {
                // first pass; the rare events it does not settle go to the
                // later tiers
                int lc = 0, lb = 0;
                bool ok;
                eval_lean<K0, K1, ORD>(q[e], tg[e], g, lc, lb, ok);
                const bool badtag = tg[e] != 0 && tg[e] != 1;
                o.cls = !in ? -1 : badtag ? CLS_INVALID : ok ? lc : CLS_DEFER;
                o.bin = in ? lb : -1;
                o.t2 = 0;
                o.why = 6;
                o.ct = 0.0;
                done = true;
            }
        }
        if (done) {
        } else if (in) {
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
                kp.xlist[slot] = ((uint64_t)o.why << 60) | ((uint64_t)s << 40) | (uint64_t)(ev0 + li);
                listed = true;
            } else {
                unres = true;
            }
        }
        if (MODE == 1 && in) {
            io.cls_out[ev0 + li] = (int8_t)(unres ? CLS_UNRESOLVED : o.cls);
            if (io.ct_out) io.ct_out[ev0 + li] = o.ct;
        }
        const bool classified = o.cls >= 0 && o.cls < 4;
        if constexpr (BINNED) {
            // out-of-range events go to the overflow row
            const int row = 1 + (o.bin >= 0 ? o.bin : g.nbtot);
            if (classified) atomicAdd(&myhist[row * 4 + o.cls], 1u);
        } else if constexpr (MODE == 0) {
            wc.c0 += wave_count(o.cls == CLS_I);
            wc.c1 += wave_count(o.cls == CLS_II);
            wc.c2 += wave_count(o.cls == CLS_III);
            wc.c3 += wave_count(o.cls == CLS_IV);
        }
        // rare outcomes: one ballot decides whether the wave counts them
        const bool rare = (o.cls >= CLS_ZERO) || o.t2;
        if (__ballot(rare)) {
            const uint32_t nz = wave_count(o.cls == CLS_ZERO);
            const uint32_t ni = wave_count(o.cls == CLS_INVALID);
            const uint32_t n2 = wave_count(o.t2 != 0);
            const uint32_t n3 = wave_count(listed);
            const uint32_t nu = wave_count(unres);
            if ((threadIdx.x & 63) == 0) {
                if (nz) atomicAdd(&myhist[srow + ST_ZERO], nz);
                if (ni) atomicAdd(&myhist[srow + ST_INVALID], ni);
                if (n2) atomicAdd(&myhist[srow + ST_TIER2], n2);
                if (n3) atomicAdd(&myhist[srow + ST_TIER3], n3);
                if (nu) atomicAdd(&myhist[srow + ST_UNRESOLVED], nu);
            }
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

// The event loop of one segment: ``len`` events of sample s from event ev0,
// addressed by 32-bit offsets (the host caps a workgroup's range).
template <typename Tin, int PREC, int MODE, int EPL, int K0, int K1, bool ORD>
__device__ __forceinline__ void run_segment(const KParams &kp, int s, const SegIO &io, const Seg &g,
                                            int64_t ev0, uint32_t len, uint32_t *myhist, int srow,
                                            WaveCounts &wc)
{
    const uint32_t lane0 = (uint32_t)EPL * threadIdx.x;
    const uint32_t step = (uint32_t)EPL * blockDim.x;
    const uint32_t last = len - 1;
    constexpr bool PF = prefetch_tiles<Tin, EPL, K0, K1>();
    if constexpr (EPL == 1) {
        // every tile takes the same (clamped) loads; tile t is evaluated while
        // tile t + 1 loads into the other register set.  The loads issue
        // unconditionally (past the end they re-read the last event), so no
        // branch merges ahead of an evaluation and its wait covers only the
        // tile being evaluated.
        Tin qa[1][4][4], qb[1][4][4];
        int ta[1], tb[1];
        load_scalar<Tin, 1>(io.S, ev0, lane0, last, qa, ta);
        for (uint32_t t0 = 0; t0 < len; t0 += 2 * step) {
            const uint32_t t1 = t0 + step;
            load_scalar<Tin, 1>(io.S, ev0, t1 + lane0, last, qb, tb);
            process_tile<Tin, PREC, MODE, 1, K0, K1, ORD>(kp, s, io, g, qa, ta, t0 + lane0, len, ev0, myhist, srow, wc);
            if (t1 >= len) break;
            load_scalar<Tin, 1>(io.S, ev0, t1 + step + lane0, last, qa, ta);
            process_tile<Tin, PREC, MODE, 1, K0, K1, ORD>(kp, s, io, g, qb, tb, t1 + lane0, len, ev0, myhist, srow, wc);
        }
        return;
    }
    // EPL > 1: tiles wholly inside the segment take vector loads (aligned
    // arrays), the partial tail tile (or everything, unaligned) scalar ones
    const uint32_t nfull = io.vec ? len / step : 0;
    if constexpr (PF) {
        if (nfull > 0) {
            // ping-pong as above; the next-tile index is clamped to the last
            // full tile, so the vector loads never leave the segment
            Tin qa[EPL][4][4], qb[EPL][4][4];
            int ta[EPL], tb[EPL];
            load_vector<Tin, EPL>(io.S, ev0, lane0, qa, ta);
            for (uint32_t t = 0; t < nfull; t += 2) {
                const uint32_t n1 = t + 1 < nfull ? t + 1 : nfull - 1;
                load_vector<Tin, EPL>(io.S, ev0, n1 * step + lane0, qb, tb);
                process_tile<Tin, PREC, MODE, EPL, K0, K1, ORD>(kp, s, io, g, qa, ta, t * step + lane0, len, ev0, myhist,
                                                           srow, wc);
                if (t + 1 >= nfull) break;
                const uint32_t n2 = t + 2 < nfull ? t + 2 : nfull - 1;
                load_vector<Tin, EPL>(io.S, ev0, n2 * step + lane0, qa, ta);
                process_tile<Tin, PREC, MODE, EPL, K0, K1, ORD>(kp, s, io, g, qb, tb, (t + 1) * step + lane0, len, ev0,
                                                           myhist, srow, wc);
            }
        }
    } else {
        for (uint32_t t = 0; t < nfull; ++t) {
            Tin q[EPL][4][4];
            int tg[EPL];
            load_vector<Tin, EPL>(io.S, ev0, t * step + lane0, q, tg);
            process_tile<Tin, PREC, MODE, EPL, K0, K1, ORD>(kp, s, io, g, q, tg, t * step + lane0, len, ev0, myhist, srow,
                                                       wc);
        }
    }
    for (uint32_t t0 = nfull * step; t0 < len; t0 += step) {
        Tin q[EPL][4][4];
        int tg[EPL];
        load_scalar<Tin, EPL>(io.S, ev0, t0 + lane0, last, q, tg);
        process_tile<Tin, PREC, MODE, EPL, K0, K1, ORD>(kp, s, io, g, q, tg, t0 + lane0, len, ev0, myhist, srow, wc);
    }
}

// The pass over samples [kp.sbeg, kp.send), all of binning scheme (K0, K1):
// each workgroup takes a contiguous range of the virtual event space, splits
// it at sample boundaries, counts into LDS and flushes every segment.
template <typename Tin, int PREC, int MODE, int EPL, int K0, int K1, bool ORD>
__global__ __launch_bounds__(512) void tp_pass_kernel(const KParams kp)
{
    constexpr bool BINNED = MODE == 0 && K0 != AX_NONE;
    extern __shared__ __align__(16) unsigned char smem[];
    uint32_t *tot = reinterpret_cast<uint32_t *>(smem);          // 8 words: class totals, out of range
    uint32_t *hist = tot + 8;
    const int hist_words = kp.lds_copies * kp.hist_stride;
    double *ecache = reinterpret_cast<double *>(smem + (((8 + hist_words) * 4 + 15) & ~15));
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    uint32_t *myhist = hist + (wave % kp.lds_copies) * kp.hist_stride;

    int64_t vbeg = kp.vbeg + (int64_t)blockIdx.x * kp.range;
    const int64_t vend = vbeg + kp.range < kp.vend ? vbeg + kp.range : kp.vend;
    if (vbeg >= vend) return;
    // the sample table is read-only for the whole launch: read it through the
    // constant address space, so its fields arrive by scalar loads
    const ctab samples = (ctab)kp.samples;
    int lo = kp.sbeg, hi = kp.send - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (samples[mid].vstart <= vbeg) lo = mid;
        else hi = mid - 1;
    }
    for (int s = lo; s < kp.send && vbeg < vend; ++s) {
        const ctab S = samples + s;
        const int64_t sv0 = S->vstart;
        const int64_t sv1 = s + 1 < kp.send ? samples[s + 1].vstart : kp.vend;
        if (sv1 <= vbeg) continue;
        const int64_t segend = vend < sv1 ? vend : sv1;
        const int64_t n = S->n;
        const int64_t ev0 = vbeg - sv0;
        const int64_t ev1 = (segend - sv0) < n ? (segend - sv0) : n;
        vbeg = segend;
        if (ev1 <= ev0) continue;

        // everything the event loop needs, read once per segment
        SegIO io;
        io.S = S;
        io.vec = S->vec != 0;
        io.cls_out = S->cls_out;
        io.ct_out = S->ct_out;
        uint64_t *counts = S->counts;
        uint64_t *stats = S->stats;
        Seg g;
        g.sigma = S->sigma;
        g.nb0 = S->nbins[0];
        g.nb1 = S->nbins[1];
        g.nbtot = S->nbtot;
        g.slots0 = S->slots[0];
        g.slots1 = S->slots[1];
        g.glo0 = S->guess_lo[0];
        g.glo1 = S->guess_lo[1];
        g.ginv0 = S->guess_inv[0];
        g.ginv1 = S->guess_inv[1];
        g.olo = S->olo;
        g.odir = S->odir;
        const int nd0 = K0 != AX_NONE ? edge_doubles(K0, g.nb0) : 0;
        const int nd1 = K1 != AX_NONE ? edge_doubles(K1, g.nb1) : 0;
        const int eoff0 = S->eoff[0], eoff1 = S->eoff[1];
        const int nrow = (g.nbtot + 1) * 4;      // counters of the output layout
        const int srow = lds_stats(g.nbtot);
        g.e0 = ecache;
        g.e1 = ecache + nd0;
        for (int i = tid; i < 8 + hist_words; i += nthr) tot[i] = 0;   // tot and hist are contiguous
        for (int i = tid; i < nd0; i += nthr) ecache[i] = kp.edges[eoff0 + i];
        for (int i = tid; i < nd1; i += nthr) ecache[nd0 + i] = kp.edges[eoff1 + i];
        __syncthreads();

        WaveCounts wc = { 0, 0, 0, 0 };
        run_segment<Tin, PREC, MODE, EPL, K0, K1, ORD>(kp, s, io, g, ev0, (uint32_t)(ev1 - ev0), myhist, srow, wc);
        if (!BINNED && MODE == 0 && lane == 0) {
            atomicAdd(&myhist[0], wc.c0);
            atomicAdd(&myhist[1], wc.c1);
            atomicAdd(&myhist[2], wc.c2);
            atomicAdd(&myhist[3], wc.c3);
        }
        __syncthreads();
        // fold the copies; bin rows also feed the class totals, the overflow
        // row the totals and the out-of-range count
        for (int i = tid; i < srow + NSTAT; i += nthr) {
            uint32_t v = 0;
            for (int k = 0; k < kp.lds_copies; ++k) v += hist[k * kp.hist_stride + i];
            if (i < srow) {
                if (BINNED && i >= 4 && v) atomicAdd(&tot[i & 3], v);
                if (BINNED && i >= nrow && v) atomicAdd(&tot[4], v);
                if (i < nrow && v && counts && (!BINNED || i >= 4))
                    atomicAdd((unsigned long long *)(counts + i), (unsigned long long)v);
            } else if (i - srow == ST_EVENTS) {
                atomicAdd((unsigned long long *)(stats + ST_EVENTS), (unsigned long long)(ev1 - ev0));
            } else if (v) {
                atomicAdd((unsigned long long *)(stats + (i - srow)), (unsigned long long)v);
            }
        }
        if (BINNED) {
            __syncthreads();
            if (tid < 4) {
                if (tot[tid] && counts) atomicAdd((unsigned long long *)(counts + tid), (unsigned long long)tot[tid]);
            } else if (tid == 4) {
                if (tot[4]) atomicAdd((unsigned long long *)(stats + ST_OOR), (unsigned long long)tot[4]);
            }
        }
        __syncthreads();
    }
}

}  // namespace

// ---------------------------------------------------------- float32 tier probe
// Per event, the float32 tier's contraction sigma * det[kernel rows] with its
// running forward bound (what TP_PREC_F32_RECHECK certifies against), and the
// float64 contraction with the sum S of the magnitudes of its Laplace terms
// (its own error is below 8.1 u S): the measurement of the float32 error.
__global__ __launch_bounds__(256) void tp_probe_kernel(const KSample k, float *det32, float *bound32,
                                                       double *det64, double *scale64)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k.n) return;
    float q[4][4];
    double x[4][4];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        q[t >> 2][t & 3] = static_cast<const float *>(k.p[t])[i];
        x[t >> 2][t & 3] = (double)q[t >> 2][t & 3];
    }
    float d32, b32;
    det_f32(q, d32, &b32);
    double m01[6], m23[6], d64;
    minors_f64<true>(x[0], x[1], m01);
    minors_f64<true>(x[2], x[3], m23);
    det_f64<true>(m01, m23, d64);
    double S = dabs(m01[0]) * dabs(m23[5]);
#pragma unroll
    for (int t = 1; t < 6; ++t) S = fma(dabs(m01[t]), dabs(m23[5 - t]), S);
    det32[i] = k.sigma > 0 ? d32 : -d32;
    bound32[i] = b32;
    det64[i] = k.sigma > 0 ? d64 : -d64;
    scale64[i] = S;
}

// ------------------------------------------------------------------ launchers
namespace {
template <typename T, int P, int M, int EPL, int K0, int K1>
void launch_one(bool ord, const KParams &kp, int grid, int block, size_t lds, hipStream_t st)
{
    // with a plane angle binned, the float32-sign variant is the float64 one
    constexpr int PE = (K0 == AX_ABSPHI || K1 == AX_ABSPHI) ? 0 : P;
    // the first pass takes the ordering of identical particles as a
    // compile-time step; the full evaluation decides it per sample
    if (lean_pass<T, M, K0, K1>() && ord)
        hipLaunchKernelGGL((tp_pass_kernel<T, PE, M, EPL, K0, K1, true>), dim3(grid), dim3(block), lds, st, kp);
    else
        hipLaunchKernelGGL((tp_pass_kernel<T, PE, M, EPL, K0, K1, false>), dim3(grid), dim3(block), lds, st, kp);
}

template <typename T, int P, int M, int K0, int K1>
void launch_epl(int epl, bool ord, const KParams &kp, int grid, int block, size_t lds, hipStream_t st)
{
    if constexpr (sizeof(T) == 4) {
        if (epl >= 4) {
            launch_one<T, P, M, 4, K0, K1>(ord, kp, grid, block, lds, st);
            return;
        }
    }
    if (epl >= 2) launch_one<T, P, M, 2, K0, K1>(ord, kp, grid, block, lds, st);
    else launch_one<T, P, M, 1, K0, K1>(ord, kp, grid, block, lds, st);
}

template <typename T, int P, int M>
bool launch_scheme(int k0, int k1, int epl, bool ord, const KParams &kp, int grid, int block, size_t lds,
                   hipStream_t st)
{
    if constexpr (M == 1) {
        if (k0 != AX_NONE || k1 != AX_NONE) return false;
        launch_epl<T, P, M, AX_NONE, AX_NONE>(epl, ord, kp, grid, block, lds, st);
        return true;
    } else {
#define TP_CASE(A, B)                                                          \
    case A * 4 + B: launch_epl<T, P, M, A, B>(epl, ord, kp, grid, block, lds, st); return true;
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

hipError_t launch_probe(const KSample &k, float *det32, float *bound32, double *det64, double *scale64,
                        hipStream_t st)
{
    const int64_t grid = (k.n + 255) / 256;
    hipLaunchKernelGGL(tp_probe_kernel, dim3((unsigned)grid), dim3(256), 0, st, k, det32, bound32, det64, scale64);
    return hipGetLastError();
}

hipError_t launch_pass(int dtype, int prec, int mode, int epl, int k0, int k1, bool ord, const KParams &kp, int grid,
                       int block, size_t lds, hipStream_t st)
{
    bool ok;
    if (dtype == 0) {
        if (prec == 1) {
            ok = mode == 0 ? launch_scheme<float, 1, 0>(k0, k1, epl, ord, kp, grid, block, lds, st)
                           : launch_scheme<float, 1, 1>(k0, k1, epl, ord, kp, grid, block, lds, st);
        } else {
            ok = mode == 0 ? launch_scheme<float, 0, 0>(k0, k1, epl, ord, kp, grid, block, lds, st)
                           : launch_scheme<float, 0, 1>(k0, k1, epl, ord, kp, grid, block, lds, st);
        }
    } else {
        ok = mode == 0 ? launch_scheme<double, 0, 0>(k0, k1, epl, ord, kp, grid, block, lds, st)
                       : launch_scheme<double, 0, 1>(k0, k1, epl, ord, kp, grid, block, lds, st);
    }
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace tpk
