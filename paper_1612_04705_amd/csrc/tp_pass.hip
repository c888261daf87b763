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

// Bin of the plane angle between kernel planes (0,1) and (2,3).
// edges: c_0 = 1 > c_1 > ... > c_n = -1; returns #{k in 1..n-1 : cos Phi <= c_k}.
__device__ __forceinline__ int bin_absphi(const double x[4][4], const double w[4], double W,
                                          double M2, double eM, double kdot,
                                          const double *edges, int n, bool &sure)
{
    double d[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) {
            d[a][b] = mink(x[a], x[b]);
            d[b][a] = d[a][b];
        }
    double PP[4], Ua[4], Va[4], Ta[4], V2a[4];
    const double uW = (7.2 * U64) * W;
    const double aM = dabs(M2);
    const double tM = (kdot * U64) * aM;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        PP[a] = (d[a][0] + d[a][1]) + (d[a][2] + d[a][3]);
        Ua[a] = uW * w[a];                 // error bound of P.p_a
        Va[a] = dabs(PP[a]);
        Ta[a] = tM * w[a];
        V2a[a] = (2.01 * U64) * Va[a];
    }
    const double uWW = U64 * W * W;
    const double cd = fma(10.2, uWW, (2.01 * U64) * aM);
    const double c2 = 94.0 * uWW * uWW;
    double G[4][4], eG[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) {
            G[a][b] = fma(PP[a], PP[b], -(M2 * d[a][b]));
            eG[a][b] = fma(Ua[a], Va[b], fma(Ua[b], Va[a], fma(cd, dabs(d[a][b]),
                          fma(Ta[a], w[b], fma(V2a[a], Va[b], c2)))));
        }
    (void)eM;
    const double u2 = 2.01 * U64;
    // X = G02 G13 - G03 G12 ; N1 = G00 G11 - G01^2 ; N2 = G22 G33 - G23^2
    const double X = fma(G[0][2], G[1][3], -(G[0][3] * G[1][2]));
    const double eX = fma(dabs(G[0][2]) + eG[0][2], eG[1][3],
                      fma(dabs(G[1][3]), eG[0][2],
                      fma(dabs(G[0][3]) + eG[0][3], eG[1][2],
                      fma(dabs(G[1][2]), eG[0][3],
                          u2 * (dabs(G[0][2] * G[1][3]) + dabs(G[0][3] * G[1][2]))))));
    const double N1 = fma(G[0][0], G[1][1], -(G[0][1] * G[0][1]));
    const double eN1 = fma(dabs(G[0][0]) + eG[0][0], eG[1][1],
                       fma(dabs(G[1][1]), eG[0][0],
                       fma(2.0 * dabs(G[0][1]) + eG[0][1], eG[0][1],
                           u2 * (dabs(G[0][0] * G[1][1]) + G[0][1] * G[0][1]))));
    const double N2 = fma(G[2][2], G[3][3], -(G[2][3] * G[2][3]));
    const double eN2 = fma(dabs(G[2][2]) + eG[2][2], eG[3][3],
                       fma(dabs(G[3][3]), eG[2][2],
                       fma(2.0 * dabs(G[2][3]) + eG[2][3], eG[2][3],
                           u2 * (dabs(G[2][2] * G[3][3]) + G[2][3] * G[2][3]))));
    bool ok = (N1 > eN1) && (N2 > eN2);
    const double D = N1 * N2;
    const double eD = fma(N1 + eN1, eN2, fma(N2, eN1, U64 * D));
    ok = ok && (eD <= 0.25 * D);
    const double r = 1.0 / sqrt(D);
    const double v = X * r;
    // |v - cos Phi| <= eX/s + eD/s^2 + 8.4u (|cos Phi| <= 1), s = sqrt(D)
    const double eps = fma(1.001, fma(eX, r, eD * r * r), 11.0 * U64);
    int bin = 0;
    for (int k = 1; k < n; ++k) {
        const double c = edges[k];
        const bool le = (v + eps) <= c;
        const bool gt = (v - eps) > c;
        bin += le ? 1 : 0;
        ok = ok && (le || gt);
    }
    sure = sure && ok;
    return bin;
}

// |cos theta| of kernel slot s against the M flight direction.
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
    const double r = 1.0 / sqrt(D);
    const double v = dabs(Nn) * r;
    const double eps = fma(1.001, fma(eNn, r, eD * r * r), 11.0 * U64);
    int bin = 0;
    for (int k = 1; k < n; ++k) {
        const double e = edges[k];
        const bool ge = (v - eps) >= e;
        const bool lt = (v + eps) < e;
        bin += ge ? 1 : 0;
        ok = ok && (ge || lt);
    }
    sure = sure && ok;
    return bin;
}

// Invariant mass of the kernel slots in ``mask``.  ed: [sq_lo(n+1) | sq_hi(n+1)].
// Returns the bin or -1 (out of range).
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
    // guess from a uniform grid, then certify against the two neighbouring edges
    const float mg = sqrtf(fmaxf((float)m2, 0.0f));
    int j = (int)floorf((float)(((double)mg - glo) * ginv));
    j = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
    bool ok = mlo >= sqhi[j] && (j == n - 1 ? mhi <= sqlo[n] : mhi < sqlo[j + 1]);
    if (ok) return j;
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
        const bool lt = mhi < sqlo[k];
        bin += ge ? 1 : 0;
        dec = dec && (ge || lt);
    }
    sure = sure && dec;
    return bin;
}

struct Seg {
    int32_t sigma, naxes, kind0, kind1, nb0, nb1, slots0, slots1;
    double glo0, ginv0, glo1, ginv1;
    const double *e0, *e1;    // LDS edge data of each axis
};

template <typename Tin, int PREC>
__device__ __forceinline__ EvOut eval_event(const Tin (&q)[4][4], int tag, const Seg &g)
{
    constexpr bool EXACTP = sizeof(Tin) == 4;
    constexpr double KDOT = EXACTP ? 3.02 : 4.02;
    EvOut o;
    o.cls = CLS_DEFER;
    o.bin = -1;
    o.t2 = 0;
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
    const double eM = (10.2 * U64) * W * W;
    const double Emin = fmin(fmin(x[0][0], x[1][0]), fmin(x[2][0], x[3][0]));
    if (!(Emin >= 0.0 && P[0] > 0.0 && M2 > (11.0 * U64) * W * W)) return o;

    // sign of the triple product
    double det;
    bool sure;
    if (PREC == 1) {
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
    if (!sure) return o;
    const int cls = tag == 0 ? (ct > 0.0 ? CLS_I : CLS_II) : (ct < 0.0 ? CLS_III : CLS_IV);

    // bins
    int bin = 0;
    bool oor = false;
    bool bsure = true;
    for (int a = 0; a < g.naxes; ++a) {
        const int kind = a == 0 ? g.kind0 : g.kind1;
        const int nb = a == 0 ? g.nb0 : g.nb1;
        const int sl = a == 0 ? g.slots0 : g.slots1;
        const double *ed = a == 0 ? g.e0 : g.e1;
        int j;
        if (kind == AX_ABSPHI) {
            j = bin_absphi(x, w, W, M2, eM, KDOT, ed, nb, bsure);
        } else if (kind == AX_MASS) {
            j = bin_mass(x, w, sl, ed, nb, a == 0 ? g.glo0 : g.glo1, a == 0 ? g.ginv0 : g.ginv1, bsure);
        } else {
            j = bin_abscos(x, w, W, P, M2, eM, KDOT, sl, ed, nb, bsure);
        }
        if (j < 0) oor = true;
        bin = bin * nb + (j < 0 ? 0 : j);
    }
    if (!bsure) return o;
    o.cls = cls;
    o.bin = oor ? -1 : bin;
    return o;
}

__device__ __forceinline__ uint32_t wave_count(bool p)
{
    return (uint32_t)__popcll(__ballot(p));
}

template <typename Tin>
__device__ __forceinline__ Tin ld(const void *p, int64_t i)
{
    return __builtin_nontemporal_load(reinterpret_cast<const Tin *>(p) + i);
}

template <typename Tin, int PREC, int MODE>
__global__ __launch_bounds__(512) void tp_pass_kernel(const KParams kp)
{
    constexpr int EPL = sizeof(Tin) == 4 ? 4 : 2;   // events per lane per step (16-byte loads)
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
        const int64_t ev0 = vbeg - sv0;
        const int64_t ev1 = (segend - sv0) < S->n ? (segend - sv0) : S->n;
        vbeg = segend;
        if (ev1 <= ev0) continue;

        Seg g;
        g.sigma = S->sigma;
        g.naxes = MODE == 0 ? S->naxes : 0;
        g.kind0 = S->kind[0];
        g.kind1 = S->kind[1];
        g.nb0 = S->nbins[0];
        g.nb1 = S->nbins[1];
        g.slots0 = S->slots[0];
        g.slots1 = S->slots[1];
        g.glo0 = S->guess_lo[0];
        g.glo1 = S->guess_lo[1];
        g.ginv0 = S->guess_inv[0];
        g.ginv1 = S->guess_inv[1];
        const int nd0 = g.naxes > 0 ? edge_doubles(g.kind0, g.nb0) : 0;
        const int nd1 = g.naxes > 1 ? edge_doubles(g.kind1, g.nb1) : 0;
        g.e0 = ecache;
        g.e1 = ecache + nd0;
        const int nrow = (S->nbtot + 1) * 4;
        const int ncnt = nrow + NSTAT;
        for (int i = tid; i < hist_words; i += nthr) hist[i] = 0;
        for (int i = tid; i < nd0; i += nthr) ecache[i] = kp.edges[S->eoff[0] + i];
        for (int i = tid; i < nd1; i += nthr) ecache[nd0 + i] = kp.edges[S->eoff[1] + i];
        __syncthreads();

        uint32_t wc0 = 0, wc1 = 0, wc2 = 0, wc3 = 0, wzero = 0, winv = 0, woor = 0, wt2 = 0,
                 wt3 = 0, wun = 0;
        const bool vec = S->vec != 0;
        for (int64_t t0 = ev0; t0 < ev1; t0 += (int64_t)EPL * nthr) {
            const int64_t base = t0 + (int64_t)EPL * tid;
            Tin q[EPL][4][4];
            int tg[EPL];
            if (vec && base + EPL <= S->n) {
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    if constexpr (EPL == 4) {
                        const f32x4 v = __builtin_nontemporal_load(
                            reinterpret_cast<const f32x4 *>(S->p[k]) + (base >> 2));
                        q[0][k >> 2][k & 3] = v.x;
                        q[1][k >> 2][k & 3] = v.y;
                        q[2][k >> 2][k & 3] = v.z;
                        q[3][k >> 2][k & 3] = v.w;
                    } else {
                        const f64x2 v = __builtin_nontemporal_load(
                            reinterpret_cast<const f64x2 *>(S->p[k]) + (base >> 1));
                        q[0][k >> 2][k & 3] = v.x;
                        q[1][k >> 2][k & 3] = v.y;
                    }
                }
                if constexpr (EPL == 4) {
                    const uint32_t t = __builtin_nontemporal_load(
                        reinterpret_cast<const uint32_t *>(S->tag) + (base >> 2));
#pragma unroll
                    for (int e = 0; e < 4; ++e) tg[e] = (int)(int8_t)(t >> (8 * e));
                } else {
                    const uint16_t t = __builtin_nontemporal_load(
                        reinterpret_cast<const uint16_t *>(S->tag) + (base >> 1));
                    tg[0] = (int)(int8_t)(t & 0xff);
                    tg[1] = (int)(int8_t)(t >> 8);
                }
            } else {
#pragma unroll
                for (int e = 0; e < EPL; ++e) {
                    const int64_t i = base + e;
                    const bool in = i < ev1;
#pragma unroll
                    for (int k = 0; k < 16; ++k) q[e][k >> 2][k & 3] = in ? ld<Tin>(S->p[k], i) : (Tin)0;
                    tg[e] = in ? (int)S->tag[i] : -1;
                }
            }
#pragma unroll
            for (int e = 0; e < EPL; ++e) {
                const int64_t i = base + e;
                const bool in = i < ev1;
                EvOut o;
                if (in) {
                    o = eval_event<Tin, PREC>(q[e], tg[e], g);
                } else {
                    o.cls = -1;
                    o.bin = -1;
                    o.t2 = 0;
                    o.ct = 0.0;
                }
                bool listed = false, unres = false;
                if (o.cls == CLS_DEFER) {
                    const uint32_t slot = atomicAdd(kp.xcount, 1u);
                    if (slot < kp.xcap) {
                        kp.xlist[slot] = ((uint64_t)s << 40) | (uint64_t)i;
                        listed = true;
                    } else {
                        unres = true;
                    }
                }
                if (MODE == 1 && in) {
                    S->cls_out[i] = (int8_t)(unres ? CLS_UNRESOLVED : (o.cls == CLS_DEFER ? CLS_DEFER : o.cls));
                    if (S->ct_out) S->ct_out[i] = o.ct;
                }
                if (MODE == 0 && o.cls >= 0 && o.cls < 4 && o.bin >= 0 && g.naxes > 0)
                    atomicAdd(&myhist[(1 + o.bin) * 4 + o.cls], 1u);
                wc0 += wave_count(o.cls == CLS_I);
                wc1 += wave_count(o.cls == CLS_II);
                wc2 += wave_count(o.cls == CLS_III);
                wc3 += wave_count(o.cls == CLS_IV);
                wzero += wave_count(o.cls == CLS_ZERO);
                winv += wave_count(o.cls == CLS_INVALID);
                woor += wave_count(o.cls >= 0 && o.cls < 4 && o.bin < 0 && g.naxes > 0);
                wt2 += wave_count(o.t2 != 0);
                wt3 += wave_count(listed);
                wun += wave_count(unres);
            }
        }
        if (lane == 0) {
            if (MODE == 0) {
                atomicAdd(&myhist[0], wc0);
                atomicAdd(&myhist[1], wc1);
                atomicAdd(&myhist[2], wc2);
                atomicAdd(&myhist[3], wc3);
            }
            atomicAdd(&myhist[nrow + ST_ZERO], wzero);
            atomicAdd(&myhist[nrow + ST_INVALID], winv);
            atomicAdd(&myhist[nrow + ST_OOR], woor);
            atomicAdd(&myhist[nrow + ST_TIER2], wt2);
            atomicAdd(&myhist[nrow + ST_TIER3], wt3);
            atomicAdd(&myhist[nrow + ST_UNRESOLVED], wun);
        }
        __syncthreads();
        for (int i = tid; i < ncnt; i += nthr) {
            uint32_t v = 0;
            for (int k = 0; k < kp.lds_copies; ++k) v += hist[k * kp.hist_stride + i];
            if (i < nrow) {
                if (v && S->counts) atomicAdd((unsigned long long *)(S->counts + i), (unsigned long long)v);
            } else if (i - nrow == ST_EVENTS) {
                atomicAdd((unsigned long long *)(S->stats + ST_EVENTS), (unsigned long long)(ev1 - ev0));
            } else if (v) {
                atomicAdd((unsigned long long *)(S->stats + (i - nrow)), (unsigned long long)v);
            }
        }
        __syncthreads();
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_pass(int dtype, int prec, int mode, const KParams &kp, int grid, int block,
                       size_t lds, hipStream_t st)
{
#define TP_L(T, P, M) hipLaunchKernelGGL((tp_pass_kernel<T, P, M>), dim3(grid), dim3(block), lds, st, kp)
    if (dtype == 0) {
        if (prec == 1) {
            if (mode == 0) TP_L(float, 1, 0);
            else TP_L(float, 1, 1);
        } else {
            if (mode == 0) TP_L(float, 0, 0);
            else TP_L(float, 0, 1);
        }
    } else {
        if (mode == 0) TP_L(double, 0, 0);
        else TP_L(double, 0, 1);
    }
#undef TP_L
    return hipGetLastError();
}

}  // namespace tpk
