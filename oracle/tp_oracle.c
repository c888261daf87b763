/*
 * Plain FP64 CPU oracle of the T-odd triple-product pass.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
 * file; only the tests, the smoke check and the CPU-baseline timing do.  It
 * shares no code, header or table with the HIP implementation.
 *
 * It follows the paper's definitions step by step, in float64, with textbook
 * formulas (Sect. 5 and eq. (4)):
 *   1. read the stored components (float32 promoted exactly, or float64);
 *   2. P = sum of the four momenta, M^2 = P.P, M = sqrt(M^2);
 *   3. boost every daughter into the M rest frame (pure boost, beta = P/E_P);
 *      if the channel has two identical particles (slots f, s), the one with
 *      the larger rest-frame energy E* is put in slot f (an exact tie keeps
 *      the stored order), since swapping them flips the sign of C_T;
 *   4. C_T = p*_A . (p*_B x p*_C) with the channel's slots (Sect. 5); for an
 *      anti-particle event the same slots hold the C-conjugates, giving Cbar_T;
 *   5. class by flavour and sign (eq. (4)): M with C_T>0 -> [I], C_T<0 -> [II];
 *      Mbar with -Cbar_T>0 -> [III], -Cbar_T<0 -> [IV];
 *   6. phase-space coordinates: the acoplanarity angle between the (i,j) and
 *      (k,l) decay planes (Sect. 5, a P-odd coordinate), two-body or multi-body
 *      invariant masses (Sect. 4.2, P-even), and the helicity-type angle of one
 *      daughter against the M flight direction (P-even);
 *   7. count per bin and class.
 *
 * Every decision (a sign, an edge comparison) whose float64 value lies within
 * a generous margin of its boundary is NOT taken here: the event is written to
 * the ``flagged`` list and left out of all counts, and the Python side decides
 * it in exact rational arithmetic.  The margins are many orders of magnitude
 * above the float64 error of these formulas (the tests measure that error).
 *
 * Validity: an event is invalid if a component is not finite, the tag is not 0
 * or 1, or P is not a future time-like vector (E_P > 0 and M^2 > 0), since
 * then there is no M rest frame.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_ABSPHI = 0, OR_MASS = 1, OR_ABSCOS = 2 };
enum { OR_I = 0, OR_II = 1, OR_III = 2, OR_IV = 3, OR_ZERO = 4, OR_INVALID = 5, OR_FLAGGED = 6 };

/* Lorentz factors above this are always sent to the exact resolver. */
#define OR_GAMMA_MAX 1.0e4
/* relative sign margin, scaled by (1 + gamma^2) */
#define OR_TAU 1.0e-9

typedef struct {
    int32_t naxes;
    int32_t kind[2];
    int32_t nbins[2];
    int32_t slots[2];
    const double *edges[2];
} or_binning;

static void cross3(const double a[3], const double b[3], double r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* Result of one event: class, bin (or -1 out of range), C_T value. */
typedef struct {
    int cls;
    int64_t bin;   /* combined bin, -1 = out of range, -2 = not binned */
    double ct;
    double coord[2];  /* per axis: cos Phi, m^2 or |cos theta| */
} or_event;

/*
 * Decide bin index of value v for increasing edges e[0..nb] with bins
 * [e_j, e_{j+1}) and the last bin closed.  Returns -1 if outside.
 * *near is set if v lies within ``margin`` of an edge.
 */
static int64_t bin_increasing(double v, const double *e, int nb, double margin, int *near)
{
    for (int k = 0; k <= nb; ++k)
        if (fabs(v - e[k]) <= margin) *near = 1;
    if (v < e[0] || v > e[nb]) return -1;
    int64_t j = 0;
    for (int k = 1; k < nb; ++k)
        if (v >= e[k]) j = k;
    return j;
}

static or_event one_event(const double pin[4][4], int tag, const int32_t triple[3],
                          const int32_t planes[4], const int32_t *ident, const or_binning *bn)
{
    or_event r = { OR_INVALID, -2, 0.0, { 0.0, 0.0 } };
    double p[4][4];
    memcpy(p, pin, sizeof p);
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 4; ++c)
            if (!isfinite(p[s][c])) return r;
    if (tag != 0 && tag != 1) return r;

    /* step 2: parent four-momentum and mass */
    double P[4] = { 0, 0, 0, 0 };
    double sumE = 0.0;
    for (int s = 0; s < 4; ++s) {
        for (int c = 0; c < 4; ++c) P[c] += p[s][c];
        sumE += fabs(p[s][0]);
    }
    double P3sq = P[1] * P[1] + P[2] * P[2] + P[3] * P[3];
    double M2 = P[0] * P[0] - P3sq;
    if (fabs(M2) <= 1e-9 * (P[0] * P[0] + P3sq) || fabs(P[0]) <= 1e-12 * sumE) {
        r.cls = OR_FLAGGED;
        return r;
    }
    if (!(P[0] > 0.0 && M2 > 0.0)) return r;
    double M = sqrt(M2);
    double gamma = P[0] / M;
    if (!(gamma <= OR_GAMMA_MAX)) {
        r.cls = OR_FLAGGED;
        return r;
    }

    /* step 3: pure boost to the rest frame: beta = P/E_P */
    double beta[3] = { P[1] / P[0], P[2] / P[0], P[3] / P[0] };
    double b2 = dot3(beta, beta);
    double ps[4][3], Es[4];   /* Es: |E*| + |p*|, a scale for the decision margins */
    for (int s = 0; s < 4; ++s) {
        const double *q = p[s];
        double bp = beta[0] * q[1] + beta[1] * q[2] + beta[2] * q[3];
        double k = (b2 > 0.0) ? (gamma - 1.0) * bp / b2 - gamma * q[0] : 0.0;
        for (int c = 0; c < 3; ++c) ps[s][c] = q[1 + c] + k * beta[c];
        Es[s] = fabs(gamma * (q[0] - bp)) + norm3(ps[s]);
    }
    double g2 = 1.0 + gamma * gamma;

    /* step 3b: identical particles ordered by rest-frame energy E* = gamma (E - beta.p) */
    if (ident && ident[0] >= 0) {
        const int f = ident[0], sl = ident[1];
        const double Ef = gamma * (p[f][0] - (beta[0] * p[f][1] + beta[1] * p[f][2] + beta[2] * p[f][3]));
        const double Esl = gamma * (p[sl][0] - (beta[0] * p[sl][1] + beta[1] * p[sl][2] + beta[2] * p[sl][3]));
        if (fabs(Ef - Esl) <= OR_TAU * g2 * (Es[f] + Es[sl])) {
            r.cls = OR_FLAGGED;
            return r;
        }
        if (Esl > Ef) {
            for (int c = 0; c < 4; ++c) { double t = p[f][c]; p[f][c] = p[sl][c]; p[sl][c] = t; }
            for (int c = 0; c < 3; ++c) { double t = ps[f][c]; ps[f][c] = ps[sl][c]; ps[sl][c] = t; }
            double t = Es[f]; Es[f] = Es[sl]; Es[sl] = t;
        }
    }

    /* step 4: triple product in the rest frame */
    double bc[3];
    cross3(ps[triple[1]], ps[triple[2]], bc);
    double ct = dot3(ps[triple[0]], bc);
    r.ct = ct;
    double scale = Es[triple[0]] * Es[triple[1]] * Es[triple[2]];
    if (fabs(ct) <= OR_TAU * g2 * scale) {
        r.cls = OR_FLAGGED;
        return r;
    }

    /* step 5: class (eq. (4)) */
    if (tag == 0) r.cls = (ct > 0.0) ? OR_I : OR_II;
    else          r.cls = (-ct > 0.0) ? OR_III : OR_IV;

    /* step 6/7: bins */
    int64_t bin = 0;
    int near = 0;
    for (int a = 0; a < bn->naxes; ++a) {
        const int nb = bn->nbins[a];
        const double *e = bn->edges[a];
        int64_t j;
        if (bn->kind[a] == OR_ABSPHI) {
            double n1[3], n2[3];
            cross3(ps[planes[0]], ps[planes[1]], n1);
            cross3(ps[planes[2]], ps[planes[3]], n2);
            double l1 = norm3(n1), l2 = norm3(n2);
            double cphi = dot3(n1, n2) / (l1 * l2);
            double margin = OR_TAU * g2 *
                (Es[planes[0]] * Es[planes[1]] / l1 + Es[planes[2]] * Es[planes[3]] / l2);
            r.coord[a] = cphi;
            if (!isfinite(cphi) || !isfinite(margin)) { r.cls = OR_FLAGGED; return r; }
            /* edges are cosines, decreasing: bin j holds c_{j+1} < cos|Phi| <= c_j */
            for (int k = 0; k <= nb; ++k)
                if (fabs(cphi - e[k]) <= margin) near = 1;
            if (cphi > e[0] || cphi < e[nb]) j = -1;
            else {
                j = 0;
                for (int k = 1; k < nb; ++k)
                    if (cphi <= e[k]) j = k;
            }
        } else if (bn->kind[a] == OR_MASS) {
            double S[4] = { 0, 0, 0, 0 };
            for (int s = 0; s < 4; ++s)
                if (bn->slots[a] & (1 << s))
                    for (int c = 0; c < 4; ++c) S[c] += p[s][c];
            double mag = S[0] * S[0] + S[1] * S[1] + S[2] * S[2] + S[3] * S[3];
            double m2 = S[0] * S[0] - S[1] * S[1] - S[2] * S[2] - S[3] * S[3];
            r.coord[a] = m2;
            /* compare m^2 with e_k^2: bin j holds e_j <= m < e_{j+1} */
            j = -1;
            int inside = 1;
            for (int k = 0; k <= nb; ++k) {
                double e2 = e[k] * e[k];
                if (fabs(m2 - e2) <= 1e-12 * (mag + e2)) near = 1;
            }
            if (m2 < e[0] * e[0] || m2 > e[nb] * e[nb]) inside = 0;
            if (inside) {
                j = 0;
                for (int k = 1; k < nb; ++k)
                    if (m2 >= e[k] * e[k]) j = k;
            }
        } else { /* OR_ABSCOS: angle of p*_slot against the M flight direction */
            const int s = bn->slots[a];
            double pl = sqrt(P3sq);
            double lp = norm3(ps[s]);
            double cth = fabs(dot3(ps[s], &P[1]) / (lp * pl));
            double margin = OR_TAU * g2 * (Es[s] / lp);
            r.coord[a] = cth;
            if (!isfinite(cth) || !isfinite(margin) || pl == 0.0) { r.cls = OR_FLAGGED; return r; }
            j = bin_increasing(cth, e, nb, margin, &near);
        }
        if (j < 0) bin = -1;
        else if (bin >= 0) bin = bin * nb + j;
    }
    if (near) {
        r.cls = OR_FLAGGED;
        return r;
    }
    r.bin = (bn->naxes > 0) ? bin : -2;
    return r;
}

/*
 * Run the pass over n events.
 *   comp[16]: slot-major arrays (slot*4 + {E,px,py,pz}), float32 if dtype==0 else float64.
 *   counts: uint64[(nbins_total+1)*4], row 0 = all classified events, row 1+b = bin b (accumulated).
 *   stats: uint64[4] = {events seen (not flagged), zero, invalid, out of range} (accumulated).
 *   flagged: indices of events left to the exact resolver (capacity cap); returns their number
 *            (may exceed cap: then only cap were written).
 *   cls_out (int8[n]), ct_out (double[n]) and coord_out (double[2n], axis values
 *   cos Phi / m^2 / |cos theta| of each event) may be NULL.
 *   ident: NULL or int32[2] = (fast slot, slow slot) of two identical particles.
 */
int64_t or_pass(int64_t n, int32_t dtype, const void *const *comp, const int8_t *tag,
                const int32_t *triple, const int32_t *planes, const int32_t *ident,
                int32_t naxes, const int32_t *kind, const int32_t *nbins, const int32_t *slots,
                const double *const *edges,
                uint64_t *counts, uint64_t *stats, int64_t *flagged, int64_t cap,
                int8_t *cls_out, double *ct_out, double *coord_out, int32_t nthreads)
{
    or_binning bn;
    memset(&bn, 0, sizeof bn);
    bn.naxes = naxes;
    int64_t nb_total = 1;
    for (int a = 0; a < naxes; ++a) {
        bn.kind[a] = kind[a];
        bn.nbins[a] = nbins[a];
        bn.slots[a] = slots[a];
        bn.edges[a] = edges[a];
        nb_total *= nbins[a];
    }
    if (naxes == 0) nb_total = 0;
    const int64_t ncnt = (nb_total + 1) * 4;
    int64_t nflag = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        uint64_t *h = (uint64_t *)calloc((size_t)ncnt, sizeof(uint64_t));
        uint64_t st[4] = { 0, 0, 0, 0 };
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double p[4][4];
            for (int s = 0; s < 4; ++s)
                for (int c = 0; c < 4; ++c)
                    p[s][c] = dtype == 0 ? (double)((const float *)comp[s * 4 + c])[i]
                                         : ((const double *)comp[s * 4 + c])[i];
            or_event ev = one_event(p, tag[i], triple, planes, ident, &bn);
            if (cls_out) cls_out[i] = (int8_t)ev.cls;
            if (ct_out) ct_out[i] = ev.ct;
            if (coord_out) { coord_out[2 * i] = ev.coord[0]; coord_out[2 * i + 1] = ev.coord[1]; }
            if (ev.cls == OR_FLAGGED) {
                int64_t k;
#pragma omp atomic capture
                k = nflag++;
                if (k < cap) flagged[k] = i;
                continue;
            }
            st[0]++;
            if (ev.cls == OR_ZERO) { st[1]++; continue; }
            if (ev.cls == OR_INVALID) { st[2]++; continue; }
            h[ev.cls]++;
            if (ev.bin == -1) st[3]++;
            else if (ev.bin >= 0) h[(1 + ev.bin) * 4 + ev.cls]++;
        }
#pragma omp critical
        {
            for (int64_t k = 0; k < ncnt; ++k) counts[k] += h[k];
            for (int k = 0; k < 4; ++k) stats[k] += st[k];
        }
        free(h);
    }
    return nflag;
}

int32_t or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
