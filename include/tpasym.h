/*
 * tpasym: T-odd triple-product asymmetry pass on AMD Instinct MI355X (gfx950).
 *
 * The operation (Parkes et al., "On model-independent searches for direct CP
 * violation in multi-body decays", Sect. 5, eq. (4)-(6)):
 *   for every event of a four-body decay M -> A B C D (or its conjugate Mbar)
 *   compute the triple product C_T = p_A . (p_B x p_C) in the M rest frame
 *   (Cbar_T for Mbar, same slots holding the C-conjugate particles), split the
 *   sample into [I] M(C_T>0), [II] M(C_T<0), [III] Mbar(-Cbar_T>0),
 *   [IV] Mbar(-Cbar_T<0), count them, integrated and in phase-space bins, and
 *   form the asymmetries.
 *
 * C_T is evaluated without a boost as the Lorentz-invariant determinant
 *   C_T^inv = det[P; p_A; p_B; p_C] = M * C_T            (P = sum of the four momenta)
 * rows being contravariant (E, px, py, pz).  Every sign and every bin-edge
 * comparison is CERTIFIED: it equals the decision on the exact real value of
 * the stored inputs (float32 storage is promoted exactly).  Decisions are taken
 * by a fast floating-point tier with a rigorous forward error bound, escalated
 * to float64 and then to exact integer arithmetic only when the bound does not
 * decide.  Counts are therefore unique and reproducible bit for bit.
 *
 * Conventions of every entry point:
 *   - Device pointers are plain HIP device pointers; the caller owns all
 *     buffers and keeps them alive until the enqueued work has completed.
 *   - Work is enqueued asynchronously on ``stream`` (a hipStream_t, NULL = the
 *     null stream).  Results are valid after the caller synchronises.
 *   - Counts and statistics ACCUMULATE (+=): zero them once, then chunks,
 *     batches or shards simply add up.
 *   - Return value: TP_OK (0) or a negative tp_status.  All argument checks run
 *     on the host before anything is enqueued; on error nothing is enqueued and
 *     no output is touched.  tp_strerror() gives a thread-local message.
 *   - Events whose decision needs the exact tier beyond its range (a single
 *     event whose nonzero components span more than 2^107 (float64) / 2^136
 *     (float32) in magnitude) are counted in tp_stats.n_unresolved and in no
 *     class; callers must treat n_unresolved != 0 as an error.
 */
#ifndef TPASYM_H
#define TPASYM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPASYM_VERSION 10000 /* 1.0.0 */

typedef enum {
    TP_OK = 0,
    TP_EINVAL = -1,        /* bad argument (null pointer, size, slot, edges ...) */
    TP_EUNSUPPORTED = -2,  /* valid request the library does not support         */
    TP_EHIP = -3,          /* a HIP runtime call failed                           */
    TP_ENOMEM = -4,        /* device allocation failed                            */
    TP_ERANGE = -5,        /* a size exceeds an implementation limit              */
    TP_EUNCERTAIN = -6     /* reserved: a decision could not be certified         */
} tp_status;

/* storage type of the 16 component arrays */
typedef enum { TP_F32 = 0, TP_F64 = 1 } tp_dtype;

/* arithmetic of the first evaluation tier */
typedef enum {
    TP_PREC_F64 = 0,         /* float64 evaluation + bound, exact fallback                    */
    TP_PREC_F32_RECHECK = 1  /* float32 contraction + bound, float64 recheck, exact fallback;
                                bins in float64.  Requires TP_F32 storage.                    */
} tp_precision;

/* One sample of events.  Layout: structure of arrays, 16 contiguous arrays of
 * n elements, p[slot][c] with c = 0..3 for (E, px, py, pz) in MeV (any unit
 * works: everything is homogeneous), plus int8 flavour tags (0 = M, 1 = Mbar).
 * Arrays 16-byte aligned and n a multiple of 4 (float32) / 2 (float64) take
 * the vector-load path; anything else works through scalar loads.  A sample
 * of n = 0 events may carry NULL pointers: every call treats it as no work
 * (its counts and statistics are left as they are, and tp_batch and
 * tp_autotune leave it out of the plan). */
typedef struct {
    int64_t n;
    int32_t dtype;            /* tp_dtype */
    int32_t reserved;
    const void *p[4][4];      /* device */
    const int8_t *tag;        /* device */
} tp_events;

/* Channel: slots of the triple product and of the two decay planes.
 * triple = (A, B, C): C_T = p_A . (p_B x p_C) in the M rest frame; the three
 * slots must be distinct.  planes = (i, j, k, l), a permutation of 0..3: the
 * acoplanarity angle Phi is the angle between the (i, j) and (k, l) planes
 * in the M rest frame (Sect. 5: a triple-product-type, P-odd coordinate).
 *
 * identical = (f, s): two slots holding identical particles (two pi- in
 * Lambda_b -> p pi- pi+ pi-, two K- in Lambda_b -> p K- K+ K-), or (-1, -1).
 * Swapping them flips the sign of C_T, so their order is part of the
 * definition: the pass puts the one with the larger energy in the M rest frame
 * (the larger P.p) in slot f and the other in slot s, whatever the stored
 * order, so unordered data can be fed as is.  The comparison is certified
 * like every other decision (float64 with an error bound, exact arithmetic
 * when that does not settle it); an exact tie keeps the stored order.  When a
 * plane angle is binned, f and s must lie in different planes with matching
 * positions up to the pair swap: {planes[0], planes[2]} or {planes[1],
 * planes[3]} (TP_EUNSUPPORTED otherwise). */
typedef struct {
    int32_t triple[3];
    int32_t planes[4];
    int32_t identical[2];
} tp_channel;

typedef enum {
    /* folded acoplanarity |Phi| in [0, pi].  edges: the cosines
     * c_0 = 1 > c_1 > ... > c_n = -1 of the angle edges; bin j holds
     * c_{j+1} < cos|Phi| <= c_j (last bin closed).  The sign of sin Phi is the
     * sign of a triple product, so folding keeps every event's class and the
     * [0, 2 pi) histogram is recovered from (bin, class).                      */
    TP_AXIS_ABSPHI = 0,
    /* invariant mass of the slots in bit mask ``slots`` (sum of their momenta);
     * edges increasing, e_0 >= 0; bin j holds e_j <= m < e_{j+1}, last bin
     * closed; outside -> out of range (Sect. 4.2).                            */
    TP_AXIS_MASS = 1,
    /* |cos theta| of slot ``slots`` in the M rest frame, measured against the
     * M flight direction in the lab; edges 0 = e_0 < ... < e_n = 1, bins as
     * for MASS.                                                                */
    TP_AXIS_ABSCOS = 2
} tp_axis_kind;

typedef struct {
    int32_t kind;             /* tp_axis_kind */
    int32_t nbins;            /* 1 .. 1024 */
    int32_t slots;            /* MASS: bit mask (>= 2 bits); ABSCOS: slot; ABSPHI: unused */
    int32_t reserved;
    const double *edges;      /* HOST pointer, nbins + 1 values */
} tp_axis;

/* naxes = 0: global counts only; 1 or 2 axes, combined bin = i0 * nbins1 + i1.
 * At most one ABSPHI axis.  Total bins <= 1024. */
typedef struct {
    int32_t naxes;
    int32_t reserved;
    tp_axis axis[2];
} tp_binning;

/* Per-sample statistics (device, uint64, accumulated). */
typedef struct {
    uint64_t n_events;        /* events processed                                   */
    uint64_t n_zero;          /* C_T = 0 exactly: in no class                       */
    uint64_t n_invalid;       /* non-finite component, tag not 0/1, or P not a
                                 future time-like vector (no rest frame)            */
    uint64_t n_out_of_range;  /* classified events outside the binning (they stay
                                 in the global row of the counts)                   */
    uint64_t n_tier2;         /* events that needed the float64 recheck of the sign
                                 (TP_PREC_F32_RECHECK only)                         */
    uint64_t n_tier3;         /* events passed to the later tiers (double-word, then
                                 exact integers)                                    */
    uint64_t n_unresolved;    /* events beyond the exact tier's range: an error     */
    uint64_t reserved;
} tp_stats;

/* Class codes written by tp_compute. */
enum { TP_CLS_I = 0, TP_CLS_II = 1, TP_CLS_III = 2, TP_CLS_IV = 3, TP_CLS_ZERO = 4,
       TP_CLS_INVALID = 5, TP_CLS_UNRESOLVED = 6 };

/*
 * tp_compute -- per-event triple product and class (Sect. 5, eq. (4)).
 *   cls_out: device int8[n] (class codes above); required when n > 0 (the
 *            later tiers write the classes of the events they decide there).
 *   ct_out:  device double[n] or NULL: C_T^inv = det[P; p_A; p_B; p_C] = M * C_T
 *            (float64 estimate; its SIGN is exact, 0.0 exactly for class zero).
 *   stats:   device tp_stats, accumulated (required).
 * Class totals are not returned here; use tp_bin with naxes = 0.
 */
int tp_compute(const tp_events *ev, const tp_channel *ch, int32_t precision,
               int8_t *cls_out, double *ct_out, tp_stats *stats, void *stream);

/*
 * tp_bin -- counts per class, integrated and per phase-space bin (eq. (4)-(6)
 * need only these counts).
 *   counts: device uint64[(nbins_total + 1) * 4], row-major [row][class]:
 *           row 0 = every classified event, row 1 + b = bin b; accumulated.
 *   stats:  device tp_stats, accumulated.
 */
int tp_bin(const tp_events *ev, const tp_channel *ch, const tp_binning *bn, int32_t precision,
           uint64_t *counts, tp_stats *stats, void *stream);

/*
 * tp_bin_noalloc -- tp_bin for callers that cannot allocate device memory
 * (code under HIP graph capture, fixed-memory serving loops): the same
 * arguments, outputs and results, but the launch tables, the exact tier's
 * counters and its deferral list live in a file-scope device array of the
 * library (32 MiB + 4 KiB, held on each device it runs on until the process
 * ends), and no hipMalloc, hipFree or other allocating call is made.
 *   Limits per call: ev->n <= 2^22 events (larger samples: call once per chunk;
 *   counts accumulate) and at most 384 doubles of edge data (a MASS axis takes
 *   3 (nbins + 1), the others nbins + 1); beyond them TP_ERANGE, nothing enqueued.
 *   Launch shape: fixed (256 threads, 8 workgroups per compute unit).
 *   Every call on one device shares the array and overwrites it at its start:
 *   calls that overlap on one device (several streams or threads) race, and
 *   must be ordered by the caller.
 */
int tp_bin_noalloc(const tp_events *ev, const tp_channel *ch, const tp_binning *bn, int32_t precision,
                   uint64_t *counts, tp_stats *stats, void *stream);

/*
 * tp_probe_f32 -- measurement of the float32 tier (float32 storage only): per
 * event the float32 contraction C_T^inv (sign convention of tp_compute) from
 * Kahan-FMA minors, its running forward error bound (the event is rechecked in
 * float64 when |det32| <= bound32), the float64 contraction and the sum of the
 * magnitudes of its six Laplace terms (the float64 value is within 8.1 u of
 * that sum, u = 2^-53).  Certifies nothing: it reports the raw values.
 *   det32, bound32: device float[n]; det64, scale64: device double[n].
 */
int tp_probe_f32(const tp_events *ev, const tp_channel *ch, float *det32, float *bound32, double *det64,
                 double *scale64, void *stream);

/* One row of asymmetries.  Value/sigma pairs:
 *   A_T      = (N_I - N_II) / (N_I + N_II)
 *   Abar_T   = (N_III - N_IV) / (N_III + N_IV)
 *   a_CP     = (A_T - Abar_T) / 2,  a_P = (A_T + Abar_T) / 2   (T-odd analyses)
 *   A_plus   = A_CP(C_T > 0) = (N_I - N_III) / (N_I + N_III)   eq. (5)
 *   A_minus  = A_CP(C_T < 0) = (N_II - N_IV) / (N_II + N_IV)   eq. (5)
 *   A_even   = (A_plus + A_minus) / 2,  A_odd = (A_plus - A_minus) / 2   eq. (6)
 * sigma of a two-count asymmetry over n events: sqrt((1 - A^2) / n); of a half
 * sum or difference of two asymmetries of disjoint samples: half the quadrature
 * sum.  Each value is the exact ratio of integers rounded once (error <= 1 ulp).
 * A zero denominator gives NaN for value and sigma and sets its flag bit. */
typedef struct {
    double A_T, s_A_T, Abar_T, s_Abar_T, a_CP, s_a_CP, a_P, s_a_P;
    double A_plus, s_A_plus, A_minus, s_A_minus, A_even, s_A_even, A_odd, s_A_odd;
    uint64_t N[4];
    uint32_t flags;   /* bit0 N_I+N_II = 0, bit1 N_III+N_IV = 0, bit2 N_I+N_III = 0,
                         bit3 N_II+N_IV = 0 */
    uint32_t reserved;
} tp_asym_row;

/*
 * tp_asym -- asymmetries of every row of a counts table (host only).
 *   counts: HOST uint64[(nrows) * 4] as written by tp_bin; out: HOST tp_asym_row[nrows].
 */
int tp_asym(const uint64_t *counts, int64_t nrows, tp_asym_row *out);

/*
 * tp_scp -- binned S_CP significance and chi^2 (eq. (1)) on the same counts,
 * host only.  mode 0 (P-even test): X = [I]+[II], Xbar = [III]+[IV];
 * mode 1 (P-odd test): X = [I]+[IV], Xbar = [II]+[III] (Sect. 5).
 *   counts: HOST uint64[(nbins + 1) * 4] (row 0 ignored); s_out: HOST double[nbins] or NULL.
 *   alpha = N_tot(X)/N_tot(Xbar); S^i = (N^i(X) - alpha N^i(Xbar)) / sqrt(N^i(X) + alpha^2 N^i(Xbar))
 *   (0 for an empty bin); chi2 = sum S^i^2, ndf = nbins - 1, p = chi^2 survival function.
 */
int tp_scp(const uint64_t *counts, int64_t nbins, int32_t mode, double *s_out,
           double *chi2, int64_t *ndf, double *pvalue);

/* One sample of a batch. */
typedef struct {
    tp_events ev;
    tp_channel ch;
    tp_binning bn;
    uint64_t *counts;   /* device, as for tp_bin */
    tp_stats *stats;    /* device */
} tp_sample;

/* Launch shape of the persistent pass.  Zero fields take defaults. */
typedef struct {
    int32_t block;          /* threads per workgroup: 256 or 512                    */
    int32_t wg_per_cu;      /* persistent workgroups per compute unit: 1..32        */
    int32_t lds_copies;     /* LDS histogram copies per workgroup: 1 .. waves/WG    */
    int32_t unroll;         /* events per lane per step: 1, 2 or 4 (float32 storage;
                               float64 storage uses at most 2)                       */
} tp_tuning;

#define TP_BATCH_GRAPH 1    /* capture the launch in a HIP graph on first use and replay it */

/*
 * tp_batch -- every sample of ``samples`` in one call.  The samples are grouped
 * by binning scheme; each group is one persistent launch whose workgroups share
 * the group's event range in equal contiguous parts (a workgroup switches
 * descriptor and flushes its LDS histogram when it crosses from one sample into
 * the next).  Several groups run as parallel branches: the largest on
 * ``stream``, the others on internal side streams of the device (default
 * priority) that wait for ``stream`` at the call and that ``stream`` waits for
 * before the exact tier over the deferred events, so all work of the call is
 * ordered on ``stream`` as one launch would be.  Calls on different streams of
 * one device share the side streams, which orders their scheme launches among
 * themselves (results are unaffected).  Samples whose arrays reach 2^32 bytes
 * are passed as several descriptors internally (at most 2^20 descriptors in
 * all, else TP_ERANGE).
 *   tuning: NULL = each group's autotuned (or default) shape; else this shape
 *   for every group.  While groups run beside each other, the largest takes 16
 *   workgroups per CU and the others at most 4, whatever the shape.
 *   flags: TP_BATCH_GRAPH to capture/replay a graph keyed by the exact sample
 *   set, the shapes and the precision (the side streams join the capture).
 */
int tp_batch(const tp_sample *samples, int32_t nsamples, int32_t precision,
             const tp_tuning *tuning, int32_t flags, void *stream);

/*
 * tp_autotune -- per scheme group of this batch, time the candidate launch
 * shapes on that group's launch alone (into internal scratch counters: the
 * samples' counts and stats are NOT touched), store each group's best in the
 * in-process cache (and in the JSON file named by TP_TUNE_CACHE if set; a later
 * process reads that file back) and return the largest group's in *best.
 * Synchronises ``stream``.  With no event in any sample nothing is timed and
 * *best is the default shape.
 */
int tp_autotune(const tp_sample *samples, int32_t nsamples, int32_t precision,
                void *stream, tp_tuning *best);

/* Average duration (ms) of the pass of one call -- from before its first pass
 * launch to after the last scheme group has joined the launch stream, the exact
 * tier excluded -- over the last ``tp_timing_reset`` window, measured with HIP
 * events recorded on the launch stream (for a graph: around the graph launch,
 * the exact tier included) when timing is enabled (tp_timing_enable(1)).
 * Returns the launches counted. */
int tp_timing_enable(int32_t on);
int tp_timing_reset(void);
int tp_timing_read(double *avg_ms, int64_t *launches);

/* Release per-device internal state (workspaces, plans, graphs, side streams
 * and their events, pair-sum flags); later calls recreate what they need.  The
 * allocation-free entry point's device array stays until the process ends. */
int tp_release(void);

const char *tp_strerror(int status);
int tp_version(void);

/* ------------------------------------------------------------------------
 * Energy test (Sect. 2.2, eq. (2); background-subtracted form Sect. 3, eq. (3))
 *
 * The statistic compares two samples through psi_ij = exp(-d_ij^2 / 2 sigma^2),
 * d_ij the Euclidean distance between events in phase-space coordinates
 * (invariant masses, Sect. 4.2 Table 1).  The device computes, for a 0/1 column
 * matrix G [n][ncols] (one column per sample indicator: the observed split,
 * each permutation of it, ...) whose leading ``nrow`` columns double as row
 * weights, the pair sums
 *     sums[c][0]     = sum_i sum_{j != i} G[i][c] psi_ij G[j][c]
 *     sums[c][1 + q] = sum_i sum_{j != i} G[i][q] psi_ij G[j][c],   q < nrow,
 * from which the host functions form T of eq. (2) per column and T of eq. (3)
 * per permutation.  Permutations are the caller's: random numbers are inputs.
 * ------------------------------------------------------------------------ */

/* Invariant masses (times ``scale``, e.g. 1e-3 for MeV -> GeV) of ``ncoord`` (1..8)
 * slot bit masks (1..15) per event: coords [ncoord][ld] float32, device, written.
 * ev as for tp_compute (the tag is not read).  Async on ``stream``.
 * relabel: TP_RELABEL_NONE, or TP_RELABEL_D4PI for D0 -> pi+ pi- pi+ pi- with
 * the slots in charge order (+ - + -): before the masses are formed, the
 * pi+ pi- pair of largest invariant mass becomes pi3 pi4 (slots 2, 3), which
 * fixes the labels of all four pions (Sect. 4.2; Table 1 then selects masks
 * m12, m14, m23, m123, m124, i.e. 0x3, 0x9, 0x6, 0x7, 0xB).  The mass
 * comparisons are certified (float64 with an error bound, exact integers
 * otherwise); equal masses go to the first pair of (2,3), (0,1), (0,3), (2,1). */
enum { TP_RELABEL_NONE = 0, TP_RELABEL_D4PI = 1 };
int tp_coords(const tp_events *ev, const int32_t *masks, int32_t ncoord, double scale, int32_t relabel,
              float *coords, int64_t ld, void *stream);

/* Pair sums above.  coords [dims][ld] float32 (device, dims 1..8, ld >= n);
 * cols [n][ncols] uint8 0/1 (device, row-major, 16-byte aligned, ncols 32, 64
 * or 128; its first nrow (0..3) columns are also the row weights); sums
 * [ncols][1 + nrow] float64 (device, accumulated: zero it once).  sigma > 0.
 * psi is formed for pairs j > i only (psi is symmetric): the squared
 * distance as a dot product of (coordinates - centre, squared norm) vectors
 * split into float16 terms on the matrix cores (centre: mean of the first 256
 * events; rounding grows with the squared distance of the events from it, in
 * units of sigma, and is of random sign), then the hardware exp2.  A range
 * check runs first: if any event lies farther than ~37 sigma from the centre
 * (scaled squared distance > 1024) or is not finite, the launch instead forms
 * the distances of every chunk of pairs that holds such an event as direct
 * float32 differences of the coordinates (slower, accurate at any distance).
 * Calls on one stream share a two-word device flag of the library.
 * psi enters the matrix cores again as two float16 terms (truncation
 * of psi * 2^14 and of the remainder: together within 2^-20 of psi,
 * relative); the 0/1 columns are exact in float16, products are accumulated
 * in float32 over 1024 j and then in float64.  Sums are accurate to ~1e-5
 * relative (typically ~1e-6) for coordinates whose spread is a few sigma.
 * Async on ``stream``. */
int tp_pairsums(const float *coords, int32_t dims, int64_t ld, int64_t n, double sigma, const uint8_t *cols,
                int32_t ncols, int32_t nrow, double *sums, void *stream);

/* eq. (2) per column c from host copies of the sums: sample X = events with
 * G[i][c] = 1 (nx[c] of them), Xbar = the other n - nx[c];
 * needs an all-ones column ``ones_col`` (< nrow, so that it is also row weight
 * ``ones_row`` = ones_col).
 * T[c] = NaN when a sample has fewer than two events. */
int tp_energy_eq2(const double *sums, int32_t ncols, int32_t nrow, int32_t ones_row, int32_t ones_col,
                  const int64_t *nx, int64_t n, double *T);

/* eq. (3) per permutation k from host copies of the sums.  Columns: col_main /
 * col_bkg mark the main and background samples (both flavours); per
 * permutation perm_cols[3k..3k+2] = (a, beta, gamma): a = main events of flavour
 * X, beta = background-sample events of flavour X, gamma = a + beta.  Row
 * weights row_main / row_bkg (< nrow) are the same columns as col_main / col_bkg.
 * n_main, n_main_bar: main-sample sizes per flavour; n_bkg, n_bkg_bar:
 * background-sample sizes (b_s, b_s bar); b, b_bar: background events in the
 * main samples.  T[k] for k < nperm. */
int tp_energy_eq3(const double *sums, int32_t ncols, int32_t nrow, int32_t col_main, int32_t col_bkg,
                  int32_t row_main, int32_t row_bkg, const int32_t *perm_cols, int32_t nperm, int64_t n_main,
                  int64_t n_main_bar, int64_t n_bkg, int64_t n_bkg_bar, double b, double b_bar, double *T);

#ifdef __cplusplus
}
#endif
#endif /* TPASYM_H */
