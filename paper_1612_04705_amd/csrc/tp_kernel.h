// Shared host/device layout of the T-odd pass launch (internal to libtpasym).
#pragma once

#include <stdint.h>

namespace tpk {

enum { MAXBINS = 1024, NSTAT = 8 };
enum { CLS_I = 0, CLS_II = 1, CLS_III = 2, CLS_IV = 3, CLS_ZERO = 4, CLS_INVALID = 5,
       CLS_UNRESOLVED = 6, CLS_DEFER = 7 };
enum { AX_ABSPHI = 0, AX_MASS = 1, AX_ABSCOS = 2, AX_NONE = 3 };
// stats slots (same order as tp_stats)
enum { ST_EVENTS = 0, ST_ZERO = 1, ST_INVALID = 2, ST_OOR = 3, ST_TIER2 = 4, ST_TIER3 = 5,
       ST_UNRESOLVED = 6 };

// Per-sample descriptor, device resident.  Particles are stored in "kernel
// order": kernel slot t holds channel slot planes[t], so the plane angle is
// always between kernel planes (0,1) and (2,3).
struct KSample {
    const void *p[16];        // [kslot * 4 + c]
    const int8_t *tag;
    int64_t n;                // n * element size < 2^32: the kernels index the arrays with
                              // 32-bit offsets (the host splits larger samples)
    int64_t vstart;           // start in the virtual event space (multiple of 256)
    uint64_t *counts;         // [(nbtot + 1) * 4]
    uint64_t *stats;          // [NSTAT]
    int8_t *cls_out;          // optional per-event class (tp_compute)
    double *ct_out;           // optional per-event C_T^inv
    int32_t sigma;            // C_T^inv = sigma * det[kernel rows 0..3]
    int32_t naxes;
    int32_t kind[2];
    int32_t nbins[2];
    int32_t slots[2];         // MASS: kernel-order bit mask; ABSCOS: kernel slot
    int32_t eoff[2];          // offset (doubles) of the axis' edge data in the edge table
    int32_t nbtot;            // product of nbins (0 if naxes == 0)
    int32_t vec;              // 1: all arrays 16-byte aligned (vector loads allowed)
    double guess_lo[2];       // MASS: first edge, for the uniform-grid guess
    double guess_inv[2];      // MASS: 1 / bin width
    int32_t olo;              // identical particles in kernel slots olo, olo + 2 (olo 0 or 1; -1: none)
    int32_t odir;             // +1: the faster goes to kernel slot olo, -1: to olo + 2
};

// Launch parameters (kernel argument).  One pass launch covers the samples
// [sbeg, send) -- all of one binning scheme -- whose virtual events are
// [vbeg, vend); the deferral list and the edge table are shared by all.
struct KParams {
    const KSample *samples;
    int32_t sbeg, send;
    int32_t lds_copies;
    int32_t hist_stride;      // uint32 counters per LDS copy
    int32_t edge_doubles;     // doubles of edge data cached in LDS per segment (max over samples)
    int32_t mode;             // 0 = counts, 1 = per-event outputs
    int64_t range;            // virtual events per workgroup (multiple of the tile, >= 256)
    int64_t vbeg, vend;       // virtual event range of this launch
    const double *edges;      // edge table
    uint64_t *xlist;          // deferred events: (stage << 60) | (sample << 40) | event
    uint32_t *xcount;         // number of listed events
    uint32_t *xdone;          // finished exact-tier workgroups (last one resets)
    uint32_t xcap;
};

// Edge data layout per axis (at eoff):
//   ABSPHI, ABSCOS: the nbins + 1 edge values
//   MASS:           nbins + 1 lower bounds of e_k^2, then nbins + 1 upper bounds,
//                   then the nbins + 1 edge values (for the exact tier)
constexpr int edge_doubles(int kind, int nbins)
{
    return kind == AX_MASS ? 3 * (nbins + 1) : (nbins + 1);
}

}  // namespace tpk
