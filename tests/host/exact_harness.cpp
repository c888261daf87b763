// Host build of the exact tier's per-event decision (tp_exact.h), for CPU tests.
#include <stdint.h>

#include "tp_dword.h"
#include "tp_exact.h"

extern "C" int hx_decide(const double *comps, int is_f32, int tag, int sigma, int naxes, const int32_t *kind,
                         const int32_t *nbins, const int32_t *slots, const double *e0, const double *e1,
                         int *bin)
{
    int64_t mant[4][4];
    int ex[4][4];
    bool finite = true;
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 4; ++c) {
            const double v = comps[s * 4 + c];
            if (!(v == v) || v - v != 0.0) finite = false;
            if (is_f32) tpx::decode_f32((float)v, mant[s][c], ex[s][c]);
            else tpx::decode_f64(v, mant[s][c], ex[s][c]);
        }
    const double *eds[2] = { e0, e1 };
    return tpx::decide(mant, ex, finite, tag, is_f32 ? 136 : 107, sigma, naxes, kind, nbins, slots, eds, *bin);
}

// Double-word tier on the same event; returns 7 when it does not decide.
extern "C" int hx_decide_dw(const double *comps, int tag, int sigma, int naxes, const int32_t *kind,
                            const int32_t *nbins, const int32_t *slots, const double *e0, const double *e1,
                            int *bin)
{
    double x[4][4];
    for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 4; ++c) x[s][c] = comps[s * 4 + c];
    const double *eds[2] = { e0, e1 };
    return tpw::decide_dw(x, tag, sigma, naxes, kind, nbins, slots, eds, *bin);
}
