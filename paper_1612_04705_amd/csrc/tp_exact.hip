// Last tiers of the T-odd pass: the events the float64 tier could not decide,
// taken from the work list and decided first in certified double-word
// arithmetic (tp_dword.h) and, if that does not settle them, in exact integer
// arithmetic (tp_exact.h): validity, sign of the triple product (Sect. 5,
// eq. (4)) and every bin-edge comparison.  Results are added to the sample's counters with
// device-scope atomics; the last workgroup clears the list for the next launch.
#include <hip/hip_runtime.h>

#define TP_HD __host__ __device__
#include "tp_dword.h"
#include "tp_exact.h"
#include "tp_kernel.h"

namespace tpk {
namespace {

__device__ __forceinline__ double dabs(double x) { return __builtin_fabs(x); }

// Rest-frame energy order of kernel slots lo, lo + 2 in float64 (the pass's
// test: s = P.(p_lo - p_hi) against 8.1u W (w_lo + w_hi)): +1 if p_lo is
// faster, -1 if slower, 0 if the bound does not settle it.
__device__ __forceinline__ int order_f64(const double (&x)[4][4], int lo)
{
    const int hi = lo + 2;
    double P[4], w[4], W = 0.0;
    for (int c = 0; c < 4; ++c) P[c] = (x[0][c] + x[1][c]) + (x[2][c] + x[3][c]);
    for (int k = 0; k < 4; ++k) {
        w[k] = (dabs(x[k][0]) + dabs(x[k][1])) + (dabs(x[k][2]) + dabs(x[k][3]));
        W += w[k];
    }
    double d[4];
    for (int c = 0; c < 4; ++c) d[c] = x[lo][c] - x[hi][c];
    const double sv = fma(-P[3], d[3], fma(-P[2], d[2], fma(-P[1], d[1], P[0] * d[0])));
    const double bound = fma((8.2 * 0x1p-53) * W, w[lo] + w[hi], 0x1p-1000);
    if (!(dabs(sv) > bound)) return 0;
    return sv > 0.0 ? 1 : -1;
}

// ------------------------------------------------------------------ exact tier
template <typename Tin, int MODE>
__global__ __launch_bounds__(64) void tp_exact_kernel(const KParams kp)
{
    const uint32_t cnt = __atomic_load_n(kp.xcount, __ATOMIC_RELAXED);
    const uint32_t n = cnt < kp.xcap ? cnt : kp.xcap;
    for (uint32_t it = blockIdx.x * blockDim.x + threadIdx.x; it < n; it += gridDim.x * blockDim.x) {
        const uint64_t ent = kp.xlist[it];
        const int s = (int)((ent >> 40) & 0xfffff);
        const int64_t i = (int64_t)(ent & ((1ull << 40) - 1));
        const KSample &S = kp.samples[s];
        const int tag = S.tag[i];
        double xv[4][4];
        bool finite = true;
        for (int k = 0; k < 4; ++k)
            for (int c = 0; c < 4; ++c) {
                xv[k][c] = (double)reinterpret_cast<const Tin *>(S.p[k * 4 + c])[i];
                if (!isfinite(xv[k][c])) finite = false;
            }
        const double *eds[2] = { nullptr, nullptr };
        for (int a = 0; a < S.naxes && a < 2; ++a)
            eds[a] = kp.edges + S.eoff[a] + (S.kind[a] == AX_MASS ? 2 * (S.nbins[a] + 1) : 0);
        const int nax = MODE == 0 ? S.naxes : 0;
        const int span = sizeof(Tin) == 4 ? 136 : 107;
        // identical particles: exact rest-frame energy order first (an exact
        // tie keeps the stored order), then every decision on the ordered rows
        bool order_unres = false;
        int osg = (finite && S.olo >= 0) ? order_f64(xv, S.olo) : 0;
        if (osg != 0 && osg * S.odir < 0) {
            for (int c = 0; c < 4; ++c) {
                const double t = xv[S.olo][c];
                xv[S.olo][c] = xv[S.olo + 2][c];
                xv[S.olo + 2][c] = t;
            }
        }
        if (finite && S.olo >= 0 && osg == 0) {
            int64_t om[4][4];
            int oe[4][4];
            for (int k = 0; k < 4; ++k)
                for (int c = 0; c < 4; ++c) {
                    if constexpr (sizeof(Tin) == 4) tpx::decode_f32((float)xv[k][c], om[k][c], oe[k][c]);
                    else tpx::decode_f64(xv[k][c], om[k][c], oe[k][c]);
                }
            const int sg = tpx::order_sign(om, oe, span, S.olo, S.olo + 2);
            if (sg == 2) {
                order_unres = true;
            } else if (sg * S.odir < 0) {
                for (int c = 0; c < 4; ++c) {
                    const double t = xv[S.olo][c];
                    xv[S.olo][c] = xv[S.olo + 2][c];
                    xv[S.olo + 2][c] = t;
                }
            }
        }
        int bin = -1;
        int cls = order_unres ? (int)CLS_UNRESOLVED
                : finite ? tpw::decide_dw(xv, tag, S.sigma, nax, S.kind, S.nbins, S.slots, eds, bin)
                         : (int)tpw::W_UNCERTAIN;
        if (cls == tpw::W_UNCERTAIN) {
            int64_t mant[4][4];
            int ex[4][4];
            for (int k = 0; k < 4; ++k)
                for (int c = 0; c < 4; ++c) {
                    if constexpr (sizeof(Tin) == 4) tpx::decode_f32((float)xv[k][c], mant[k][c], ex[k][c]);
                    else tpx::decode_f64(xv[k][c], mant[k][c], ex[k][c]);
                }
            cls = tpx::decide(mant, ex, finite, tag, span, S.sigma, nax, S.kind,
                              S.nbins, S.slots, eds, bin);
        }
        const bool unres = cls == CLS_UNRESOLVED;
        if (MODE == 1) {
            S.cls_out[i] = (int8_t)cls;
            if (S.ct_out) {
                const double est = S.ct_out[i];
                double mag = dabs(est);
                if (mag == 0.0 || !(mag < 1e308)) mag = 0x1p-1074;
                S.ct_out[i] = cls == CLS_ZERO ? 0.0
                            : (cls < 4 ? (((cls == CLS_I) || (cls == CLS_IV)) ? mag : -mag) : est);
            }
        }
        unsigned long long *st = (unsigned long long *)S.stats;
        if (cls == CLS_UNRESOLVED) {
            atomicAdd(st + ST_UNRESOLVED, 1ull);
        } else if (cls == CLS_ZERO) {
            atomicAdd(st + ST_ZERO, 1ull);
        } else if (cls == CLS_INVALID) {
            atomicAdd(st + ST_INVALID, 1ull);
        } else if (MODE == 0) {
            if (S.counts) {
                atomicAdd((unsigned long long *)S.counts + cls, 1ull);
                if (S.naxes > 0 && bin >= 0)
                    atomicAdd((unsigned long long *)S.counts + (1 + bin) * 4 + cls, 1ull);
            }
            if (S.naxes > 0 && bin < 0) atomicAdd(st + ST_OOR, 1ull);
        }
    }
    // the last workgroup to finish clears the list for the next launch
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t t = atomicAdd(kp.xdone, 1u);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (last && threadIdx.x == 0) {
        *kp.xcount = 0u;
        *kp.xdone = 0u;
        __threadfence();
    }
}

}  // namespace

hipError_t launch_exact(int dtype, int mode, const KParams &kp, int grid, hipStream_t st)
{
#define TP_X(T, M) hipLaunchKernelGGL((tp_exact_kernel<T, M>), dim3(grid), dim3(64), 0, st, kp)
    if (dtype == 0) {
        if (mode == 0) TP_X(float, 0);
        else TP_X(float, 1);
    } else {
        if (mode == 0) TP_X(double, 0);
        else TP_X(double, 1);
    }
#undef TP_X
    return hipGetLastError();
}

}  // namespace tpk
