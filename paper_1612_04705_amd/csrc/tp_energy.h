// Launch layout of the energy-test kernels (internal to libtpasym).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tpe {

enum { MAXD = 8, MAXR = 3 };

// Pair-sum launch: coordinates Y [D][ldY] (float32, device), columns G [n][C]
// (uint8 0/1, device, 16-byte aligned, C 32, 64 or 128), the leading R columns
// also row weights, output sums [C][1 + R] (float64, device, +=).
struct EParams {
    const float *Y;
    int64_t ldY;
    int64_t n;
    int32_t D, C, R;
    float yscale;             // sqrt(log2(e) / (2 sigma^2)): psi = 2^-(yscale d)^2
    const uint8_t *G;
    double *sums;
    uint32_t *flag;           // device [2]: range flag, finished workgroups (zero between launches)
};

// Coordinate launch: invariant masses of ncoord slot masks per event.
struct CParams {
    const void *p[16];        // [slot * 4 + component], device
    int64_t n;
    int32_t ncoord;
    int32_t masks[MAXD];
    double scale;             // unit factor applied to the masses
    float *out;               // [ncoord][ldo], device
    int64_t ldo;
    int32_t relabel;          // 0: stored slots; 1: pi+ pi- pi+ pi- rule (largest-mass pair to slots 2, 3)
};

hipError_t launch_pairsums(const EParams &p, hipStream_t st);
hipError_t launch_coords(const CParams &c, int dtype, hipStream_t st);

}  // namespace tpe
