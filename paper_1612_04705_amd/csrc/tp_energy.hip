// Energy-test pair sums on gfx950 (Sect. 2.2 eq. (2), Sect. 4 eq. (3)).
//
// For coordinates y_i (D <= 8 per event), psi_ij = exp(-|y_i - y_j|^2 / 2 sigma^2)
// for i != j (0 on the diagonal) and a 0/1 column matrix G [n][C], the kernel
// accumulates for every column c
//   sums[c][0]     = sum_i sum_{j != i} G[i][c]      psi_ij G[j][c]
//   sums[c][1 + r] = sum_i sum_{j != i} w_r(i)       psi_ij G[j][c]
// with row weights w_r = G[.][rowcol[r]] (or 1 when rowcol[r] < 0).  Every
// within-sample and cross-sample sum of eq. (2) and eq. (3) -- for the observed
// split and every permutation at once -- is a combination of these.
//
// V = Psi G is a dense contraction over j, done by MFMA (v_mfma_f32_32x32x2f32):
// each lane produces one psi per step (VALU: distance, exp2), the matrix core
// multiplies the 32 x 2 psi tile by the 2 x 32 column tile.  j streams through
// LDS in chunks; at each chunk end the float32 tile is reduced per column into
// float64 partials, so float32 only ever sums 2 * JC terms.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tp_energy.h"

namespace tpe {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));

constexpr int ROWS = 128;     // rows i per workgroup (4 waves x 32)
constexpr int JC = 256;       // j per LDS chunk

template <int NT>
__global__ __launch_bounds__(256) void tp_pairsum_kernel(const EParams p)
{
    constexpr int C = 32 * NT;
    __shared__ float ys[MAXD][JC];
    __shared__ uint8_t gs[JC * C];
    __shared__ uint8_t gi[ROWS * C];
    __shared__ float wi[MAXR][ROWS];
    __shared__ double red[C][1 + MAXR];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int h = lane >> 5;                    // which k (j) of the step this lane feeds
    const int col = lane & 31;
    const int64_t ib = (int64_t)blockIdx.x * ROWS;
    const int64_t i = ib + wave * 32 + col;     // the row whose psi this lane computes
    const int D = p.D, R = p.R;

    // this workgroup's rows of G and the row weights; zero beyond n
    for (int e = tid; e < ROWS * C; e += 256) {
        const int64_t r = ib + e / C;
        gi[e] = r < p.n ? p.G[r * C + (e % C)] : (uint8_t)0;
    }
    for (int e = tid; e < MAXR * ROWS; e += 256) {
        const int rr = e / ROWS;
        const int64_t r = ib + e % ROWS;
        float w = 0.0f;
        if (rr < R && r < p.n) w = p.rowcol[rr] < 0 ? 1.0f : (float)p.G[r * C + p.rowcol[rr]];
        wi[rr][e % ROWS] = w;
    }
    for (int e = tid; e < C * (1 + MAXR); e += 256) (&red[0][0])[e] = 0.0;
    float yi[MAXD];
#pragma unroll
    for (int d = 0; d < MAXD; ++d) yi[d] = (d < D && i < p.n) ? p.Y[d * p.ldY + i] : 0.0f;

    double part[NT][1 + MAXR];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q <= MAXR; ++q) part[t][q] = 0.0;

    for (int64_t j0 = 0; j0 < p.n; j0 += JC) {
        __syncthreads();
        for (int e = tid; e < MAXD * JC; e += 256) {
            const int d = e / JC;
            const int64_t j = j0 + e % JC;
            ys[d][e % JC] = (d < D && j < p.n) ? p.Y[d * p.ldY + j] : 0.0f;
        }
        for (int e = tid; e < JC * C; e += 256) {
            const int64_t j = j0 + e / C;
            gs[e] = j < p.n ? p.G[j * C + (e % C)] : (uint8_t)0;
        }
        __syncthreads();
        f16v acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f16v{};
#pragma unroll 2
        for (int jj = 0; jj < JC; jj += 2) {
            const int jl = jj + h;
            float d2 = 0.0f;
#pragma unroll
            for (int d = 0; d < MAXD; ++d) {
                if (d < D) {
                    const float df = yi[d] - ys[d][jl];
                    d2 = fmaf(df, df, d2);
                }
            }
            float psi = __builtin_amdgcn_exp2f(d2 * p.kexp);
            psi = (j0 + jl == i) ? 0.0f : psi;    // j != i; rows beyond n carry zero weights
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const float b = (float)gs[jl * C + 32 * t + col];
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(psi, b, acc[t], 0, 0, 0);
            }
        }
        // reduce the chunk per column: lane (col, h) holds column 32 t + col for
        // rows 8 (r / 4) + 4 h + r % 4 of this wave's 32
        float s0[NT], sr[NT][MAXR];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            s0[t] = 0.0f;
#pragma unroll
            for (int q = 0; q < MAXR; ++q) sr[t][q] = 0.0f;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = wave * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
            float w[MAXR];
#pragma unroll
            for (int q = 0; q < MAXR; ++q) w[q] = wi[q][row];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const float v = acc[t][r];
                s0[t] = fmaf((float)gi[row * C + 32 * t + col], v, s0[t]);
#pragma unroll
                for (int q = 0; q < MAXR; ++q) sr[t][q] = fmaf(w[q], v, sr[t][q]);
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            part[t][0] += (double)s0[t];
#pragma unroll
            for (int q = 0; q < MAXR; ++q) part[t][1 + q] += (double)sr[t][q];
        }
    }
    // combine the two row halves of each column, then the four waves, then workgroups
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q <= MAXR; ++q) {
            double v = part[t][q];
            v += __shfl_xor(v, 32);
            if (h == 0 && (q == 0 || q <= R)) atomicAdd(&red[32 * t + col][q], v);
        }
    __syncthreads();
    for (int e = tid; e < C * (1 + R); e += 256) {
        const int c = e / (1 + R), q = e % (1 + R);
        if (c < p.C) atomicAdd(&p.sums[(int64_t)c * (1 + R) + q], red[c][q]);
    }
}

template <int NT>
void launch_nt(const EParams &p, hipStream_t st)
{
    const int64_t grid = (p.n + ROWS - 1) / ROWS;
    hipLaunchKernelGGL(tp_pairsum_kernel<NT>, dim3((unsigned)grid), dim3(256), 0, st, p);
}

// Invariant mass of the slots in a mask, per event (Sect. 4 coordinates).
template <typename Tin>
__global__ void tp_coords_kernel(CParams c)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= c.n) return;
    const Tin *const *P = reinterpret_cast<const Tin *const *>(c.p);
    for (int k = 0; k < c.ncoord; ++k) {
        double S[4] = { 0.0, 0.0, 0.0, 0.0 };
        for (int s = 0; s < 4; ++s)
            if (c.masks[k] & (1 << s))
                for (int q = 0; q < 4; ++q) S[q] += (double)P[s * 4 + q][e];
        const double m2 = S[0] * S[0] - S[1] * S[1] - S[2] * S[2] - S[3] * S[3];
        c.out[(int64_t)k * c.ldo + e] = (float)(m2 > 0.0 ? sqrt(m2) * c.scale : 0.0);
    }
}

}  // namespace

hipError_t launch_pairsums(const EParams &p, hipStream_t st)
{
    const int nt = p.C / 32;
    switch (nt) {
    case 1: launch_nt<1>(p, st); break;
    case 2: launch_nt<2>(p, st); break;
    case 4: launch_nt<4>(p, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_coords(const CParams &c, int dtype, hipStream_t st)
{
    const int64_t grid = (c.n + 255) / 256;
    if (dtype == 0) hipLaunchKernelGGL(tp_coords_kernel<float>, dim3((unsigned)grid), dim3(256), 0, st, c);
    else hipLaunchKernelGGL(tp_coords_kernel<double>, dim3((unsigned)grid), dim3(256), 0, st, c);
    return hipGetLastError();
}

}  // namespace tpe
