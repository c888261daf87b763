// Energy-test pair sums on gfx950 (Sect. 2.2 eq. (2), Sect. 4 eq. (3)).
//
// For coordinates y_i (D <= 8 per event), psi_ij = exp(-|y_i - y_j|^2 / 2 sigma^2)
// for i != j (0 on the diagonal) and a 0/1 column matrix G [n][C], the kernel
// accumulates for every column c
//   sums[c][0]     = sum_i sum_{j != i} G[i][c] psi_ij G[j][c]
//   sums[c][1 + q] = sum_i sum_{j != i} G[i][q] psi_ij G[j][c],   q < R,
// i.e. the leading R columns double as row weights.  Every within-sample and
// cross-sample sum of eq. (2) and eq. (3) -- for the observed split and every
// permutation at once -- is a combination of these.
//
// psi is symmetric, so only pairs j > i are formed: the first sum is twice its
// upper-triangle part, and the second is the upper-triangle part of
// sum w_i psi_ij G_jc plus the transposed term sum_i G_ic (Psi_upper w_q)_i,
// where (Psi_upper w_q) is column q of the same product.
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
constexpr int JC = 256;       // j per LDS chunk (one per thread when staging)

template <int NT>
struct Smem {
    static constexpr int C = 32 * NT;
    float ys[JC][MAXD];                 // staged coordinates of a j chunk (padded with zeros)
    uint8_t gs[JC * C];                 // staged columns of the chunk
    uint8_t gi[ROWS * C];               // columns of this block's rows
    float rw[ROWS][8];                  // per row: weights G[i][q] (0..2), chunk (Psi_upper G)[i][q] (4..6)
    double red[C][1 + MAXR];            // workgroup totals
};

// psi products of one staged chunk into the float32 tiles: lane (col, h) forms
// psi for row i (its yi) and local j = jj + h, the matrix core adds the 32 x 2
// psi tile times the 2 x 32 column tile t.  MASK keeps only local j > rel
// (rel = i - j0), needed only in the chunk that holds the diagonal.
template <int NT, int DP, bool MASK>
__device__ __forceinline__ void chunk_products(const Smem<NT> &sm, const float (&yi)[DP], int rel, f16v (&acc)[NT])
{
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    constexpr int C = 32 * NT;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    const int col = lane & 31;
#pragma unroll 2
    for (int jj = 0; jj < JC; jj += 2) {
        const int jl = jj + h;
        float yj[8];
        const f32x4 ya = reinterpret_cast<const f32x4 *>(&sm.ys[jl][0])[0];
        yj[0] = ya.x; yj[1] = ya.y; yj[2] = ya.z; yj[3] = ya.w;
        if (DP > 4) {
            const f32x4 yb = reinterpret_cast<const f32x4 *>(&sm.ys[jl][0])[1];
            yj[4] = yb.x; yj[5] = yb.y; yj[6] = yb.z; yj[7] = yb.w;
        }
        float d2 = 0.0f;
#pragma unroll
        for (int d = 0; d < DP; ++d) {
            const float df = yi[d] - yj[d];
            d2 = fmaf(df, df, d2);
        }
        float psi = __builtin_amdgcn_exp2f(-d2);
        if (MASK) psi = (jl > rel) ? psi : 0.0f;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const float b = (float)sm.gs[jl * C + 32 * t + col];
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(psi, b, acc[t], 0, 0, 0);
        }
    }
}

// One block of ROWS rows i against every j > i (upper triangle).  Coordinates
// enter scaled by yscale, so that psi = 2^-(scaled distance)^2.
template <int NT, int DP>
__device__ __forceinline__ void pair_block(const EParams &p, Smem<NT> &sm, int64_t ib, double (&part)[NT][1 + MAXR])
{
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    typedef float f32x4 __attribute__((ext_vector_type(4)));
    constexpr int C = 32 * NT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int h = lane >> 5;
    const int col = lane & 31;
    const int64_t i = ib + wave * 32 + col;     // the row whose psi this lane computes
    const int R = p.R;

    __syncthreads();
    for (int e = tid; e < ROWS * C / 16; e += 256) {
        const int64_t r = ib + (e * 16) / C;
        u32x4 w = u32x4{ 0u, 0u, 0u, 0u };
        if (r < p.n) w = reinterpret_cast<const u32x4 *>(p.G + ib * C)[e];
        reinterpret_cast<u32x4 *>(sm.gi)[e] = w;
    }
    if (tid < ROWS) {
        const int64_t r = ib + tid;
#pragma unroll
        for (int q = 0; q < MAXR; ++q)
            sm.rw[tid][q] = (q < R && r < p.n) ? (float)p.G[r * C + q] : 0.0f;
#pragma unroll
        for (int q = 3; q < 8; ++q) sm.rw[tid][q] = 0.0f;
    }
    float yi[DP];
#pragma unroll
    for (int d = 0; d < DP; ++d) yi[d] = (d < p.D && i < p.n) ? p.Y[d * p.ldY + i] * p.yscale : 0.0f;

    const int64_t jfirst = ib - ib % JC;        // the chunk that holds the diagonal
    for (int64_t j0 = jfirst; j0 < p.n; j0 += JC) {
        __syncthreads();
        {   // coordinates: one j per thread (JC == 256 threads), padded with zeros
            const int64_t j = j0 + tid;
            float v[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) v[d] = (d < p.D && j < p.n) ? p.Y[d * p.ldY + j] * p.yscale : 0.0f;
            reinterpret_cast<f32x4 *>(&sm.ys[tid][0])[0] = f32x4{ v[0], v[1], v[2], v[3] };
            reinterpret_cast<f32x4 *>(&sm.ys[tid][0])[1] = f32x4{ v[4], v[5], v[6], v[7] };
        }
        // columns: 16-byte loads of whole rows (C is a multiple of 32, rows 16-byte aligned)
        for (int e = tid; e < JC * C / 16; e += 256) {
            const int64_t j = j0 + (e * 16) / C;
            u32x4 w = u32x4{ 0u, 0u, 0u, 0u };
            if (j < p.n) w = reinterpret_cast<const u32x4 *>(p.G + j0 * C)[e];
            reinterpret_cast<u32x4 *>(sm.gs)[e] = w;
        }
        __syncthreads();
        f16v acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = f16v{};
        // rows beyond n carry zero weights and j beyond n zero columns: only j <= i needs a mask
        if (j0 == jfirst) chunk_products<NT, DP, true>(sm, yi, (int)(i - j0), acc);
        else chunk_products<NT, DP, false>(sm, yi, 0, acc);
        // Reduce the chunk.  Lane (col, h) holds column 32 t + col for rows
        // 8 (r / 4) + 4 h + r % 4 of this wave's 32.  The leading R columns are
        // the row weights; their values (Psi_upper w_q)_i go through LDS so that
        // every column can take the transposed term sum_i G_ic (Psi_upper w_q)_i.
        if (col < R) {
#pragma unroll
            for (int r = 0; r < 16; ++r) sm.rw[wave * 32 + 8 * (r >> 2) + 4 * h + (r & 3)][4 + col] = acc[0][r];
        }
        __syncthreads();
        float s0[NT], s1[NT], s2[NT], s3[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) s0[t] = s1[t] = s2[t] = s3[t] = 0.0f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = wave * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
            const f32x4 wq = reinterpret_cast<const f32x4 *>(&sm.rw[row][0])[0];
            const f32x4 vq = reinterpret_cast<const f32x4 *>(&sm.rw[row][0])[1];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const float v = acc[t][r];
                const float g = (float)sm.gi[row * C + 32 * t + col];
                s0[t] = fmaf(g, v, s0[t]);
                s1[t] = fmaf(wq.x, v, fmaf(g, vq.x, s1[t]));
                s2[t] = fmaf(wq.y, v, fmaf(g, vq.y, s2[t]));
                s3[t] = fmaf(wq.z, v, fmaf(g, vq.z, s3[t]));
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            part[t][0] += 2.0 * (double)s0[t];       // diagonal-type sums are symmetric
            part[t][1] += (double)s1[t];
            part[t][2] += (double)s2[t];
            part[t][3] += (double)s3[t];
        }
    }
}

// Workgroup g takes row blocks g and nb - 1 - g: together about n pairs per row.
template <int NT, int DP>
__global__ __launch_bounds__(256) void tp_pairsum_kernel(const EParams p)
{
    constexpr int C = 32 * NT;
    __shared__ __align__(16) Smem<NT> sm;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int h = lane >> 5;
    const int col = lane & 31;
    const int64_t nb = (p.n + ROWS - 1) / ROWS;
    for (int e = tid; e < C * (1 + MAXR); e += 256) (&sm.red[0][0])[e] = 0.0;
    double part[NT][1 + MAXR];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q <= MAXR; ++q) part[t][q] = 0.0;
    const int64_t b1 = blockIdx.x, b2 = nb - 1 - (int64_t)blockIdx.x;
    for (int k = 0; k < (b2 > b1 ? 2 : 1); ++k) pair_block<NT, DP>(p, sm, (k == 0 ? b1 : b2) * ROWS, part);
    // combine the two row halves of each column, then the four waves, then workgroups
    const int R = p.R;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q <= MAXR; ++q) {
            double v = part[t][q];
            v += __shfl_xor(v, 32);
            if (h == 0 && q <= R) atomicAdd(&sm.red[32 * t + col][q], v);
        }
    __syncthreads();
    for (int e = tid; e < C * (1 + R); e += 256) {
        const int c = e / (1 + R), q = e % (1 + R);
        if (c < p.C) atomicAdd(&p.sums[(int64_t)c * (1 + R) + q], sm.red[c][q]);
    }
}

template <int NT, int DP>
void launch_ntd(const EParams &p, hipStream_t st)
{
    const int64_t nb = (p.n + ROWS - 1) / ROWS;
    const int64_t grid = (nb + 1) / 2;
    hipLaunchKernelGGL((tp_pairsum_kernel<NT, DP>), dim3((unsigned)grid), dim3(256), 0, st, p);
}

template <int NT>
void launch_nt(const EParams &p, hipStream_t st)
{
    switch (p.D) {   // coordinates per event, padded up to the next instantiated count
    case 1: case 2: launch_ntd<NT, 2>(p, st); break;
    case 3: case 4: launch_ntd<NT, 4>(p, st); break;
    case 5: launch_ntd<NT, 5>(p, st); break;
    case 6: launch_ntd<NT, 6>(p, st); break;
    default: launch_ntd<NT, 8>(p, st); break;
    }
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
