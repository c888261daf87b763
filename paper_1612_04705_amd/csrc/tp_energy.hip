// Energy-test pair sums on gfx950 (Sect. 2.2 eq. (2), Sect. 3 eq. (3)).
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
// Both steps run on the matrix cores.  Distances: with the scaled coordinates
// centred on the mean c of the first 256 events, v = y yscale - c, the vectors
// x_j = (v_j, |v_j|^2, 1) and x_i = (-2 v_i, 1, |v_i|^2) give
// x_i . x_j = |v_i - v_j|^2.  Each vector is split into two float16 terms
// (hi, lo: 2^-22 relative) and laid out so that one float16 contraction over
// 32 slots forms hi.hi + hi.lo + lo.hi - 14 (the -14, the psi scale, is an
// exact extra slot): two v_mfma_f32_32x32x16_f16 per 32 x 32 pairs, with exact
// products and float32 accumulation.  Then psi * 2^14 = 2^-(that) costs one
// exp2 per pair on the vector ALU.  The rounding of the squared distance is
// about 2^-22 (2 |v_i|^2 + 2 |v_j|^2) plus the float32 accumulation; centring
// keeps |v|^2 small (a few units for invariant masses at sigma ~ 0.3 GeV, ~100
// at 0.05 GeV), and the errors are of random sign, so sums over many pairs
// keep ~1e-8.  An event with |v|^2 > VMAX2 (or a non-finite one) is outside
// that range.  A range check over all events runs first and sets a device
// flag; the kernel is launched in two instantiations, of which only one does
// the work: without the flag the matrix-core form above, with it the SAFE form,
// in which every chunk of pairs that holds such an event as a row or as a
// column forms its distances as direct float32 differences of the raw
// coordinates, (y_i - y_j) yscale, squared and summed on the vector ALU
// (accurate at any distance from the centre), the matrix-core operands of
// those events being finite placeholders.
// V = Psi G is then a dense contraction over j in half precision with float32
// accumulation (v_mfma_f32_32x32x16_f16): psi * 2^14 is split into two float16
// terms hi = rtz(psi), lo = rtz(psi - hi): the difference is exact in float32
// and hi + lo is within 2^-20 (relative, from below) of the float32 psi; the
// scale keeps both terms clear of the float16 subnormals for every psi above
// 2^-17.  The 0/1 columns are exact in float16, so each product is exact and
// only the float32 accumulation rounds.  The distance tile of 32 rows x 32 j
// leaves each lane 16 psi of its row, which are the lane's half of two 32 x 16
// operand tiles; columns are staged in LDS transposed ([c][j], float16, in the
// j order those tiles use), so a lane's 8 values of one column are one 16-byte
// read.  The next chunk's columns and coordinates are loaded into registers
// while the current one is multiplied.  Every FL chunks the float32 tiles are
// reduced per column into float64 partials, so float32 only sums 2 * FL * JC
// products.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tp_energy.h"
#define TP_HD __host__ __device__
#include "tp_exact.h"

namespace tpe {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int ROWS = 128;     // rows i per workgroup (4 waves x 32)
constexpr int JC = 128;       // j per LDS chunk
constexpr int KS = 16;        // j per matrix-core step
constexpr int FL = 8;         // chunks per float32 -> float64 reduction
constexpr int GPAD = 8;       // float16 padding per staged column (spreads LDS banks)
constexpr int XS = 40;        // float16 slots per staged j vector: 32 used, 8 padding (spreads LDS banks)
constexpr float PSI_LOG2 = 14.0f;             // psi is formed scaled by 2^14
// Largest |v|^2 (squared scaled distance from the centre) of an event whose
// distances go through the matrix cores: their rounding grows as 2^-22 |v|^2,
// and float16 holds |v|^2 only below 65504.
constexpr float VMAX2 = 1024.0f;
constexpr double PSI_UNSCALE = 1.0 / 16384.0;

template <int NT, bool SAFE>
struct Smem {
    static constexpr int C = 32 * NT;
    uint16_t xh[JC][XS];                // chunk j distance operands, float16 slots (see slot())
    float cw[4][MAXD];                  // per-wave coordinate sums for the centre c
    float cen[MAXD];                    // the centre c
    uint16_t gs[C][JC + GPAD];          // columns of the chunk, [c][j], float16 0 or 1
    uint8_t gi[ROWS * C];               // columns of this block's rows, [i][c]
    float rw[ROWS][8];                  // per row: weights G[i][q] (0..2), (Psi_upper G)[i][q] (4..6)
    double red[C][1 + MAXR];            // workgroup totals
    // SAFE: raw coordinates of the block's rows and of the chunk's events (direct distances)
    float yr[SAFE ? ROWS : 1][MAXD + 1];
    float yc[SAFE ? JC : 1][MAXD];
};

// The centre's scratch of the range check (same fields as Smem).
struct CentreSmem {
    float cw[4][MAXD];
    float cen[MAXD];
};

// Centre c of the scaled coordinates: the mean of the first min(n, 256)
// events, formed in a fixed order so that every workgroup gets the same bits.
template <class SM>
__device__ __forceinline__ void centre(const EParams &p, SM &sm)
{
    const int tid = threadIdx.x;
    const int64_t m = p.n < 256 ? p.n : 256;
#pragma unroll
    for (int d = 0; d < MAXD; ++d) {
        float x = (d < p.D && tid < m) ? p.Y[d * p.ldY + tid] * p.yscale : 0.0f;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o);
        if ((tid & 63) == 0) sm.cw[tid >> 6][d] = x;
    }
    __syncthreads();
    if (tid < MAXD)
        sm.cen[tid] = ((sm.cw[0][tid] + sm.cw[1][tid]) + (sm.cw[2][tid] + sm.cw[3][tid])) / (float)(m > 0 ? m : 1);
    __syncthreads();
}

// Distance operands in float16.  A float32 vector x of KA <= 10 components is
// split into hi = f16(x) and lo = f16(x - hi) (the difference exact in
// float32, hi + lo within 2^-22 |x|); a row vector takes the 32 slots
// [hi | lo | hi | -14 | 0] and a column vector [hi | hi | lo | 1 | 0], so that
// their float16 dot product over the 32 slots, with exact products and float32
// accumulation, is hi.hi + lo.hi + hi.lo - 14: x_i . x_j - 14 up to the lo.lo
// term (2^-22 relative).
// Slot s of the row (COL = false) or column (COL = true) pattern:
template <int KA, bool COL>
__device__ __forceinline__ uint16_t slot(const uint16_t (&hi)[KA], const uint16_t (&lo)[KA], int s)
{
    if (s < KA) return hi[s];
    if (s < 2 * KA) return COL ? hi[s - KA] : lo[s - KA];
    if (s < 3 * KA) return COL ? lo[s - 2 * KA] : hi[s - 2 * KA];
    // the scale of psi, exact in float16: 1 x (-14) in the first free slot
    if (s == 3 * KA) return __builtin_bit_cast(uint16_t, COL ? (_Float16)1.0f : (_Float16)(-PSI_LOG2));
    return 0;
}

template <int KA>
__device__ __forceinline__ void split16(const float (&x)[KA], uint16_t (&hi)[KA], uint16_t (&lo)[KA])
{
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        const _Float16 a = (_Float16)x[k];
        const _Float16 b = (_Float16)(x[k] - (float)a);
        hi[k] = __builtin_bit_cast(uint16_t, a);
        lo[k] = __builtin_bit_cast(uint16_t, b);
    }
}

// Row block setup: columns and row weights of rows ib .. ib + ROWS - 1, and
// this lane's operand halves of its row's vector x_i = (-2 (y_i - c), 1,
// |y_i - c|^2) (scaled coordinates, so psi = 2^-(scaled distance)^2):
// x_i . x_j = |y_i - y_j|^2 for the chunk vectors x_j.  Lane half h holds
// slots 16 m + 8 h .. + 7 of the row pattern for the two distance steps m.
template <int NT, int NS, bool SAFE>
__device__ __forceinline__ bool setup_rows(const EParams &p, Smem<NT, SAFE> &sm, int64_t ib, u32x4 (&xi)[2])
{
    constexpr int C = 32 * NT;
    constexpr int KA = 2 * NS;
    const int tid = threadIdx.x;
    const int h = (tid >> 5) & 1;
    const int64_t i = ib + (tid >> 6) * 32 + (tid & 31);
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
            sm.rw[tid][q] = (q < p.R && r < p.n) ? (float)p.G[r * C + q] : 0.0f;
#pragma unroll
        for (int q = 3; q < 8; ++q) sm.rw[tid][q] = 0.0f;
    }
    float x[KA];
    float nrm = 0.0f;
#pragma unroll
    for (int k = 0; k < KA; ++k) x[k] = 0.0f;
    const int rl = (tid >> 6) * 32 + (tid & 31);
#pragma unroll
    for (int d = 0; d < KA - 2; ++d) {
        const float y = (d < p.D && i < p.n) ? p.Y[d * p.ldY + i] : 0.0f;
        const float v = (d < p.D && i < p.n) ? y * p.yscale - sm.cen[d] : 0.0f;
        nrm = fmaf(v, v, nrm);
        if (d < p.D) x[d] = -2.0f * v;
        if constexpr (SAFE)
            if (h == 0 && d < p.D) sm.yr[rl][d] = y;
    }
    // outside the matrix-core range (only in the SAFE form, by the range check):
    // finite placeholders; the chunks of this row block take the direct distances
    const bool far = !(nrm <= VMAX2);
    if (SAFE && far) {
        nrm = 0.0f;
#pragma unroll
        for (int k = 0; k < KA; ++k) x[k] = 0.0f;
    }
#pragma unroll
    for (int k = 0; k < KA; ++k) {
        if (k == p.D) x[k] = 1.0f;
        if (k == p.D + 1) x[k] = nrm;
    }
    uint16_t hi[KA], lo[KA];
    split16<KA>(x, hi, lo);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int s0 = 16 * m + 8 * h + 2 * w;
            xi[m][w] = (uint32_t)slot<KA, false>(hi, lo, s0) | ((uint32_t)slot<KA, false>(hi, lo, s0 + 1) << 16);
        }
    if constexpr (SAFE) return __syncthreads_or(far) != 0;
    return false;
}

// Position of local j in a staged column: bits 2 and 3 swapped, the order in
// which the distance tiles deliver psi to the matrix-core operand (see
// chunk_products).
__device__ __forceinline__ int swap23(int j) { return (j & ~12) | ((j & 4) << 1) | ((j & 8) >> 1); }

// Stage chunk j0 .. j0 + JC - 1: the vectors x_j = (y_j - c, |y_j - c|^2, 1)
// as [k][j] (padding events j >= n get y_j = c, so every psi stays finite; their
// columns are 0), and the columns transposed to [c][swap23(j)] as float16.
// Each item takes 4 rows x 16 columns (four 16-byte loads) and writes, per
// column, the 4 rows as one 8-byte word: bytes b of two rows are placed as the
// 16-bit lanes of one word (b0 | b1 << 16), and the 24-bit multiply by 0x3C00
// turns each lane's 0/1 into float16 0 or 1.0.
// One chunk in flight in registers: thread tid < JC holds the coordinates of
// event j0 + tid, thread it < ITEMS the 4 rows x 16 columns of its item.  The
// loads for chunk v + 1 are issued before chunk v is multiplied and written to
// LDS after it, so their latency hides behind the products.
template <int KA>
struct Pending {
    float y[KA - 2];
    u32x4 w[4];
};

template <int NT, int KA>
__device__ __forceinline__ void load_chunk(const EParams &p, int64_t j0, Pending<KA> &pd)
{
    constexpr int C = 32 * NT;
    constexpr int ITEMS = (JC / 4) * (C / 16);
    static_assert(ITEMS <= 256, "one item per thread");
    const int tid = threadIdx.x;
    const int64_t j = j0 + tid;
#pragma unroll
    for (int d = 0; d < KA - 2; ++d) pd.y[d] = (tid < JC && d < p.D && j < p.n) ? p.Y[d * p.ldY + j] : 0.0f;
    const int jq = (tid % (JC / 4)) * 4;
    const int cg = tid / (JC / 4);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
        const int64_t jr = j0 + jq + rr;
        pd.w[rr] = (tid < ITEMS && jr < p.n) ? *reinterpret_cast<const u32x4 *>(p.G + jr * C + 16 * cg) : u32x4{ 0u, 0u, 0u, 0u };
    }
}

template <int NT, int KA, bool SAFE>
__device__ __forceinline__ bool store_chunk(const EParams &p, Smem<NT, SAFE> &sm, int64_t j0, const Pending<KA> &pd)
{
    constexpr int C = 32 * NT;
    constexpr int ITEMS = (JC / 4) * (C / 16);
    const int tid = threadIdx.x;
    bool far = false;
    if (tid < JC) {
        const bool real = j0 + tid < p.n;   // padding events sit at the centre
        float x[KA];
        float nrm = 0.0f;
#pragma unroll
        for (int k = 0; k < KA; ++k) x[k] = 0.0f;
#pragma unroll
        for (int d = 0; d < KA - 2; ++d) {
            const float v = (d < p.D && real) ? pd.y[d] * p.yscale - sm.cen[d] : 0.0f;
            nrm = fmaf(v, v, nrm);
            if (d < p.D) x[d] = v;
            if constexpr (SAFE)
                if (d < p.D) sm.yc[tid][d] = real ? pd.y[d] : 0.0f;
        }
        far = !(nrm <= VMAX2);
        if (SAFE && far) {
            nrm = 0.0f;
#pragma unroll
            for (int k = 0; k < KA; ++k) x[k] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < KA; ++k) {
            if (k == p.D) x[k] = nrm;
            if (k == p.D + 1) x[k] = 1.0f;
        }
        uint16_t hi[KA], lo[KA];
        split16<KA>(x, hi, lo);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            u32x4 w;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int s0 = 8 * q + 2 * e;
                w[e] = (uint32_t)slot<KA, true>(hi, lo, s0) | ((uint32_t)slot<KA, true>(hi, lo, s0 + 1) << 16);
            }
            *reinterpret_cast<u32x4 *>(&sm.xh[tid][8 * q]) = w;
        }
    }
    if (tid < ITEMS) {
        const int jq = (tid % (JC / 4)) * 4;
        const int cg = tid / (JC / 4);
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int m = q & 3, wd = q >> 2;
            // byte m of the second source (first row of the pair) to bits 0..7,
            // byte m of the first source (second row) to bits 16..23, zeros elsewhere
            const uint32_t sel = (uint32_t)m | (0x0cu << 8) | ((uint32_t)(4 + m) << 16) | (0x0cu << 24);
            const uint32_t x01 = __builtin_amdgcn_perm(pd.w[1][wd], pd.w[0][wd], sel);
            const uint32_t x23 = __builtin_amdgcn_perm(pd.w[3][wd], pd.w[2][wd], sel);
            *reinterpret_cast<u32x2 *>(&sm.gs[16 * cg + q][swap23(jq)]) = u32x2{ (uint32_t)__umul24(x01, 0x3C00u), (uint32_t)__umul24(x23, 0x3C00u) };
        }
    }
    return far;
}

// psi products of one staged chunk into the float32 tiles, 32 j per step.
// The distances come from the matrix cores too: the 32 float16 slots of the
// column and row vectors (two v_mfma_f32_32x32x16_f16) give lane (col, h)
// |y_i - y_j|^2 - 14 for its row i and the 16 j = 8 (r / 4) + 4 h + r % 4,
// r < 16.  Then psi * 2^14 = 2^-(that), split into float16 hi and lo.
// Taken in pairs of r, the values for r < 8 are the lane's 8 consecutive k of
// the first 32 x 16 psi tile and r >= 8 those of the second; k = 8 h + (r % 8)
// stands for local j = 8 (r % 8 / 4) + 4 h + r % 4 (+16 for the second tile),
// which is k with bits 2 and 3 swapped, the order in which the columns are
// staged.  MASK keeps only j > rel (rel = i - j0), needed only in the chunk
// that holds the diagonal.
// DIRECT (SAFE form only): the distances of the chunk as direct float32
// differences of the raw coordinates instead, |(y_i - y_j) yscale|^2 - 14 for
// the same lane layout.
template <int NT, bool MASK, bool SAFE, bool DIRECT>
__device__ __forceinline__ void chunk_products(const Smem<NT, SAFE> &sm, const u32x4 (&xi)[2], int rel,
                                               f32x16 (&acc)[NT], int D, float yscale)
{
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    const int col = lane & 31;
#pragma unroll 1
    for (int jb = 0; jb < JC; jb += 2 * KS) {
        f32x16 dd = f32x16{};
        if constexpr (DIRECT) {
            const int row = (threadIdx.x >> 6) * 32 + col;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = jb + 8 * (r >> 2) + 4 * h + (r & 3);
                float d2 = 0.0f;
                for (int d = 0; d < D; ++d) {
                    const float t = (sm.yr[row][d] - sm.yc[j][d]) * yscale;
                    d2 = fmaf(t, t, d2);
                }
                dd[r] = d2 - PSI_LOG2;
            }
        } else {
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const f16x8 A = *reinterpret_cast<const f16x8 *>(&sm.xh[jb + col][16 * m + 8 * h]);
                dd = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, __builtin_bit_cast(f16x8, xi[m]), dd, 0, 0, 0);
            }
        }
        u32x4 ah[2], al[2];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int r = 2 * k;
            float a = __builtin_amdgcn_exp2f(-dd[r]);
            float b = __builtin_amdgcn_exp2f(-dd[r + 1]);
            if (MASK) {
                const int ja = jb + 8 * (r >> 2) + 4 * h + (r & 3);
                a = (ja > rel) ? a : 0.0f;
                b = (ja + 1 > rel) ? b : 0.0f;
            }
            const uint32_t hw = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(a, b));
            // residuals a - hi_a, b - hi_b, each one mixed-precision multiply-add
            // reading its float16 half of hw directly (exact: hi is a truncation of a)
            float ra, rb;
            asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(ra) : "v"(hw), "v"(a));
            asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(rb) : "v"(hw), "v"(b));
            ah[k >> 2][k & 3] = hw;
            al[k >> 2][k & 3] = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(ra, rb));
        }
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const f16x8 A_hi = __builtin_bit_cast(f16x8, ah[m]);
            const f16x8 A_lo = __builtin_bit_cast(f16x8, al[m]);
            const int jl = jb + KS * m + 8 * h;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const f16x8 B = *reinterpret_cast<const f16x8 *>(&sm.gs[32 * t + col][jl]);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A_hi, B, acc[t], 0, 0, 0);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A_lo, B, acc[t], 0, 0, 0);
            }
        }
    }
}

// Reduce the float32 tiles into the float64 partials and clear them.  Lane
// (col, h) holds column 32 t + col for rows 8 (r / 4) + 4 h + r % 4 of its
// wave's 32.  The leading R columns are the row weights; their values
// (Psi_upper w_q)_i go through LDS so that every column can take the
// transposed term sum_i G_ic (Psi_upper w_q)_i.
template <int NT, int RR, bool SAFE>
__device__ __forceinline__ void flush(const EParams &p, Smem<NT, SAFE> &sm, f32x16 (&acc)[NT],
                                      double (&part)[NT][1 + RR])
{
    constexpr int C = 32 * NT;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int h = lane >> 5;
    const int col = lane & 31;
    if (col < p.R) {
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
            if (RR > 1) s2[t] = fmaf(wq.y, v, fmaf(g, vq.y, s2[t]));
            if (RR > 2) s3[t] = fmaf(wq.z, v, fmaf(g, vq.z, s3[t]));
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        part[t][0] += 2.0 * (double)s0[t];       // diagonal-type sums are symmetric
        part[t][1] += (double)s1[t];
        if (RR > 1) part[t][RR > 1 ? 2 : 1] += (double)s2[t];
        if (RR > 2) part[t][RR > 2 ? 3 : 1] += (double)s3[t];
        acc[t] = f32x16{};
    }
}

// Work split.  Row blocks g and nb - 1 - g pair up (together about n pairs per
// row); their chunks, block g's first, form one list that K workgroups share in
// equal contiguous pieces, so the launch has enough equal-sized workgroups to
// keep every compute unit busy to the end.
// RR: row-weight columns the reduction carries (RR covers R <= RR).
template <int NT, int NS, int RR, bool SAFE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void tp_pairsum_kernel(const EParams p, const int K)
{
    constexpr int C = 32 * NT;
    // the range check's flag selects the one instantiation that works
    const bool flagged = __atomic_load_n(p.flag, __ATOMIC_RELAXED) != 0u;
    if (flagged != SAFE) return;
    __shared__ __align__(16) Smem<NT, SAFE> sm;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int h = lane >> 5;
    const int col = lane & 31;
    const int64_t nb = (p.n + ROWS - 1) / ROWS;
    for (int e = tid; e < C * (1 + MAXR); e += 256) (&sm.red[0][0])[e] = 0.0;
    double part[NT][1 + RR];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q <= RR; ++q) part[t][q] = 0.0;
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x16{};

    const int64_t g = blockIdx.x / K, k = blockIdx.x % K;
    const int64_t b1 = g, b2 = nb - 1 - g;
    // ROWS == JC: a row block starts a chunk, and its first chunk holds the diagonal
    const int64_t L1 = (p.n - b1 * ROWS + JC - 1) / JC;
    const int64_t L2 = b2 > b1 ? (p.n - b2 * ROWS + JC - 1) / JC : 0;
    const int64_t L = L1 + L2;
    const int64_t v0 = k * L / K, v1 = (k + 1) * L / K;
    centre(p, sm);
    u32x4 xi[2];
    int64_t cur = -1;
    int since = 0;
    // chunk v: row block b1 for v < L1 (chunk v of its row), else b2 (chunk v - L1)
    auto chunk_j0 = [&](int64_t v) { return v < L1 ? b1 * ROWS + v * JC : b2 * ROWS + (v - L1) * JC; };
    Pending<2 * NS> pd;
    if (v0 < v1) load_chunk<NT, 2 * NS>(p, chunk_j0(v0), pd);
    bool rows_far = false;
    for (int64_t v = v0; v < v1; ++v) {
        const int64_t blk = v < L1 ? b1 : b2;
        const int64_t c0 = v < L1 ? v : v - L1;      // chunk within the block's row
        const int64_t j0 = chunk_j0(v);
        if (blk != cur) {
            rows_far = setup_rows<NT, NS, SAFE>(p, sm, blk * ROWS, xi);
            cur = blk;
        }
        __syncthreads();
        const bool cfar = store_chunk<NT, 2 * NS, SAFE>(p, sm, j0, pd);
        bool far = false;
        if constexpr (SAFE) far = __syncthreads_or(cfar) != 0 || rows_far;
        else __syncthreads();
        if (v + 1 < v1) load_chunk<NT, 2 * NS>(p, chunk_j0(v + 1), pd);
        if (SAFE && far) {    // uniform over the workgroup
            if (c0 == 0) chunk_products<NT, true, SAFE, SAFE>(sm, xi, wave * 32 + col, acc, p.D, p.yscale);
            else chunk_products<NT, false, SAFE, SAFE>(sm, xi, 0, acc, p.D, p.yscale);
        } else {
            if (c0 == 0) chunk_products<NT, true, SAFE, false>(sm, xi, wave * 32 + col, acc, p.D, p.yscale);
            else chunk_products<NT, false, SAFE, false>(sm, xi, 0, acc, p.D, p.yscale);
        }
        const bool block_ends = v + 1 == v1 || v + 1 == L1;
        if (++since == FL || block_ends) {
            flush<NT, RR, SAFE>(p, sm, acc, part);
            since = 0;
        }
    }
    // combine the two row halves of each column, then the four waves, then workgroups
    const int R = p.R;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q <= RR; ++q) {
            double x = part[t][q];
            x += __shfl_xor(x, 32);
            if (h == 0 && q <= R) atomicAdd(&sm.red[32 * t + col][q], x);
        }
    __syncthreads();
    if (v1 > v0)
        for (int e = tid; e < C * (1 + R); e += 256) {
            const int c = e / (1 + R), q = e % (1 + R);
            if (c < p.C) atomicAdd(&p.sums[(int64_t)c * (1 + R) + q], sm.red[c][q] * PSI_UNSCALE);
        }
    if constexpr (SAFE) {
        // the last workgroup clears the flag and the count for the next launch
        __shared__ bool last;
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            last = atomicAdd(p.flag + 1, 1u) == gridDim.x - 1;
        }
        __syncthreads();
        if (last && tid == 0) {
            p.flag[0] = 0u;
            p.flag[1] = 0u;
            __threadfence();
        }
    }
}

// Range check: sets p.flag[0] when any event lies outside the matrix-core
// range of the centre (|v|^2 > VMAX2, or not finite), with the same centre
// and the same arithmetic as the pair-sum kernels.
__global__ __launch_bounds__(256) void tp_range_kernel(const EParams p)
{
    __shared__ CentreSmem sm;
    centre(p, sm);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= p.n) return;
    float nrm = 0.0f;
    for (int d = 0; d < p.D; ++d) {
        const float v = p.Y[d * p.ldY + i] * p.yscale - sm.cen[d];
        nrm = fmaf(v, v, nrm);
    }
    if (!(nrm <= VMAX2)) atomicOr(p.flag, 1u);
}

template <int NT, int NS, int RR>
void launch_ntd(const EParams &p, hipStream_t st)
{
    const int64_t nb = (p.n + ROWS - 1) / ROWS;
    const int64_t pairs = (nb + 1) / 2;
    // pieces per block pair: about 64 workgroups per compute unit in all (the
    // last partial wave of workgroups then costs a few percent), no piece
    // shorter than two chunks
    const int64_t chunks = (p.n + JC - 1) / JC;
    int64_t K = (16384 + pairs - 1) / pairs;
    K = K > chunks / 2 ? chunks / 2 : K;
    K = K < 1 ? 1 : K;
    // one of the two instantiations works (the range check's flag), the other exits
    hipLaunchKernelGGL((tp_pairsum_kernel<NT, NS, RR, false>), dim3((unsigned)(pairs * K)), dim3(256), 0, st, p, (int)K);
    hipLaunchKernelGGL((tp_pairsum_kernel<NT, NS, RR, true>), dim3((unsigned)(pairs * K)), dim3(256), 0, st, p, (int)K);
}

template <int NT, int RR>
void launch_ntr(const EParams &p, hipStream_t st)
{
    switch (p.D) {   // distance-vector components D + 2, in pairs
    case 1: case 2: launch_ntd<NT, 2, RR>(p, st); break;
    case 3: case 4: launch_ntd<NT, 3, RR>(p, st); break;
    case 5: case 6: launch_ntd<NT, 4, RR>(p, st); break;
    default: launch_ntd<NT, 5, RR>(p, st); break;
    }
}

template <int NT>
void launch_nt(const EParams &p, hipStream_t st)
{
    if (p.R <= 1) launch_ntr<NT, 1>(p, st);
    else if (p.R == 2) launch_ntr<NT, 2>(p, st);
    else launch_ntr<NT, 3>(p, st);
}

// Certified order of two pair masses m^2(a, b) against m^2(c, d): +1 if
// larger, -1 if smaller, 0 if equal.  float64 with the magnitude bound
// |m^2_computed - m^2| <= 8u (sum_q |x_aq| + |x_bq|)^2 (one rounding for each
// component sum, four for the squares and their sum), exact integers when the
// two intervals overlap.
template <typename Tin>
__device__ int pair_cmp(const double (&x)[4][4], int a, int b, int c, int d)
{
    double m2[2], mag[2];
    const int sl[2][2] = { { a, b }, { c, d } };
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        double S[4], A = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            S[q] = x[sl[k][0]][q] + x[sl[k][1]][q];
            A += __builtin_fabs(x[sl[k][0]][q]) + __builtin_fabs(x[sl[k][1]][q]);
        }
        m2[k] = fma(-S[3], S[3], fma(-S[2], S[2], fma(-S[1], S[1], S[0] * S[0])));
        mag[k] = fma(8.0 * 0x1p-53 * A, A, 0x1p-1000);
    }
    const double diff = m2[0] - m2[1];
    const double err = (mag[0] + mag[1]) * (1.0 + 0x1p-50);
    if (diff > err) return 1;
    if (diff < -err) return -1;
    int64_t mant[4][4];
    int ex[4][4];
    for (int s = 0; s < 4; ++s)
        for (int q = 0; q < 4; ++q) {
            if constexpr (sizeof(Tin) == 4) tpx::decode_f32((float)x[s][q], mant[s][q], ex[s][q]);
            else tpx::decode_f64(x[s][q], mant[s][q], ex[s][q]);
        }
    const int r = tpx::pair_mass2_cmp(mant, ex, sizeof(Tin) == 4 ? 136 : 107, a, b, c, d);
    return r == 2 ? 0 : r;
}

// Invariant mass of the slots in a mask, per event (Sect. 4.2 coordinates).
// With relabel 1 (D0 -> pi+ pi- pi+ pi-, slots in charge order + - + -) the
// event is first relabelled as Sect. 4.2 prescribes: of the four pi+ pi- pairs
// the one of largest invariant mass becomes pi3 pi4 (slots 2, 3), which fixes
// the order of all four pions.  Ties go to the first pair in the order
// (2,3), (0,1), (0,3), (2,1) (the stored labelling, then the swap of both
// pairs, of the pi+, of the pi-).
template <typename Tin>
__global__ void tp_coords_kernel(CParams c)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= c.n) return;
    const Tin *const *P = reinterpret_cast<const Tin *const *>(c.p);
    double x[4][4];
    for (int s = 0; s < 4; ++s)
        for (int q = 0; q < 4; ++q) x[s][q] = (double)P[s * 4 + q][e];
    int perm[4] = { 0, 1, 2, 3 };   // new slot t holds stored slot perm[t]
    if (c.relabel == 1) {
        const int pa[4][2] = { { 2, 3 }, { 0, 1 }, { 0, 3 }, { 2, 1 } };
        const int pm[4][4] = { { 0, 1, 2, 3 }, { 2, 3, 0, 1 }, { 2, 1, 0, 3 }, { 0, 3, 2, 1 } };
        int best = 0;
        for (int k = 1; k < 4; ++k)
            if (pair_cmp<Tin>(x, pa[k][0], pa[k][1], pa[best][0], pa[best][1]) > 0) best = k;
        for (int t = 0; t < 4; ++t) perm[t] = pm[best][t];
    }
    for (int k = 0; k < c.ncoord; ++k) {
        double S[4] = { 0.0, 0.0, 0.0, 0.0 };
        for (int s = 0; s < 4; ++s)
            if (c.masks[k] & (1 << s))
                for (int q = 0; q < 4; ++q) S[q] += x[perm[s]][q];
        const double m2 = S[0] * S[0] - S[1] * S[1] - S[2] * S[2] - S[3] * S[3];
        c.out[(int64_t)k * c.ldo + e] = (float)(m2 > 0.0 ? sqrt(m2) * c.scale : 0.0);
    }
}

}  // namespace

hipError_t launch_pairsums(const EParams &p, hipStream_t st)
{
    hipLaunchKernelGGL(tp_range_kernel, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, st, p);
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
