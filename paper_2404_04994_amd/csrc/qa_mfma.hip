// qa_mfma.hip -- matrix-core scorer for the floor/ceil box (Sec. 3.2.1), its
// thresholded sub-boxes (Sec. 3.2.2) and, for closed arrays, the subsets of
// the free dots with the required number raised, at T = 0 (Eq. argmin),
// 9 <= N <= 16 dots.
//
// Every candidate of pixel p is n0 + b, b in {0,1}^N, and (Eq. free_energy)
//     U(n0 + b) - U(n0) = b^T g + 1/2 b^T A b,       g = A (n0 - x_u).
// The box is split into a low part (dots 0..7, index c_lo, 256 values) and a
// high part (dots 8..N-1, index c_hi).  With A_LH the low/high block of A,
//     E(c_hi, c_lo) = b_lo^T g'(c_hi) + h_lo(c_lo) + C(c_hi),
//     g'(c_hi)     = g_lo + A_LH b_hi,
//     C(c_hi)      = b_hi^T g_hi + 1/2 b_hi^T A_HH b_hi,
// so the pixels x candidates contraction becomes one matrix-core tile per
// 16 high x 16 low indices: rows carry g' and C (they depend on the pixel),
// columns carry the 0/1 patterns of b_lo and h_lo (the same for every pixel,
// kept in registers for the whole kernel).  Each 16x16 tile is a single
// v_mfma_f32_16x16x32_bf16 whose K = 32 slots hold
//     chunk 0..2 : three BF16 parts of g' (exact truncation split of the FP32
//                  value; BF16X2 keeps two round-to-nearest parts) x b_lo bits
//     chunk 3    : three parts of C x 1 and 1 x three parts of h_lo,
// so the tile is the complete energy, accumulated in FP32.  The FP32 form
// uses three v_mfma_f32_16x16x4_f32 per tile instead (K = 4 each: g'[0..3],
// g'[4..7], and {C, 1} against {1, h_lo}).
//
// Epilogue: a running minimum (v_min3) per lane and high-index row tile;
// the lane/row-tile minima give the best value and a certified runner-up
// bound; the winning row tile is recomputed to recover the index and the
// runner-up inside it.  When the runner-up lies within twice the certified
// error bound of the best, the exact argmin is one of the states whose
// approximate energy lies within that band of the best: the wave sweeps the
// row tiles that hold such states once more and every lane scores its own
// in-band states in FP64 (ties to the lexicographically smallest state).
// Otherwise n* = n0 + b is written directly.
#include "qa_internal.h"

namespace qa {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

union Pack8 {
    uint32_t u[4];
    bf16x8_t v;
};

__device__ __forceinline__ uint32_t fbits(float x) { return __float_as_uint(x); }
__device__ __forceinline__ float trunc16(float x)
{
    return __uint_as_float(__float_as_uint(x) & 0xFFFF0000u);
}
// round to nearest even at 16 significant bits (finite inputs)
__device__ __forceinline__ float rne16(float x)
{
    const uint32_t b = __float_as_uint(x);
    return __uint_as_float((b + 0x7FFFu + ((b >> 16) & 1u)) & 0xFFFF0000u);
}
// two FP32 values whose low 16 bits are zero -> packed BF16 pair
__device__ __forceinline__ uint32_t pack2(float lo, float hi)
{
    return (fbits(lo) >> 16) | (fbits(hi) & 0xFFFF0000u);
}

// sum over each 16-lane row (every lane of the row gets it; the exchanges
// pair lanes symmetrically, so the lanes' sums are identical)
__device__ __forceinline__ float row_sumf(float x)
{
    x += dppf<kDppXor1>(x);
    x += dppf<kDppXor2>(x);
    x += dppf<kDppHalfMirror>(x);
    return x + dppf<kDppMirror>(x);
}

// bitwise OR over the 64 lanes (every lane gets it)
__device__ __forceinline__ uint32_t wave_or32(uint32_t x)
{
    x |= dpp32<kDppXor1>(x);
    x |= dpp32<kDppXor2>(x);
    x |= dpp32<kDppHalfMirror>(x);
    x |= dpp32<kDppMirror>(x);
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    x = r[0] | r[1];
    const auto t = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return __builtin_amdgcn_readfirstlane(t[0] | t[1]);
}
__device__ __forceinline__ uint64_t wave_or64(uint64_t x)
{
    return (uint64_t)wave_or32((uint32_t)x) | ((uint64_t)wave_or32((uint32_t)(x >> 32)) << 32);
}

// compile-time loop: f(integral_constant<int, I>) for I in [I0, I1)
template <int I0, int I1, typename Fn>
__device__ __forceinline__ void sfor(Fn &&f)
{
    if constexpr (I0 < I1) {
        f(std::integral_constant<int, I0>{});
        sfor<I0 + 1, I1>(f);
    }
}

// LDS writes of a wave made visible to all of its lanes (requests of one
// wave are served in order; the fences keep the compiler from moving them)
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


constexpr int kPrecFP32 = 1, kPrecX3 = 2, kPrecX2 = 3;

#ifndef QA_SCORER_WAVES
#define QA_SCORER_WAVES 3
#endif
// waves per SIMD of the bound-ordered scorer (measured): five for the FP32
// dense box, four otherwise (the split-BF16 forms read their column
// operands from LDS once per product, and a fifth wave per SIMD costs more
// in LDS bandwidth than it hides)
#ifndef QA_BOUND_WAVES
#define QA_BOUND_WAVES(PREC, MODE) ((MODE) == kDense && (PREC) == kPrecFP32 ? 5 : 4)
#endif
#ifndef QA_BOUND_B_LDS
#define QA_BOUND_B_LDS 1
#endif
#ifndef QA_BOUND_B_REGS
#define QA_BOUND_B_REGS 0
#endif

// MODE kDense: the floor/ceil box.  kPruned: the thresholded candidate set
// (Sec. 3.2.2), n0 + b with b a subset of the pixel's free dots.  kClosed:
// closed arrays (Sec. 2, constraint iii), b a subset of the free dots with
// exactly k raised (k and the free dots from the setup, after any threshold
// doubling); a state's popcount is popc(row bits) + popc(column bits) of its
// tile, so each lane knows which of its four elements qualify for a tile's
// uniform remainder k - popc(rt) - popc(ct) and sets the others to +inf
// before every minimum, and tiles with no qualifying element are skipped.
// kPruned and kClosed:  A fixed dot i gets the penalty 2^100 added to
// g_i, so every state that raises it scores above 2^99 and never wins, and
// the tables are unchanged; row tiles that raise a fixed dot of 12..15 and
// column tiles that raise a fixed dot of 4..7 are skipped.  A 0/1 operand
// times the penalty is an exact 0 or the penalty, so the valid states score
// exactly as in the dense form and the same error bound holds for them.
constexpr int kDense = 0, kPruned = 1, kClosed = 2;

template <int PREC, int MODE>
__global__ __launch_bounds__(256, QA_SCORER_WAVES) void k_score_mfma(const DiagRec *__restrict__ dr,
                                                    const PixRec *__restrict__ pr, int64_t P,
                                                    int32_t *__restrict__ n_out,
                                                    int64_t *__restrict__ counters)
{
    constexpr bool PRUNED = MODE != kDense;
    constexpr bool CLOSED = MODE == kClosed;
    __shared__ float sT1[16][8];
    __shared__ float sT2[16][8];
    __shared__ float sH[256];
    __shared__ double sT1d[16][8], sT2d[16][8];  // FP64 tables of the near-tie re-score
    __shared__ double sHd[256], sLd[256];
    __shared__ double sG64[4][kMaxDot];
    __shared__ uint2 sCt[4][256];  // per wave: BF16 parts of C(c_hi) of its pixel
    __shared__ float sGm[4][16][64];  // per wave: lane minima of each row tile
    __shared__ unsigned long long sflag, sgap, scand;
    for (int e = threadIdx.x; e < 128; e += blockDim.x) {
        sT1[e / 8][e % 8] = dr->T1[e / 8][e % 8];
        sT2[e / 8][e % 8] = dr->T2[e / 8][e % 8];
    }
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        sH[e] = dr->Hhi[e];
        sHd[e] = dr->Hhid[e];
        sLd[e] = dr->hlod[e];
        if (e < 128) {
            sT1d[e / 8][e % 8] = dr->T1d[e / 8][e % 8];
            sT2d[e / 8][e % 8] = dr->T2d[e / 8][e % 8];
        }
    }
    if (threadIdx.x == 0) { sflag = 0; sgap = 0; scand = 0; }
    __syncthreads();

    const int n = dr->n;
    const int nh = n - 8;
    const int nrt = nh > 4 ? 1 << (nh - 4) : 1;
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4;     // K chunk of this lane's A/B operand slots
    const int mrow = lane & 15;  // A row (high index within tile) = B column (low index)
    const float sumabs = dr->sumabs;

    // ---- pixel-independent column operands, one set per 16-wide low tile ----
    uint32_t bw[16][4];
    float bf[16][3];
#pragma unroll
    for (int ct = 0; ct < 16; ++ct) {
        const int clo = ct * 16 + mrow;
        const float h = dr->hlo[clo];
        if (PREC == kPrecFP32) {
            bf[ct][0] = (float)((clo >> q) & 1);
            bf[ct][1] = (float)((clo >> (4 + q)) & 1);
            bf[ct][2] = (q == 0) ? 1.0f : (q == 1 ? h : 0.0f);
        } else {
            if (q < 3) {
#pragma unroll
                for (int d = 0; d < 4; ++d)
                    bw[ct][d] = ((clo >> (2 * d) & 1) ? 0x3F80u : 0u) |
                                ((clo >> (2 * d + 1) & 1) ? 0x3F800000u : 0u);
            } else {
                const float h1 = trunc16(h);
                const float r = h - h1;
                const float h2 = trunc16(r);
                const float h3 = r - h2;  // exact in BF16
                bw[ct][0] = 0x3F803F80u;
                bw[ct][1] = 0x3F80u | (fbits(h1) & 0xFFFF0000u);
                bw[ct][2] = pack2(h2, h3);
                bw[ct][3] = 0u;
            }
        }
    }

    // Persistent waves: wave w scores pixels w, w + nwaves, ... (a static
    // interleave: a shared work-queue cursor costs more in same-address
    // atomics than it recovers in balance).  Lane i < 16 holds g0_i and n0_i
    // of its pixel (vector loads, one pixel ahead).
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    int64_t nflag = 0, ngap = 0, ncand = 0;
    const int li = lane & 15;
    float *gmrec = &sGm[threadIdx.x >> 6][0][0];
    double gnext = 0.0;
    int nnext = 0, knext = 0;
    uint32_t fnext = 0;
    if (wave < P) {
        gnext = pr[wave].g0[li];
        nnext = pr[wave].n0[li];
        if (PRUNED) fnext = pr[wave].free;
        if (CLOSED) knext = pr[wave].k;
    }
    // closed: popcount of this lane's element i within a tile (row bits
    // 4q + i, column bits mrow)
    int cq[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) cq[i] = __popc((uint32_t)(4 * q + i)) + __popc((uint32_t)mrow);
    for (int64_t pw = wave; pw < P; pw += nwaves) {
        const int64_t p = pw;
        const double gcur = gnext;
        const int ncur = nnext;
        // free dots of the pixel (a wave-uniform value)
        const uint32_t F = PRUNED ? __builtin_amdgcn_readfirstlane(fnext) : 0xFFFFu;
        const int kc = CLOSED ? __builtin_amdgcn_readfirstlane(knext) : 0;
        if (pw + nwaves < P) {
            gnext = pr[pw + nwaves].g0[li];
            nnext = pr[pw + nwaves].n0[li];
            if (PRUNED) fnext = pr[pw + nwaves].free;
            if (CLOSED) knext = pr[pw + nwaves].k;
        }
        // g0 beyond n is zero in the record; every lane gets all sixteen
        // (the error bound takes the unpenalised values)
        const float gl = (float)gcur;
        const float glp = (PRUNED && !(F >> li & 1u)) ? 0x1p100f : gl;
        float g[16];
        float gabs = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            g[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(glp), i));
            gabs += fabsf(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(gl), i)));
        }
        if (MODE == kPruned) ncand += 1ll << __popc(F & ((1u << n) - 1u));
        if (CLOSED) {
            // C(free dots, k)
            const int nf = __popc(F & ((1u << n) - 1u));
            int64_t b = 1;
            for (int j = 0; j < kc && j < nf; ++j) b = b * (nf - j) / (j + 1);
            ncand += (kc >= 0 && kc <= nf) ? b : 0;
        }
        // row tiles (high dots 12..15) and column tiles (low dots 4..7) that
        // raise no fixed dot (closed: and that can hold k raised dots)
        auto rt_ok = [&](int rt) {
            if (!PRUNED) return true;
            if (((uint32_t)rt << 12) & ~F) return false;
            return !CLOSED || (kc - __popc((uint32_t)rt) >= 0 && kc - __popc((uint32_t)rt) <= 12);
        };
        auto ct_ok = [&](int ct) { return !PRUNED || !(((uint32_t)ct << 4) & ~F); };
        // closed: tile (rt, ct) holds a qualifying element, and the masking
        auto tile_ok = [&](int rt, int ct) {
            if (!CLOSED) return true;
            const int r = kc - __popc((uint32_t)rt) - __popc((uint32_t)ct);
            return r >= 0 && r <= 8;
        };
        auto qualify = [&](f32x4_t d, int rt, int ct) -> f32x4_t {
            if (CLOSED) {
                const int r = kc - __popc((uint32_t)rt) - __popc((uint32_t)ct);
#pragma unroll
                for (int i = 0; i < 4; ++i) d[i] = (cq[i] == r) ? d[i] : INFINITY;
            }
            return d;
        };
        // per-lane row constants: G1 = g_lo + A_LH b_hi(row bits), P1 = b_hi(row)^T g_hi
        float G1[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) G1[i] = g[i] + sT1[mrow][i];
        float P1 = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (mrow >> j & 1) P1 += g[8 + j];
        // split-BF16 forms: the lane builds low dots 2q and 2q + 1 of its row
        float G1a = G1[0], G1b = G1[1];
#pragma unroll
        for (int d = 1; d < 4; ++d)
            if (q == d) { G1a = G1[2 * d]; G1b = G1[2 * d + 1]; }
        // and the wave tabulates the constant chunk of every high index once:
        // C(c_hi) = b_hi^T g_hi + 1/2 b_hi^T A_HH b_hi as three BF16 parts,
        // dword 0 = (C_1, C_2), dword 1 = (C_3, 1)
        uint2 *ctab = sCt[threadIdx.x >> 6];
        if (PREC != kPrecFP32) {
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) {
                const int rt = q + 4 * e4;
                float P2 = 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (rt >> j & 1) P2 += g[12 + j];
                const float C = (P1 + P2) + sH[rt * 16 + mrow];
                const float c1 = trunc16(C);
                const float cr = C - c1;
                const float c2 = trunc16(cr);
                ctab[rt * 16 + mrow] = make_uint2(pack2(c1, c2), pack2(cr - c2, 1.0f));
            }
            __builtin_amdgcn_wave_barrier();
        }

        // Build the A operand of row tile rt for this lane.  Split-BF16 forms:
        // the four lanes of a row share the work.  Lane (q, row) splits
        // g'_{2q} and g'_{2q+1} into their BF16 parts (dword p = part p of the
        // pair) and forms dword q of the constant chunk (C parts and ones);
        // a 4 x 4 transpose of those dwords across the four 16-lane rows
        // (two v_permlane32_swap, two v_permlane16_swap) leaves lane (q, row)
        // with part q of g'_0..g'_7 (q < 3) or the constant chunk (q = 3).
        auto build_a = [&](int rt, Pack8 &a, float (&af)[3]) {
            if (PREC == kPrecFP32) {
                float P2 = 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (rt >> j & 1) P2 += g[12 + j];
                const float C = (P1 + P2) + sH[rt * 16 + mrow];
                float v0 = 0.0f, v1 = 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (q == j) {
                        v0 = G1[j] + sT2[rt][j];
                        v1 = G1[4 + j] + sT2[rt][4 + j];
                    }
                }
                af[0] = v0;
                af[1] = v1;
                af[2] = (q == 0) ? C : (q == 1 ? 1.0f : 0.0f);
            } else {
                const float v0 = G1a + sT2[rt][2 * q];
                const float v1 = G1b + sT2[rt][2 * q + 1];
                uint32_t R0, R1, R2;
                if (PREC == kPrecX3) {
                    // exact three-way truncation split: v = p0 + p1 + p2
                    const float a0 = trunc16(v0), b0 = trunc16(v1);
                    const float r0 = v0 - a0, s0 = v1 - b0;
                    const float a1 = trunc16(r0), b1 = trunc16(s0);
                    R0 = pack2(a0, b0);
                    R1 = pack2(a1, b1);
                    R2 = pack2(r0 - a1, s0 - b1);
                } else {
                    // two round-to-nearest parts; chunk 2 unused
                    const float a0 = rne16(v0), b0 = rne16(v1);
                    R0 = pack2(a0, b0);
                    R1 = pack2(rne16(v0 - a0), rne16(v1 - b0));
                    R2 = 0u;
                }
                const uint2 cw = ctab[rt * 16 + mrow];
                uint32_t R3 = (q == 2) ? 0x3F803F80u : 0u;
                R3 = (q == 1) ? cw.y : R3;
                R3 = (q == 0) ? cw.x : R3;
                const auto t02 = __builtin_amdgcn_permlane32_swap(R0, R2, false, false);
                const auto t13 = __builtin_amdgcn_permlane32_swap(R1, R3, false, false);
                const auto u01 = __builtin_amdgcn_permlane16_swap(t02[0], t13[0], false, false);
                const auto u23 = __builtin_amdgcn_permlane16_swap(t02[1], t13[1], false, false);
                a.u[0] = u01[0];
                a.u[1] = u01[1];
                a.u[2] = u23[0];
                a.u[3] = u23[1];
            }
        };
        auto tile = [&](const Pack8 &a, const float (&af)[3], int ct) -> f32x4_t {
            f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
            if (PREC == kPrecFP32) {
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0], bf[ct][0], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1], bf[ct][1], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[2], bf[ct][2], acc, 0, 0, 0);
            } else {
                Pack8 b;
                b.u[0] = bw[ct][0]; b.u[1] = bw[ct][1]; b.u[2] = bw[ct][2]; b.u[3] = bw[ct][3];
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc, 0, 0, 0);
            }
            return acc;
        };

        // ---- main sweep: minimum per (lane, row tile) ----
        float best1 = INFINITY, best2 = INFINITY;
        int rt1 = 0;
        for (int rt = 0; rt < nrt; ++rt) {
            if (!rt_ok(rt)) continue;
            Pack8 a;
            float af[3];
            build_a(rt, a, af);
            // software-pipelined: the minima of tile ct - 1 are taken while
            // tile ct is on the matrix core (two independent minimum chains)
            float gm = INFINITY, gm2 = INFINITY;
            if (PRUNED) {
#pragma unroll
                for (int ct = 0; ct < 16; ++ct) {
                    if (!ct_ok(ct) || !tile_ok(rt, ct)) continue;
                    const f32x4_t d = qualify(tile(a, af, ct), rt, ct);
                    gm = fminf(fminf(gm, d[0]), d[1]);
                    gm2 = fminf(fminf(gm2, d[2]), d[3]);
                }
            } else {
                f32x4_t dp = tile(a, af, 0);
#pragma unroll
                for (int ct = 1; ct < 16; ++ct) {
                    const f32x4_t d = tile(a, af, ct);
                    float &m = (ct & 1) ? gm : gm2;
                    m = fminf(fminf(m, dp[0]), dp[1]);
                    m = fminf(fminf(m, dp[2]), dp[3]);
                    dp = d;
                }
                gm2 = fminf(fminf(gm2, dp[0]), dp[1]);
                gm2 = fminf(fminf(gm2, dp[2]), dp[3]);
            }
            gm = fminf(gm, gm2);
            gmrec[rt * 64 + lane] = gm;
            if (gm < best1) { best2 = best1; best1 = gm; rt1 = rt; }
            else best2 = fminf(best2, gm);
        }
        // ---- best group over the wave and the runner-up among group minima ----
        float wmin = best1;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) wmin = fminf(wmin, __shfl_xor(wmin, off));
        const unsigned long long hit = __ballot(best1 == wmin);
        const int winner = __ffsll((long long)hit) - 1;
        float other = (lane == winner) ? best2 : best1;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) other = fminf(other, __shfl_xor(other, off));
        const int rtw = __shfl(rt1, winner);
        // ---- recompute the winning row tile: per lane the two smallest tile
        // minima and the tile of the smallest; then the winner's tile once
        // more for the index and the runner-up inside it ----
        float e1, e2;
        int iw;
        {
            Pack8 a;
            float af[3];
            build_a(rtw, a, af);
            float t1 = INFINITY, t2 = INFINITY;
            int ct1 = 0;
#pragma unroll
            for (int ct = 0; ct < 16; ++ct) {
                if (!ct_ok(ct) || !tile_ok(rtw, ct)) continue;
                const f32x4_t d = qualify(tile(a, af, ct), rtw, ct);
                const float tm = fminf(fminf(d[0], d[1]), fminf(d[2], d[3]));
                const bool lt = tm < t1;
                t2 = lt ? t1 : fminf(t2, tm);
                t1 = lt ? tm : t1;
                ct1 = lt ? ct : ct1;
            }
            // the winner lane's tile: a scalar (readfirstlane) choice among
            // static indices, so the branch is taken by the whole wave (a
            // matrix-core instruction ignores the lane mask)
            const int ctw = __builtin_amdgcn_readfirstlane(__shfl(ct1, winner));
            const float t2w = __shfl(t2, winner);
            f32x4_t d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ct = 0; ct < 16; ++ct)
                if (ct == ctw) d = qualify(tile(a, af, ct), rtw, ct);
            float v1 = d[0], v2 = INFINITY;
            int i1 = 0;
#pragma unroll
            for (int i = 1; i < 4; ++i) {
                if (d[i] < v1) { v2 = v1; v1 = d[i]; i1 = i; }
                else v2 = fminf(v2, d[i]);
            }
            e1 = __shfl(v1, winner);
            iw = ctw * 4 + __shfl(i1, winner);
            e2 = fminf(other, fminf(t2w, __shfl(v2, winner)));
        }
        // Certified bound on |E_approx - E| for every candidate of the pixel.
        // All inputs of the tile sum are bounded by S = sum|g| + 1/2 sum|A|
        // (g' parts, C parts and h parts together), FP32 rounding of the
        // operands adds a few 2^-24 S and the 32-term FP32 accumulation at most
        // 31 * 2^-24 S (2^-23 per term if the hardware truncates); 2^-17 S
        // covers that with room to spare.  Two-part BF16 adds the 2^-16 |g'|
        // truncation of the split.
        const float S = gabs + sumabs;
        const float delta = (PREC == kPrecX2 ? 0x1p-15f : 0x1p-17f) * S;
        const bool tie = !(e2 - e1 > 2.0f * delta);
        if (!tie) {
            if (lane < n) {
                const int ct = iw >> 2, i = iw & 3;
                const int row = 4 * (winner >> 4) + i;
                const uint32_t chi = (uint32_t)(rtw * 16 + row);
                const uint32_t clo = (uint32_t)(ct * 16 + (winner & 15));
                const uint32_t b = clo | (chi << 8);
                n_out[p * n + lane] = ncur + (int32_t)((b >> lane) & 1u);
            }
            continue;
        }
        // ---- near tie: every candidate within 2 delta of the best holds the
        // exact argmin.  The wave sweeps the row tiles again (those whose lane
        // minima all lie above the band are skipped) and each lane scores its
        // own in-band states in FP64 from the split tables:
        //   U(n0 + b) - U(n0) = b_lo^T (g_lo + A_LH b_hi) + h_lo(c_lo)
        //                     + b_hi^T g_hi + 1/2 b_hi^T A_HH b_hi
        // then the wave takes the smallest (ties to the lexicographically
        // smallest state) ----
        ++nflag;
        const float thr = e1 + 2.0f * delta;
        double *g64 = sG64[threadIdx.x >> 6];
        if (lane < kMaxDot) g64[lane] = gcur;
        __builtin_amdgcn_wave_barrier();
        double b1 = INFINITY, b2 = INFINITY;
        uint32_t c1 = 0;
        for (int rt = 0; rt < nrt; ++rt) {
            if (!rt_ok(rt) || !__ballot(gmrec[rt * 64 + lane] <= thr)) continue;
            Pack8 a;
            float af[3];
            build_a(rt, a, af);
            uint64_t inband = 0;  // bit 4 ct + i: element i of tile ct
#pragma unroll
            for (int ct = 0; ct < 16; ++ct) {
                if (!ct_ok(ct) || !tile_ok(rt, ct)) continue;
                const f32x4_t d = qualify(tile(a, af, ct), rt, ct);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (d[i] <= thr) inband |= 1ull << (4 * ct + i);
            }
            while (inband) {
                const int bit = __ffsll((long long)inband) - 1;
                inband &= inband - 1;
                const uint32_t clo = (uint32_t)((bit >> 2) * 16 + mrow);
                const uint32_t chi = (uint32_t)(rt * 16 + 4 * q + (bit & 3));
                const uint32_t c = clo | (chi << 8);
                const int row = chi & 15, rth = chi >> 4;
                double e = sLd[clo] + sHd[chi];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    if (chi >> i & 1u) e += g64[8 + i];
                    if (clo >> i & 1u) e += (g64[i] + sT1d[row][i]) + sT2d[rth][i];
                }
                if (e < b1 || (e == b1 && __brev(c) < __brev(c1))) { b2 = b1; b1 = e; c1 = c; }
                else b2 = fmin(b2, e);
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            const double ob1 = __shfl_xor(b1, off);
            const double ob2 = __shfl_xor(b2, off);
            const uint32_t oc1 = __shfl_xor(c1, off);
            if (ob1 < b1 || (ob1 == b1 && __brev(oc1) < __brev(c1))) {
                b2 = fmin(b1, ob2); b1 = ob1; c1 = oc1;
            } else {
                b2 = fmin(b2, ob1);
            }
        }
        if (lane < n) n_out[p * n + lane] = ncur + (int32_t)((c1 >> lane) & 1u);
        if (lane == 0 && b2 - b1 < 1e-9) ++ngap;
    }
    if (lane == 0) {
        if (nflag) atomicAdd(&sflag, (unsigned long long)nflag);
        if (ngap) atomicAdd(&sgap, (unsigned long long)ngap);
        if (ncand) atomicAdd(&scand, (unsigned long long)ncand);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        block_add_counter(counters, C_NEAR_TIE, (int64_t)sflag);
        block_add_counter(counters, C_GAP_1E9, (int64_t)sgap);
        // dense: every pixel scores all 2^n candidates of its box
        if (PRUNED) block_add_counter(counters, C_CANDIDATES, (int64_t)scand);  // summed per pixel
        else if (blockIdx.x == 0) block_add_counter(counters, C_CANDIDATES, P << n);
    }
}

// ---------------------------------------------------------------------------
// Bound-ordered search of the candidate sets of N >= 13 dots (more than one
// row tile): the dense box, the thresholded sub-boxes (MODE kPruned) and the
// closed subsets (kClosed).
//
// The argmin over the 2^N states of the box is found without scoring all of
// them.  With y = n0 - x_u (so g = A y and U(n0 + b) - U(n0) = b^T g +
// 1/2 b^T A b = 1/2 (y + b)^T A (y + b) - 1/2 y^T A y), fixing the high part
// b_hi and minimising over a real-valued low part b_lo gives the Schur
// complement of A_LL in A, which is (C_dd,HH)^{-1} =: S:
//     E(b_hi, b_lo) >= L(b_hi) = K + b_hi^T s + 1/2 b_hi^T S b_hi,
//     s = S y_hi,  K = 1/2 y_hi^T s - U(n0)
// (the setup forms S in its Gauss-Jordan sweep, the table of
// 1/2 b_hi^T S b_hi, and s and K of every pixel in FP64).
// Closed arrays fix the low part's sum at m = k - popc(b_hi), which adds
// (m - mu - w^T b_hi)^2 / (2 gamma) to the bound.
// L is a lower bound for all 256 states of a high index, so a high index
// whose bound lies above an upper bound of the best approximate energy (plus
// a margin that covers the FP32 error of the bound and three times the
// certified error band) holds neither the exact argmin nor any state of the
// near-tie band.  The upper bound is the energy of the setup's guess (a state
// of the candidate set, its energy computed by the setup in FP64) or, when
// that leaves more than two tiles of rows, the best of the row tile with the
// smallest bound, scored first.  The rows are scored sixteen to a tile (a row
// of the tile is any high index); the next tile's table reads are issued
// while a tile is on the matrix cores.  Each lane keeps the three smallest
// minima over groups of four column tiles (16 elements) and where the first
// two lie; the winner's group is recomputed for the position and the
// runner-up.  Near ties re-score in FP64 the in-band states of the groups
// that can hold them (the lanes' two best groups when no lane has a third
// group in the band, else every scored tile).  The error band and the FP64
// re-score are those of the exhaustive scorer over the scored rows, so the
// result is the argmin over the whole candidate set, as in the exhaustive
// form.  Per pixel the kernel is a chain of dependent steps (LDS reads,
// cross-lane reductions, matrix products), so several waves share a SIMD;
// the column operands sit in an LDS table (one read per product) so that
// the registers allow four or five waves.
// ---------------------------------------------------------------------------
template <int PREC, int MODE>
__global__ __launch_bounds__(256, QA_BOUND_WAVES(PREC, MODE)) void k_score_bound(const DiagRec *__restrict__ dr,
                                                     const PixRec *__restrict__ pr, int64_t P,
                                                     int32_t *__restrict__ n_out,
                                                     int64_t *__restrict__ counters)
{
    constexpr bool PRUNED = MODE != kDense;
    constexpr bool CLOSED = MODE == kClosed;
    __shared__ float sT1[16][8];
    __shared__ float sT2[16][8];
    __shared__ float sH[256];
    __shared__ float sHlo[256];                  // 1/2 b_lo^T A_LL b_lo
    __shared__ float sHs[256];                   // 1/2 b_hi^T S b_hi (1e30 beyond 2^(N-8))
    __shared__ double sT1d[16][8], sT2d[16][8];  // FP64 tables of the near-tie re-score
    __shared__ double sHd[256], sLd[256];
    __shared__ double sG64[4][kMaxDot];
    __shared__ float sPt[4][32];                 // per wave: b_hi^T g_hi over bits 0..3 / 4..7
    __shared__ float sWin[4][16];                // per wave: the winning lane's group
    __shared__ uint8_t sList[4][256];            // per wave: high index of every scored row
    __shared__ uint32_t sBand[4][128];           // per wave: near-tie states to re-score
    __shared__ uint4 sB[16][64];                 // column operands: [column tile][lane]
    __shared__ unsigned long long sflag, sgap, srows, scand;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int q = lane >> 4;
    const int mrow = lane & 15;
    const int li = lane & 15;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    // the diagram's scalars first (their loads lead the staging)
    const int n = dr->n;
    const int nh = n - 8;
    const int nrt = 1 << (nh - 4);
    const float sumabs = dr->sumabs;
    const float hsabs = dr->sabsS;
    // closed arrays: w and 1 / (2 gamma) of the low-sum term of the bound
    float wb[8];
    float wabs = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        wb[j] = CLOSED ? dr->wB[j] : 0.0f;
        wabs += fabsf(wb[j]);
    }
    const float inv2g = CLOSED ? dr->inv2g : 0.0f;
    // the first pixel's record, requested before the tables are staged:
    // lane i < 16 holds g0_i and n0_i, lanes 8..15 also s_{i-8}, lane 0 K,
    // lane 1 mu (vector loads, one pixel ahead from here on)
    // (read unconditionally, from the last pixel for waves past the end:
    // P >= 1, and no branch holds the staging below behind these loads)
    const int64_t w0 = wave < P ? wave : P - 1;
    // byte offset of the lane's float in the record (s_{li-8}, mu or K),
    // fixed per lane, so the per-pixel read is one load without branches
    const int soff = li >= 8 ? (int)offsetof(PixRec, s) + 4 * (li - 8)
                             : (li == 1 ? (int)offsetof(PixRec, mu) : (int)offsetof(PixRec, K));
    auto rec_f = [&](int64_t i) -> float {
        return *reinterpret_cast<const float *>(reinterpret_cast<const char *>(pr + i) + soff);
    };
    double gnext = pr[w0].g0[li];
    int nnext = pr[w0].n0[li];
    float snext = rec_f(w0);
    uint32_t fnext = PRUNED ? pr[w0].free : 0u;
    int knext = CLOSED ? pr[w0].k : 0;
    float egnext = pr[w0].eg;
    {
        // the diagram's tables, one entry per thread (the blocks are 256
        // threads): every read issued before the first LDS write, so the
        // staging is one round trip
        const int e = threadIdx.x;
        const int r8 = (e & 127) >> 3, c8 = e & 7;
        const float t1 = dr->T1[r8][c8], t2 = dr->T2[r8][c8];
        const double t1d = dr->T1d[r8][c8], t2d = dr->T2d[r8][c8];
        const float hh = dr->Hhi[e], hs = dr->Hs[e], hl = dr->hlo[e];
        const double hhd = dr->Hhid[e], hld = dr->hlod[e];
        if (e < 128) {
            sT1[r8][c8] = t1;
            sT2[r8][c8] = t2;
            sT1d[r8][c8] = t1d;
            sT2d[r8][c8] = t2d;
        }
        sH[e] = hh;
        sHd[e] = hhd;
        sLd[e] = hld;
        sHs[e] = hs;
        sHlo[e] = hl;
    }
    if (threadIdx.x == 0) { sflag = 0; sgap = 0; srows = 0; scand = 0; }
    __syncthreads();

    // pixel-independent column operands (as in the dense scorer), from the
    // staged h_lo table: the B operand of column tile ct for this lane
    auto col_operand = [&](int ct) -> uint4 {
        const int clo = ct * 16 + mrow;
        const float h = sHlo[clo];
        uint4 w;
        if (PREC == kPrecFP32) {
            w.x = fbits((float)((clo >> q) & 1));
            w.y = fbits((float)((clo >> (4 + q)) & 1));
            w.z = fbits(h);  // h_lo of the lane's column, added with C before the products
            w.w = 0u;
        } else if (q < 3) {
            uint32_t d4[4];
#pragma unroll
            for (int d = 0; d < 4; ++d)
                d4[d] = ((clo >> (2 * d) & 1) ? 0x3F80u : 0u) |
                        ((clo >> (2 * d + 1) & 1) ? 0x3F800000u : 0u);
            w = make_uint4(d4[0], d4[1], d4[2], d4[3]);
        } else {
            const float h1 = trunc16(h);
            const float r = h - h1;
            const float h2 = trunc16(r);
            const float h3 = r - h2;
            w = make_uint4(0x3F803F80u, 0x3F80u | (fbits(h1) & 0xFFFF0000u), pack2(h2, h3), 0u);
        }
        return w;
    };
    // in LDS, one table per block (the operands depend on the lane, not the
    // wave): wave w builds column tiles 4 w .. 4 w + 3.  The near-tie sweep
    // reads them there; the main sweep too, or from registers.
#pragma unroll
    for (int k = 0; k < 4; ++k) sB[4 * wv + k][lane] = col_operand(4 * wv + k);
    __syncthreads();
    auto bop_lds = [&](int ct) -> uint4 { return sB[ct][lane]; };
#if QA_BOUND_B_LDS
    // the first QA_BOUND_B_REGS column tiles' operands also in registers
    // (less LDS traffic per product), the others read from LDS
    // (split-BF16 forms only: the FP32 form's registers are taken)
    constexpr int kBRegs = PREC == kPrecFP32 ? 0 : QA_BOUND_B_REGS;
    uint4 bw[kBRegs > 0 ? kBRegs : 1];
#pragma unroll
    for (int ct = 0; ct < kBRegs; ++ct) bw[ct] = col_operand(ct);
    auto bop = [&](int ct) -> uint4 { return ct < kBRegs ? bw[ct] : bop_lds(ct); };
#else
    // in registers for the whole kernel
    uint4 bw[16];
#pragma unroll
    for (int ct = 0; ct < 16; ++ct) bw[ct] = col_operand(ct);
    auto bop = [&](int ct) -> uint4 { return bw[ct]; };
#endif
    // constant chunk of an unused row: C = 1e30, so its states never win
    uint2 csent;
    {
        const float C = 1e30f;
        const float c1 = trunc16(C);
        const float cr = C - c1;
        const float c2 = trunc16(cr);
        csent = (PREC == kPrecFP32) ? make_uint2(fbits(C), 0u)
                                    : make_uint2(pack2(c1, c2), pack2(cr - c2, 1.0f));
    }

    int64_t nflag = 0, ngap = 0, nrows = 0, ncand = 0;
    uint8_t *list = sList[wv];
    double *g64 = sG64[wv];
    float *ptab = sPt[wv];
    float *win = sWin[wv];
    for (int64_t p = wave; p < P; p += nwaves) {
        const double gcur = gnext;
        const int ncur = nnext;
        const float scur = snext;
        // free dots, raised count and guess of the pixel (wave-uniform)
        const uint32_t F = PRUNED ? __builtin_amdgcn_readfirstlane(fnext) : 0xFFFFu;
        const int kc = CLOSED ? __builtin_amdgcn_readfirstlane(knext) : 0;
        const float egf = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(egnext)));
        if (p + nwaves < P) {
            gnext = pr[p + nwaves].g0[li];
            nnext = pr[p + nwaves].n0[li];
            snext = rec_f(p + nwaves);
            if (PRUNED) fnext = pr[p + nwaves].free;
            if (CLOSED) knext = pr[p + nwaves].k;
            egnext = pr[p + nwaves].eg;
        }
        // g0 beyond n is zero in the record.  Thresholded and closed sets: a
        // fixed dot's entry carries the penalty 2^100 (states raising it never
        // win; the others score as in the dense form), the error bound takes
        // the unpenalised values.
        const float gl = (float)gcur;
        const float glp = (PRUNED && !(F >> li & 1u)) ? 0x1p100f : gl;
        float g[16];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            g[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(glp), i));
        // sum |g_i| (every 16-lane row holds g0_0..15)
        const float gabs = __int_as_float(__builtin_amdgcn_readfirstlane(
            __float_as_int(row_sumf(fabsf(gl)))));
        const uint32_t Fhi = (F >> 8) & 0xFFu;
        const int nflo = __popc(F & 0xFFu);
        if (MODE == kPruned) ncand += 1ll << __popc(F & ((1u << n) - 1u));
        if (CLOSED) {
            // C(free dots, k)
            const int nf = __popc(F & ((1u << n) - 1u));
            int64_t bc = 1;
            for (int j = 0; j < kc && j < nf; ++j) bc = bc * (nf - j) / (j + 1);
            ncand += (kc >= 0 && kc <= nf) ? bc : 0;
        }
        // ---- the bound terms of the setup: s = S (n0 - x_u)_hi and K ----
        if (lane < kMaxDot) g64[lane] = gcur;  // FP64 g of the near-tie re-score
        float sb[8];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            sb[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(scur), 8 + i));
        const float sabs = __int_as_float(__builtin_amdgcn_readfirstlane(
            __float_as_int(row_sumf(li >= 8 ? fabsf(scur) : 0.0f))));
        const float Kf = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(scur), 0));
        const float muf = CLOSED ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(scur), 1))
                                 : 0.0f;
        // Certified bound on |E_approx - E| (as in the dense scorer), and the
        // FP32 error of the bound: at most a dozen roundings of partial sums
        // that are bounded by |K| + sum|s| + 1/2 sum|S|; 2^-19 of that covers
        // them with room to spare.
        const float S = gabs + sumabs;
        const float delta = (PREC == kPrecX2 ? 0x1p-15f : 0x1p-17f) * S;
        // closed: the low-sum term (m - mu - w^T b_hi)^2 / (2 gamma) adds the
        // FP32 error of a square of terms bounded by 8 + |mu| + sum|w|
        const float lsum = 8.0f + fabsf(muf) + wabs;
        const float margin = 4.0f * delta + 0x1p-19f * (fabsf(Kf) + sabs + hsabs) +
                             (CLOSED ? 0x1p-19f * lsum * lsum * inv2g : 0.0f);

        // ---- per lane: the bounds of high indices (q + 4 e4) * 16 + row.
        // Bits 0..3 of the index are the lane's row, bits 4 and 5 its quarter
        // q, bits 6 and 7 the compile-time e4: the lane's part of b_hi^T s
        // (and of w^T b_hi, popc) is summed once, e4's part added per index.
        float Rb = Kf, Wb = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (mrow >> j & 1) {
                Rb += sb[j];
                Wb += wb[j];
            }
        }
        if (q & 1) { Rb += sb[4]; Wb += wb[4]; }
        if (q & 2) { Rb += sb[5]; Wb += wb[5]; }
        const float s67 = sb[6] + sb[7], w67 = wb[6] + wb[7];
        const int pcl = __popc((uint32_t)mrow) + __popc((uint32_t)q);
        float lb[4];
#pragma unroll
        for (int e4 = 0; e4 < 4; ++e4) {
            const int rt = q + 4 * e4;
            const int chi = rt * 16 + mrow;
            const float R = e4 == 0 ? Rb : Rb + (e4 == 1 ? sb[6] : (e4 == 2 ? sb[7] : s67));
            float L = R + sHs[chi];
            bool ok = rt < nrt;
            if (PRUNED) ok = ok && !((uint32_t)chi & ~Fhi);  // raises a fixed high dot
            if (CLOSED) {
                // m raised low dots: none of this high part's states is admissible
                // unless 0 <= m <= free low dots
                const int m = kc - (pcl + __popc((uint32_t)e4));
                const float W = e4 == 0 ? Wb : Wb + (e4 == 1 ? wb[6] : (e4 == 2 ? wb[7] : w67));
                const float dm = ((float)m - muf) - W;
                L += dm * dm * inv2g;
                ok = ok && m >= 0 && m <= nflo;
            }
            lb[e4] = ok ? L : INFINITY;
        }
        // b_hi^T g_hi over the low four and the high four bits of the high
        // index (lanes 0..15 and 16..31), for the constant chunks
        // C(c_hi) = b_hi^T g_hi + 1/2 b_hi^T A_HH b_hi of the scored rows
        if (lane < 32) {
            float v = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (li >> j & 1) v += (lane < 16) ? g[8 + j] : g[12 + j];
            ptab[lane] = v;
        }
        // The rows to score.  The setup's guess (the rounding of x* and its
        // best single flip when that lowers the energy; closed: the k free
        // dots with the largest fractional parts) is a state of
        // the candidate set; its energy E_g (FP64 in the setup, rounded to
        // FP32) bounds the approximate best from above (by E_g + 1.1 delta),
        // so a high part whose bound exceeds E_g + margin + delta holds
        // neither the argmin nor a near-tie state.  When at most two tiles'
        // worth of high parts pass that test they are the rows (most pixels);
        // otherwise the row tile with the smallest bound is scored first and
        // the high parts within the margin of its best (and under the first
        // threshold) follow.
        int rts = -1;
        int cnt = 0;  // scored rows (wave-uniform)
        // appends the high indices whose bound is at most thr (except those
        // of row tile skip_rt) to the list after position cnt
        auto list_rows = [&](float thr, int skip_rt) {
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) {
                const int rt = q + 4 * e4;
                const bool take = lb[e4] <= thr && rt != skip_rt;
                const unsigned long long m = __ballot(take);
                if (take)
                    list[cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0))] =
                        (uint8_t)(rt * 16 + mrow);
                cnt += __popcll(m);
            }
        };
        const float thr_g = egf + margin + delta;
        int ng = 0;
#pragma unroll
        for (int e4 = 0; e4 < 4; ++e4) ng += __popcll(__ballot(lb[e4] <= thr_g));
        const bool by_guess = ng <= 32;
        // wave priority by the wave's remaining work: the kernel ends with
        // the waves whose pixels score more than one tile of rows and with
        // those that still hold a pixel after this one, so while the SIMDs
        // are shared those waves issue first (two levels for a pixel of more
        // than one tile, one for a pixel still to come; 3 in the near-tie
        // re-score below)
        {
            const int lv = __builtin_amdgcn_readfirstlane((ng > 16 ? 2 : 0) + (p + nwaves < P ? 1 : 0));
            if (lv == 3) __builtin_amdgcn_s_setprio(3);
            else if (lv == 2) __builtin_amdgcn_s_setprio(2);
            else if (lv == 1) __builtin_amdgcn_s_setprio(1);
            else __builtin_amdgcn_s_setprio(0);
        }
        if (by_guess) {
            list_rows(thr_g, -1);
        } else {
            float rlb[4];
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) rlb[e4] = row_min(lb[e4]);
            float mb = rlb[0];
            int me = 0;
#pragma unroll
            for (int e4 = 1; e4 < 4; ++e4)
                if (rlb[e4] < mb) { mb = rlb[e4]; me = e4; }
            const float gmb = rows_min(mb);
            const unsigned long long hb = __ballot(mb == gmb);
            const int wl = __ffsll((long long)hb) - 1;
            rts = __builtin_amdgcn_readlane(q + 4 * me, wl);
            if (lane < 16) list[lane] = (uint8_t)(rts * 16 + lane);
            cnt = 16;
        }
        wave_sync();  // the row list and the b_hi^T g_hi tables

        // g_{2q}, g_{2q+1} (split-BF16 forms) or g_q, g_{4+q} (FP32) of this lane
        float ga = g[0], gb = g[1];
#pragma unroll
        for (int d = 1; d < 4; ++d) {
            if (q == d) {
                ga = (PREC == kPrecFP32) ? g[d] : g[2 * d];
                gb = (PREC == kPrecFP32) ? g[4 + d] : g[2 * d + 1];
            }
        }
        if (PREC == kPrecFP32) gb = (q == 0) ? g[4] : gb;

        auto ct_ok = [&](int ct) { return !PRUNED || !(((uint32_t)ct << 4) & ~F & 0xF0u); };
        // C(c_hi) in FP32: the same sums as b_hi^T g_hi + table
        auto cconst = [&](int chi) { return (ptab[chi & 15] + ptab[16 + (chi >> 4)]) + sH[chi]; };
        // closed: popcounts of this lane's four elements of tile t less that of
        // the column tile (rows 4q..4q+3, column bits mrow)
        auto elem_pc = [&](int t, int (&eq)[4]) {
            if (CLOSED) {
                const uint32_t r4 = *reinterpret_cast<const uint32_t *>(&list[t * 16 + 4 * q]);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    eq[i] = __popc((r4 >> (8 * i)) & 0xFFu) + __popc((uint32_t)mrow);
            }
        };
        // closed: elements whose state does not raise exactly k dots are +inf
        auto qualify = [&](f32x4_t d, const int (&eq)[4], int ct) -> f32x4_t {
            if (CLOSED) {
                const int r = kc - __popc((uint32_t)ct);
#pragma unroll
                for (int i = 0; i < 4; ++i) d[i] = (eq[i] == r) ? d[i] : INFINITY;
            }
            return d;
        };
        // The A operand of tile t (row r of the tile is high index
        // list[16 t + r]; unused rows past cnt get the sentinel constant
        // chunk), in two steps so that the next tile's LDS reads are in
        // flight while this tile is on the matrix core: fetch reads the
        // tables, assemble forms the operand.
        struct Rows {
            float t1a, t1b, t2a, t2b;  // T1 and T2 entries of the lane's two dots
            float c[4];                // X3/X2: c[0] = C of the lane's row; FP32: C of rows 4q + i
            bool real;
        };
        auto fetch = [&](int t) -> Rows {
            Rows r;
            const int idx = t * 16 + mrow;
            r.real = idx < cnt;
            const int chi = r.real ? (int)list[idx] : 0;
            const int row = chi & 15, rtt = chi >> 4;
            const int da = (PREC == kPrecFP32) ? q : 2 * q;
            const int db = (PREC == kPrecFP32) ? 4 + q : 2 * q + 1;
            r.t1a = sT1[row][da];
            r.t1b = sT1[row][db];
            r.t2a = sT2[rtt][da];
            r.t2b = sT2[rtt][db];
            if (PREC == kPrecFP32) {
                // C of the four output rows 4q..4q+3 of this lane: the
                // accumulator starts at C(row) + h_lo(column), so two
                // K = 4 products per tile suffice
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int ri = t * 16 + 4 * q + i;
                    r.c[i] = ri < cnt ? cconst(list[ri]) : 1e30f;
                }
            } else {
                r.c[0] = r.real ? cconst(chi) : 0.0f;
            }
            return r;
        };
        auto assemble = [&](const Rows &r, Pack8 &a, float (&af)[6]) {
            const float v0 = (ga + r.t1a) + r.t2a;
            const float v1 = (gb + r.t1b) + r.t2b;
            if (PREC == kPrecFP32) {
                af[0] = v0;
                af[1] = v1;
#pragma unroll
                for (int i = 0; i < 4; ++i) af[2 + i] = r.c[i];
            } else {
                uint2 cw = csent;
                if (r.real) {
                    const float C = r.c[0];
                    const float c1 = trunc16(C);
                    const float cr = C - c1;
                    const float c2 = trunc16(cr);
                    cw = make_uint2(pack2(c1, c2), pack2(cr - c2, 1.0f));
                }
                uint32_t R0, R1, R2;
                if (PREC == kPrecX3) {
                    const float a0 = trunc16(v0), b0 = trunc16(v1);
                    const float r0 = v0 - a0, s0 = v1 - b0;
                    const float a1 = trunc16(r0), b1 = trunc16(s0);
                    R0 = pack2(a0, b0);
                    R1 = pack2(a1, b1);
                    R2 = pack2(r0 - a1, s0 - b1);
                } else {
                    const float a0 = rne16(v0), b0 = rne16(v1);
                    R0 = pack2(a0, b0);
                    R1 = pack2(rne16(v0 - a0), rne16(v1 - b0));
                    R2 = 0u;
                }
                uint32_t R3 = (q == 2) ? 0x3F803F80u : 0u;
                R3 = (q == 1) ? cw.y : R3;
                R3 = (q == 0) ? cw.x : R3;
                const auto t02 = __builtin_amdgcn_permlane32_swap(R0, R2, false, false);
                const auto t13 = __builtin_amdgcn_permlane32_swap(R1, R3, false, false);
                const auto u01 = __builtin_amdgcn_permlane16_swap(t02[0], t13[0], false, false);
                const auto u23 = __builtin_amdgcn_permlane16_swap(t02[1], t13[1], false, false);
                a.u[0] = u01[0];
                a.u[1] = u01[1];
                a.u[2] = u23[0];
                a.u[3] = u23[1];
            }
        };
        auto build_rows = [&](int t, Pack8 &a, float (&af)[6]) { assemble(fetch(t), a, af); };
        auto tile = [&](const Pack8 &a, const float (&af)[6], int ct,
                        bool from_lds = false) -> f32x4_t {
            f32x4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
            const uint4 bb = from_lds ? bop_lds(ct) : bop(ct);
            if (PREC == kPrecFP32) {
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[i] = af[2 + i] + __uint_as_float(bb.z);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[0], __uint_as_float(bb.x), acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(af[1], __uint_as_float(bb.y), acc, 0, 0, 0);
            } else {
                Pack8 b;
                b.u[0] = bb.x; b.u[1] = bb.y; b.u[2] = bb.z; b.u[3] = bb.w;
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc, 0, 0, 0);
            }
            return acc;
        };
        // the four column tiles 4 cg .. 4 cg + 3 of row tile (a, af): the
        // lane's 16 elements (element 4 k + i: column tile 4 cg + k, output
        // row 4 q + i); column tiles without a candidate read +inf
        auto group = [&](const Pack8 &a, const float (&af)[6], const int (&eq)[4], auto cgc,
                         f32x4_t (&d)[4]) {
            constexpr int cg = decltype(cgc)::value;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ct = 4 * cg + k;
                if (ct_ok(ct)) d[k] = qualify(tile(a, af, ct), eq, ct);
                else d[k] = f32x4_t{INFINITY, INFINITY, INFINITY, INFINITY};
            }
        };
        // Per lane: the three smallest group minima b1 <= b2 <= b3 and the
        // group codes 4 t + cg of the first two (a1, a2), a group being the
        // lane's 16 elements of four column tiles.  The A operand of tile 0 is
        // kept for the winner's group.
        float b1 = INFINITY, b2 = INFINITY, b3 = INFINITY;
        int a1 = 0, a2 = 0;
        uint32_t ac0 = 0, ac1 = 0, ac2 = 0, ac3 = 0;  // A operand of tile 0
        float afc0 = 0.0f, afc1 = 0.0f, afc2 = 0.0f, afc3 = 0.0f, afc4 = 0.0f, afc5 = 0.0f;
        auto score = [&](int t, const Pack8 &a, const float (&af)[6]) {
            int eq[4];
            elem_pc(t, eq);
            sfor<0, 4>([&](auto cgc) {
                constexpr int cg = decltype(cgc)::value;
                float m = INFINITY;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int ct = 4 * cg + k;
                    if (!ct_ok(ct)) continue;
                    const f32x4_t d = qualify(tile(a, af, ct), eq, ct);
                    m = __builtin_fminf(m, __builtin_fminf(d[0], d[1]));
                    m = __builtin_fminf(m, __builtin_fminf(d[2], d[3]));
                }
                const int code = 4 * t + cg;
                // the group codes by bitwise selects (the compiler turns
                // nested conditional moves into branches here)
                const int lt1 = -(int)(m < b1), lt2 = -(int)(m < b2);
                const int n2 = a2 ^ ((code ^ a2) & lt2);
                b3 = __builtin_amdgcn_fmed3f(b2, b3, m);
                a2 = n2 ^ ((a1 ^ n2) & lt1);
                b2 = __builtin_amdgcn_fmed3f(b1, b2, m);
                a1 = a1 ^ ((code ^ a1) & lt1);
                b1 = __builtin_fminf(b1, m);
                // one group's products in flight at a time (their results
                // are 16 registers)
                __builtin_amdgcn_sched_barrier(0);
            });
        };
        // tiles t0 .. t1 - 1, the next tile's tables read while this one is
        // scored
        auto score_range = [&](int t0, int t1) {
            Rows rn = fetch(t0);
            for (int t = t0; t < t1; ++t) {
                Pack8 a;
                float af[6];
                assemble(rn, a, af);
                if (t + 1 < t1) rn = fetch(t + 1);
                if (t == 0) {
                    ac0 = a.u[0]; ac1 = a.u[1]; ac2 = a.u[2]; ac3 = a.u[3];
                    afc0 = af[0]; afc1 = af[1]; afc2 = af[2];
                    afc3 = af[3]; afc4 = af[4]; afc5 = af[5];
                }
                score(t, a, af);
            }
        };
        if (!by_guess) {
            score_range(0, 1);
            // the other high indices whose bound admits a state within the
            // margin of the best so far, after the first row tile's 16
            list_rows(fminf(wave_min(b1) + margin, thr_g), rts);
            wave_sync();
        }
        const int ntiles = (cnt + 15) >> 4;
        score_range(by_guess ? 0 : 1, ntiles);
        nrows += cnt;

        // ---- best over the wave (the smallest and second smallest group
        // minima of all lanes in one reduction), runner-up bound, winner's
        // group once more ----
        float m1 = b1, m2 = INFINITY;
        auto pair_step = [&](float o1, float o2) {
            const float n2 = __builtin_fminf(__builtin_fmaxf(m1, o1), __builtin_fminf(m2, o2));
            m1 = __builtin_fminf(m1, o1);
            m2 = n2;
        };
        pair_step(dppf<kDppXor1>(m1), dppf<kDppXor1>(m2));
        pair_step(dppf<kDppXor2>(m1), dppf<kDppXor2>(m2));
        pair_step(dppf<kDppHalfMirror>(m1), dppf<kDppHalfMirror>(m2));
        pair_step(dppf<kDppMirror>(m1), dppf<kDppMirror>(m2));
        {
            auto swap_pair = [&](auto swap) {
                const auto s1 = swap(__float_as_uint(m1));
                const auto s2 = swap(__float_as_uint(m2));
                m1 = __uint_as_float(s1[0]);
                m2 = __uint_as_float(s2[0]);
                pair_step(__uint_as_float(s1[1]), __uint_as_float(s2[1]));
            };
            swap_pair([](uint32_t v) { return __builtin_amdgcn_permlane16_swap(v, v, false, false); });
            swap_pair([](uint32_t v) { return __builtin_amdgcn_permlane32_swap(v, v, false, false); });
        }
        const float wmin = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m1)));
        const float wsec = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(m2)));
        const unsigned long long hit = __ballot(b1 == wmin);
        const int winner = __ffsll((long long)hit) - 1;
        const float other = fminf(wsec, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(b2), winner)));
        const int aw = __builtin_amdgcn_readlane(a1, winner);
        const int tw = aw >> 2, cgw = aw & 3;
        {
            Pack8 a;
            float af[6];
            if (tw == 0) {
                a.u[0] = ac0; a.u[1] = ac1; a.u[2] = ac2; a.u[3] = ac3;
                af[0] = afc0; af[1] = afc1; af[2] = afc2;
                af[3] = afc3; af[4] = afc4; af[5] = afc5;
            } else {
                build_rows(tw, a, af);
            }
            int eq[4];
            elem_pc(tw, eq);
            f32x4_t d[4] = {};
            sfor<0, 4>([&](auto cgc) {
                if (decltype(cgc)::value == cgw) group(a, af, eq, cgc, d);
            });
            if (lane == winner) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int i = 0; i < 4; ++i) win[4 * k + i] = d[k][i];
            }
        }
        wave_sync();
        // lanes 0..15: element `lane` of the winner's group; the best, its
        // first position and the second best by row reductions
        const float x = lane < 16 ? win[lane] : INFINITY;
        const float e1 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(row_min(x))));
        const int jw = __ffsll((long long)__ballot(lane < 16 && x == e1)) - 1;
        const float x2 = lane == jw ? INFINITY : x;
        const float v2 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(row_min(x2))));
        const float e2 = fminf(other, v2);
        const bool tie = !(e2 - e1 > 2.0f * delta);
        if (!tie) {
            if (lane < n) {
                const int ctw = 4 * cgw + (jw >> 2);
                const int row = 4 * (winner >> 4) + (jw & 3);
                const uint32_t chi = list[tw * 16 + row];
                const uint32_t clo = (uint32_t)(ctw * 16 + (winner & 15));
                const uint32_t b = clo | (chi << 8);
                n_out[p * n + lane] = ncur + (int32_t)((b >> lane) & 1u);
            }
            continue;
        }
        // ---- near tie: the exact argmin is one of the scored states whose
        // approximate energy lies within 2 delta of the best (the band).  The
        // groups that hold them are swept once more, the in-band states are
        // gathered into a per-wave list (state codes clo | chi << 8), and the
        // lanes score them in FP64, one state each, from the split tables
        //   U(n0 + b) - U(n0) = h_lo(c_lo) + H_hi(c_hi) + b_hi^T g_hi
        //                     + b_lo^T (g_lo + A_LH b_hi)
        // keeping the smallest (ties to the lexicographically smallest
        // state) ----
        ++nflag;
        __builtin_amdgcn_s_setprio(3);
        const float thr = e1 + 2.0f * delta;
        double c1best = INFINITY, c2best = INFINITY;
        uint32_t cbest = 0;
        uint32_t *band = sBand[wv];
        int nb = 0;  // states in the band list (wave-uniform)
        auto flush = [&]() {
            wave_sync();
            for (int j = lane; j < nb; j += 64) {
                // keep the FP64 tables in LDS (loads not hoisted into registers)
                __asm__ volatile("" ::: "memory");
                const uint32_t c = band[j];
                const uint32_t clo = c & 0xFFu, chi = c >> 8;
                const int row = chi & 15, rth = chi >> 4;
                double e = sLd[clo] + sHd[chi];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    if (chi >> i & 1u) e += g64[8 + i];
                    if (clo >> i & 1u) e += (g64[i] + sT1d[row][i]) + sT2d[rth][i];
                }
                if (e < c1best || (e == c1best && __brev(c) < __brev(cbest))) {
                    c2best = c1best; c1best = e; cbest = c;
                } else {
                    c2best = fmin(c2best, e);
                }
            }
            wave_sync();
            nb = 0;
        };
        // the in-band states of column tile ct of row tile (a, af) = tile t
        // into the band list
        auto gather = [&](int t, const Pack8 &a, const float (&af)[6], const int (&eq)[4], int ct) {
            if (!ct_ok(ct)) return;
            const f32x4_t d = qualify(tile(a, af, ct, true), eq, ct);
            const float dm = fminf(fminf(d[0], d[1]), fminf(d[2], d[3]));
            if (!__ballot(dm <= thr)) return;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool in = d[i] <= thr;
                const unsigned long long m = __ballot(in);
                if (in) {
                    const uint32_t chi = list[t * 16 + 4 * q + i];
                    band[nb + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0))] =
                        (uint32_t)(ct * 16 + mrow) | (chi << 8);
                }
                nb += __popcll(m);
                if (nb >= 64) flush();
            }
        };
        auto operand = [&](int t, Pack8 &a, float (&af)[6]) {
            if (t == 0) {
                a.u[0] = ac0; a.u[1] = ac1; a.u[2] = ac2; a.u[3] = ac3;
                af[0] = afc0; af[1] = afc1; af[2] = afc2;
                af[3] = afc3; af[4] = afc4; af[5] = afc5;
            } else {
                build_rows(t, a, af);
            }
        };
        if (!__ballot(b3 <= thr)) {
            // no lane has a third group in the band: the in-band states lie
            // in the groups a1 (where b1 <= thr) and a2 (where b2 <= thr) of
            // the lanes; those groups (a mask over the codes 4 t + cg < 64)
            // once more
            uint64_t gm = (b1 <= thr ? 1ull << a1 : 0ull) | (b2 <= thr ? 1ull << a2 : 0ull);
            gm = wave_or64(gm);
            while (gm) {
                const int gc = __ffsll((long long)gm) - 1;
                gm &= gm - 1;
                const int t = gc >> 2, cgs = gc & 3;
                Pack8 a;
                float af[6];
                int eq[4];
                operand(t, a, af);
                elem_pc(t, eq);
#pragma unroll
                for (int k = 0; k < 4; ++k) gather(t, a, af, eq, 4 * cgs + k);
            }
        } else {
            // otherwise every scored row tile
            for (int t = 0; t < ntiles; ++t) {
                Pack8 a;
                float af[6];
                int eq[4];
                operand(t, a, af);
                elem_pc(t, eq);
                for (int ct = 0; ct < 16; ++ct) gather(t, a, af, eq, ct);
            }
        }
        if (nb) flush();
        // (best, runner-up, state) over the wave: exchange with the partner
        // lanes of the row steps, then combine the swapped rows
        auto merge = [&](double ob1, double ob2, uint32_t oc1) {
            if (ob1 < c1best || (ob1 == c1best && __brev(oc1) < __brev(cbest))) {
                c2best = fmin(c1best, ob2); c1best = ob1; cbest = oc1;
            } else {
                c2best = fmin(c2best, ob1);
            }
        };
        merge(dppd<kDppXor1>(c1best), dppd<kDppXor1>(c2best), dpp32<kDppXor1>(cbest));
        merge(dppd<kDppXor2>(c1best), dppd<kDppXor2>(c2best), dpp32<kDppXor2>(cbest));
        merge(dppd<kDppHalfMirror>(c1best), dppd<kDppHalfMirror>(c2best),
              dpp32<kDppHalfMirror>(cbest));
        merge(dppd<kDppMirror>(c1best), dppd<kDppMirror>(c2best), dpp32<kDppMirror>(cbest));
        {
            // rows 2k and 2k + 1, then the two halves: the swaps hand each lane
            // its own value and the partner's, in an order that depends on the
            // lane, so both are merged into a fresh triple
            auto swap_merge = [&](auto swap) {
                const uint64_t u1 = (uint64_t)__double_as_longlong(c1best);
                const uint64_t u2 = (uint64_t)__double_as_longlong(c2best);
                const auto l1 = swap((uint32_t)u1), h1 = swap((uint32_t)(u1 >> 32));
                const auto l2 = swap((uint32_t)u2), h2 = swap((uint32_t)(u2 >> 32));
                const auto cc = swap(cbest);
                const double x1 = __longlong_as_double((long long)((uint64_t)l1[0] | ((uint64_t)h1[0] << 32)));
                const double y1 = __longlong_as_double((long long)((uint64_t)l1[1] | ((uint64_t)h1[1] << 32)));
                const double x2 = __longlong_as_double((long long)((uint64_t)l2[0] | ((uint64_t)h2[0] << 32)));
                const double y2 = __longlong_as_double((long long)((uint64_t)l2[1] | ((uint64_t)h2[1] << 32)));
                c1best = x1; c2best = x2; cbest = cc[0];
                merge(y1, y2, cc[1]);
            };
            swap_merge([](uint32_t v) { return __builtin_amdgcn_permlane16_swap(v, v, false, false); });
            swap_merge([](uint32_t v) { return __builtin_amdgcn_permlane32_swap(v, v, false, false); });
        }
        if (lane < n) n_out[p * n + lane] = ncur + (int32_t)((cbest >> lane) & 1u);
        if (lane == 0 && c2best - c1best < 1e-9) ++ngap;
    }
    if (lane == 0) {
        if (nflag) atomicAdd(&sflag, (unsigned long long)nflag);
        if (ngap) atomicAdd(&sgap, (unsigned long long)ngap);
        if (nrows) atomicAdd(&srows, (unsigned long long)nrows);
        if (ncand) atomicAdd(&scand, (unsigned long long)ncand);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        block_add_counter(counters, C_NEAR_TIE, (int64_t)sflag);
        block_add_counter(counters, C_GAP_1E9, (int64_t)sgap);
        block_add_counter(counters, C_SCORED, (int64_t)srows << 8);  // 256 states per row
        if (PRUNED) block_add_counter(counters, C_CANDIDATES, (int64_t)scand);  // summed per pixel
        else if (blockIdx.x == 0) block_add_counter(counters, C_CANDIDATES, P << n);
    }
}

// blocks of 256 threads of a scorer kernel that fit on the device at once
// (cached per kernel slot and device; 0 if unknown)
template <typename Kernel>
static int resident_blocks(Kernel kernel, int slot)
{
    static int cache[24][64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || slot < 0 || slot >= 24) return 0;
    int &c = cache[slot][dev];
    if (c) return c;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
        per_cu <= 0)
        return 0;
    c = cus * per_cu;
    return c;
}

template <typename Kernel>
static hipError_t launch_persistent(Kernel kernel, int slot, const DiagRec *dr, const PixRec *pr,
                                    int64_t P, int32_t *n_out, int64_t *counters, hipStream_t s)
{
    // persistent waves: as many blocks as the chip keeps resident, at most
    // one wave per pixel
    int64_t blocks = (P + 3) / 4;
    const int resident = resident_blocks(kernel, slot);
    if (resident > 0 && blocks > resident) blocks = resident;
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(256), 0, s, dr, pr, P, n_out,
                       counters);
    return hipGetLastError();
}

hipError_t launch_score_mfma(const DiagRec *dr, const PixRec *pr, int64_t P, int prec, int mode,
                             bool exhaustive, int32_t *n_out, int64_t *counters, int n_dot,
                             hipStream_t s)
{
    if (n_dot < 9 || n_dot > 16 || mode < kDense || mode > kClosed) return hipErrorInvalidValue;
    if (P <= 0) return hipSuccess;
    if (n_dot >= 13 && !exhaustive) {
#define QA_BOUND_CASE(PR, MD, SLOT)                                                             \
    if (prec == PR && mode == MD)                                                               \
        return launch_persistent(k_score_bound<PR, MD>, SLOT, dr, pr, P, n_out, counters, s);
        QA_BOUND_CASE(kPrecFP32, kDense, 9)
        QA_BOUND_CASE(kPrecX3, kDense, 10)
        QA_BOUND_CASE(kPrecX2, kDense, 11)
        QA_BOUND_CASE(kPrecFP32, kPruned, 12)
        QA_BOUND_CASE(kPrecX3, kPruned, 13)
        QA_BOUND_CASE(kPrecX2, kPruned, 14)
        QA_BOUND_CASE(kPrecFP32, kClosed, 15)
        QA_BOUND_CASE(kPrecX3, kClosed, 16)
        QA_BOUND_CASE(kPrecX2, kClosed, 17)
#undef QA_BOUND_CASE
        return hipErrorInvalidValue;
    }
#define QA_SCORER_CASE(PR, MD, SLOT)                                                            \
    if (prec == PR && mode == MD)                                                               \
        return launch_persistent(k_score_mfma<PR, MD>, SLOT, dr, pr, P, n_out, counters, s);
    QA_SCORER_CASE(kPrecFP32, kDense, 0)
    QA_SCORER_CASE(kPrecX3, kDense, 1)
    QA_SCORER_CASE(kPrecX2, kDense, 2)
    QA_SCORER_CASE(kPrecFP32, kPruned, 3)
    QA_SCORER_CASE(kPrecX3, kPruned, 4)
    QA_SCORER_CASE(kPrecX2, kPruned, 5)
    QA_SCORER_CASE(kPrecFP32, kClosed, 6)
    QA_SCORER_CASE(kPrecX3, kClosed, 7)
    QA_SCORER_CASE(kPrecX2, kClosed, 8)
#undef QA_SCORER_CASE
    return hipErrorInvalidValue;
}

}  // namespace qa
