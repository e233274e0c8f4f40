// qa_kernels.hip -- gfx950 kernels of the constant-capacitance ground-state
// path (van Straaten et al., arXiv 2404.04994), except the matrix-core
// scorer (qa_mfma.hip).
//
//   k_prep      per diagram: A = C_dd^{-1} (FP64 Gauss-Jordan), C_dd 1, the
//               pixel-independent energy tables (Sec. 2, Eq. free_energy).
//   k_setup     per pixel (a group of lanes, lane = dot): x_u = C_gd V, the
//               analytic continuous minimum (Sec. 3.1.1, App. C/D) and, where
//               it is negative, the constrained minimum of Sec. 3.1.2 in FP64
//               by an active-set elimination across the group; then the
//               candidate set (Sec. 3.2) and the base-state gradient.
//   k_score_fp64  T = 0 argmin (Eq. argmin) over each pixel's candidate set,
//               FP64, a group of lanes per pixel walking a Gray code.
//   k_soft_fwd  kT > 0 softargmin (Sec. 4.2, Eq. softargmin), FP64.
//   k_soft_bwd  its adjoint with respect to C_dd, C_gd and V.
#include "qa_device.h"

namespace qa {

__global__ void k_zero_i64(int64_t *p, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_zero_i64(int64_t *p, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_i64, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_put_inputs(DiagRec *__restrict__ dr, const InputChunk c)
{
    if (c.part == 0) {
        if (threadIdx.x == 0) {
            dr->n = c.n;
            dr->g = c.g;
            dr->closed = c.closed;
            dr->nhat = c.nhat;
            dr->kT = c.kT;
            dr->t = c.t;
            dr->prec = c.prec;
            dr->pad0 = 0;
        }
        for (int e = threadIdx.x; e < kMaxDot * kMaxDot; e += blockDim.x) {
            const int i = e / kMaxDot, j = e % kMaxDot;
            dr->Cdd[e] = (i < c.n && j < c.n) ? c.v[i * c.n + j] : 0.0;
        }
    } else {
        const int rows = c.row1 - c.row0;
        for (int e = threadIdx.x; e < rows * kMaxGate; e += blockDim.x) {
            const int i = e / kMaxGate, j = e % kMaxGate, r = c.row0 + i;
            dr->Cgd[r * kMaxGate + j] = (r < c.n && j < c.g) ? c.v[i * c.g + j] : 0.0;
        }
    }
}

hipError_t launch_put_inputs(DiagRec *dr, const InputChunk &c, hipStream_t s)
{
    hipLaunchKernelGGL(k_put_inputs, dim3(1), dim3(256), 0, s, dr, c);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K0: per-diagram prologue, one 256-thread block per diagram
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPrepThreads) void k_prep(DiagRec *dr_all, int64_t *counters,
                                                      double *zero, int64_t nzero)
{
    __shared__ double sCdd[kMaxDot * kMaxDot];
    __shared__ double M[kMaxDot * kMaxDot];
    __shared__ double cvec[kMaxDot];
    __shared__ double red[8];
    // the call's counters (and accumulators) start at zero: no separate
    // memset or fill kernel in the launch sequence
    if (counters && blockIdx.x == 0)
        for (int i = threadIdx.x; i < kCounterWords; i += blockDim.x) counters[i] = 0;
    if (zero && blockIdx.x == 0)
        for (int64_t i = threadIdx.x; i < nzero; i += blockDim.x) zero[i] = 0.0;
    prep_body(dr_all + blockIdx.x, sCdd, M, cvec, red);
}

hipError_t launch_prep(DiagRec *dr, int n_diag, int64_t *counters, hipStream_t s, double *zero,
                       int64_t nzero)
{
    hipLaunchKernelGGL(k_prep, dim3(n_diag), dim3(kPrepThreads), 0, s, dr, counters, zero, nzero);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K1: continuous minimum, candidate set and base-state gradient.
//
// A group of NM lanes per pixel, lane i = dot i (NM = 16: four pixels per
// wave).  Every branch is uniform within a group and the shuffles read lanes
// of the same group only.  The matrices sit in LDS transposed, so that the
// lanes of a group read consecutive addresses.
//
// The QP of Sec. 3.1.2 (where the analytic minimum is negative) is solved in
// its KKT form: for the active set W (x_W = 0) the multipliers solve
// K_WW mu_W = -x0_W and the free dots follow as x = x0 + K_{.W} mu_W, with
// x0 the analytic minimum and K = C_dd (open) or C_dd - c c^T / 1^T c with
// c = C_dd 1 (closed: the equality multiplier eliminated).  The system is
// Gauss-Jordan eliminated on [K | x0], one pivot per dot of W (rows held by
// their lanes, the pivot row broadcast by shuffles): afterwards the column
// holds -mu_i on W and x_i off W.  The active set follows the primal-dual
// update (Hintermueller, Ito and Kunisch, SIAM J. Optim. 13, 2003): keep dots
// with mu > -tol, add dots with x < -tol, stop when W repeats.  Added dots are
// pivoted on the current elimination; a dot leaving W restarts it.  For open
// arrays C_dd is an M-matrix and W only grows (Chandrasekaran's method), so
// at most N pivots are taken.  Every non-pivot K_WW is a principal submatrix
// of a positive definite matrix (closed: on any proper subset of the dots),
// so no pivoting is needed.
// ---------------------------------------------------------------------------
template <int NM>
__device__ __forceinline__ uint32_t group_ballot(bool pred)
{
    const unsigned long long b = __ballot(pred);
    const int sh = (threadIdx.x & (kWave - 1)) & ~(NM - 1);
    return (uint32_t)((b >> sh) & ((1ull << NM) - 1ull));
}

// Group reductions: a group of 16 is a DPP row (row-local exchanges, no
// LDS); smaller groups use shuffles.
template <int NM>
__device__ __forceinline__ int group_isum(int v)
{
    if constexpr (NM == 16) {
        v += (int)dpp32<kDppXor1>((uint32_t)v);
        v += (int)dpp32<kDppXor2>((uint32_t)v);
        v += (int)dpp32<kDppHalfMirror>((uint32_t)v);
        return v + (int)dpp32<kDppMirror>((uint32_t)v);
    } else {
#pragma unroll
        for (int off = NM / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, NM);
        return v;
    }
}

template <int NM>
__device__ __forceinline__ double group_dsum(double v)
{
    if constexpr (NM == 16) {
        return row_sum(v);
    } else {
#pragma unroll
        for (int off = NM / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, NM);
        return v;
    }
}

template <int NM>
__device__ __forceinline__ double group_dmax(double v)
{
    if constexpr (NM == 16) {
        v = fmax(v, dppd<kDppXor1>(v));
        v = fmax(v, dppd<kDppXor2>(v));
        v = fmax(v, dppd<kDppHalfMirror>(v));
        return fmax(v, dppd<kDppMirror>(v));
    } else {
#pragma unroll
        for (int off = NM / 2; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, NM));
        return v;
    }
}

// z of lane Q of the caller's group (NM = 16: a DPP row broadcast)
template <int NM, int Q>
__device__ __forceinline__ double group_bcast(double z, int base)
{
    if constexpr (NM == 16)
        return dppd<kDppRowBcast0 + Q>(z);
    else
        return __shfl(z, base + Q, kWave);
}


// One Gauss-Jordan pivot on dot k of [K | x]: lane `dot` holds row `dot` in
// r[] and its right-hand side in v; `base` is the group's first lane.
template <int NM>
__device__ __forceinline__ void gj_pivot(double (&r)[NM], double &v, int k, int dot, int base)
{
    const int src = base + k;
    double rik = r[0];
#pragma unroll
    for (int q = 1; q < NM; ++q) rik = (k == q) ? r[q] : rik;
    const double piv = __shfl(rik, src, kWave);
    double pr[NM];
#pragma unroll
    for (int q = 0; q < NM; ++q) pr[q] = __shfl(r[q], src, kWave);
    const double pv = __shfl(v, src, kWave);
    const double rp = recip_nr(piv);
    if (dot == k) {
#pragma unroll
        for (int q = 0; q < NM; ++q) r[q] = pr[q] * rp;
        v = pv * rp;
    } else {
        const double f = rik * rp;
#pragma unroll
        for (int q = 0; q < NM; ++q) r[q] -= f * pr[q];
        v -= f * pv;
    }
}

// The same pivot with k fixed at compile time, for 16-lane groups (a DPP
// row): the pivot row, right-hand side and pivot come by row broadcasts.
template <int NM, int K>
__device__ __forceinline__ void gj_pivot_row(double (&r)[NM], double &v, int dot)
{
    static_assert(NM == 16, "row broadcasts need 16-lane groups");
    const double rik = r[K];
    const double piv = dppd<kDppRowBcast0 + K>(rik);
    double pr[NM];
#pragma unroll
    for (int q = 0; q < NM; ++q) pr[q] = dppd<kDppRowBcast0 + K>(r[q]);
    const double pv = dppd<kDppRowBcast0 + K>(v);
    const double rp = recip_nr(piv);
    if (dot == K) {
#pragma unroll
        for (int q = 0; q < NM; ++q) r[q] = pr[q] * rp;
        v = pv * rp;
    } else {
        const double f = rik * rp;
#pragma unroll
        for (int q = 0; q < NM; ++q) r[q] -= f * pr[q];
        v -= f * pv;
    }
}

// The block is eight waves: wave 0 inverts C_dd (the diagram prologue, in
// every block, so that no prologue launch precedes this one) while waves 1-7
// take 7 * 64 / NM pixels through x_u, the QP and the candidate set, which
// need C_dd but not its inverse; a barrier then hands A to the pixel waves
// for the base-state gradient.  (Eight waves: two blocks fill a CU at four
// waves per SIMD; four-wave blocks measured the same, five-wave blocks left
// a fifth of the grid waiting for a second round.)
constexpr int kSetupThreads = kWave + kSetupPixThreads;
static_assert(kSetupThreads >= kMaxDot * kMaxDot, "C_dd staging: one entry per thread");

template <int NM, bool CLOSED>
__global__ __launch_bounds__(kSetupThreads, CLOSED ? 3 : 4) void k_setup(DiagRec *__restrict__ dr,
                                                         const double *__restrict__ V, int64_t P,
                                                         PixRec *__restrict__ pr,
                                                         int64_t *__restrict__ counters,
                                                         int32_t *__restrict__ bstats,
                                                         double *__restrict__ x_out,
                                                         int32_t *__restrict__ flags_out,
                                                         const VGrid vg)
{
    __shared__ double sCdd[kMaxDot * kMaxDot];  // C_dd (input)
    __shared__ double sA[kMaxDot * kMaxDot];    // A (symmetric), from wave 0
    __shared__ double sc[kMaxDot];              // C_dd 1
    __shared__ double red[8];                   // [4] 1^T C_dd 1, [5] sum|A| / 2
    __shared__ double sS[kMaxDot * kMaxDot];    // the elimination after the high pivots, from wave 0
    __shared__ double sG[kMaxGate * NM];        // C_gd transposed: sG[j * NM + i]
    __shared__ int cnt[4];
    // Staging in one round trip: every load below is issued before any of
    // them is used.  C_gd (transposed, only the gates the diagram has) by
    // the first threads, C_dd by wave 0 (four entries per lane, the layout of
    // the inverse: lane 16 b + j holds column j of rows 4 b .. 4 b + 3); the
    // pixel waves of 16-dot groups also fetch their voltages (lane j: V_j
    // and V_16+j).
    const int tid = threadIdx.x;
    const int n = dr->n, g = dr->g, nhat = dr->nhat;
    const double t_in = dr->t;
    const bool pixel_wave = tid >= kWave;
    const int tp = tid - kWave;  // thread index among the pixel waves
    const int dot = tp & (NM - 1);
    const int base = (tid & (kWave - 1)) & ~(NM - 1);
    // wave w of block b takes group-set w * gridDim.x + b: the groups of one
    // wave are adjacent pixels (similar active sets, so the union of their QP
    // pivots stays small) while the waves of one block come from across the
    // sweep, so the QP-heavy regions are shared out among the blocks
    const int64_t p = ((int64_t)(tp / kWave) * gridDim.x + blockIdx.x) * (kWave / NM) +
                      (tp & (kWave - 1)) / NM;
    const int64_t pc = p < P ? p : P - 1;  // groups past the end repeat the last pixel
    const bool is_dot = dot < n;
    // (C_gd transposed: entry e = j NM + i, the gates j < g only)
    constexpr int kGv = (kMaxGate * NM + kSetupThreads - 1) / kSetupThreads;
    double gv[kGv];
#pragma unroll
    for (int r = 0; r < kGv; ++r) {
        const int e = tid + r * kSetupThreads;
        gv[r] = (e < g * NM) ? dr->Cgd[(e % NM) * kMaxGate + e / NM] : 0.0;
    }
    double m4[4];
    if (!pixel_wave) {
        const int j = tid & 15, b = tid >> 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) m4[q] = dr->Cdd[(4 * b + q) * kMaxDot + j];
    }
    double v0 = 0.0, v1 = 0.0;
    if (NM == 16 && pixel_wave && !vg.on) {
        if (dot < g) v0 = V[pc * g + dot];
        if (16 + dot < g) v1 = V[pc * g + 16 + dot];
    }
#pragma unroll
    for (int r = 0; r < kGv; ++r) {
        const int e = tid + r * kSetupThreads;
        if (e < g * NM) sG[e] = gv[r];
    }
    if (tid < 4) cnt[tid] = 0;
    if (!pixel_wave) {
        // wave 0 holds all of C_dd (lane 16 b + j: column j of rows
        // 4 b .. 4 b + 3): the input into LDS for the pixel waves' QP, C_dd 1
        // by row sums within each DPP row, 1^T C_dd 1 over the four rows of
        // DPP rows, then identity rows and columns past n for the inverse
        const int j = tid & 15, b = tid >> 4;
        double ct = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = 4 * b + q;
            sCdd[i * kMaxDot + j] = m4[q];
            const double ri = row_sum((i < n && j < n) ? m4[q] : 0.0);
            if (j == 0) sc[i] = ri;
            ct += ri;
            m4[q] = (i < n && j < n) ? m4[q] : (i == j ? 1.0 : 0.0);
        }
        ct += __shfl_xor(ct, 16, 64);
        ct += __shfl_xor(ct, 32, 64);
        if (tid == 0) red[4] = ct;
    }
    __syncthreads();
    const double one_c = red[4];

    double xu = 0.0, x = 0.0;
    int n0 = 0, k = -1, flags = 0, cflags = 0;
    uint32_t fm = 0;
    uint32_t gm = 0;  // rounding of x* inside the candidate set
    if (!pixel_wave) {
        // the inverse is the block's critical path: its wave issues first
        __builtin_amdgcn_s_setprio(3);
        prep_inverse_wave(m4, n, sA, red, sS);
        // a grid of at least 256 blocks: wave 0 of block b fills energy-table
        // entry b while the pixel waves finish (off the kernel's tail)
        if (gridDim.x >= 256) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            prep_tables_spread(dr, sA, sS, (int)blockIdx.x, (int)gridDim.x, n);
        }
        __builtin_amdgcn_s_setprio(0);
    } else {
        // x_u = C_gd V (V read, or formed from the sweep)
        if (vg.on) {
            double a, b;
            grid_ab(vg, pc, a, b);
            for (int j = 0; j < g; ++j) xu += sG[j * NM + dot] * grid_v(vg, j, a, b);
        } else if constexpr (NM == 16) {
            // V_j from lane j of the group (prefetched before the barrier)
            static_for_dev<0, kMaxGate>([&](auto jc) {
                constexpr int j = decltype(jc)::value;
                if (j < g) xu += sG[j * NM + dot] * dppd<kDppRowBcast0 + (j & 15)>(j < 16 ? v0 : v1);
            });
        } else {
            for (int j = 0; j < g; ++j) xu += sG[j * NM + dot] * V[pc * g + j];
        }
        if (!is_dot) xu = 0.0;
        // analytic minimum: open x = x_u; closed adds (N_hat - 1^T x_u) C_dd 1 / (1^T C_dd 1)
        double x0 = xu;
        if (CLOSED) {
            const double lam = ((double)nhat - group_dsum<NM>(xu)) / one_c;
            x0 = is_dot ? xu + lam * sc[dot] : 0.0;
        }
        x = x0;
        uint32_t W = group_ballot<NM>(is_dot && x0 < 0.0);
        if (CLOSED && nhat == 0) {
            // x = 0 is the only admissible point of a closed empty array
            flags = W ? 1 : 0;
            x = 0.0;
            W = 0;
        }
        if (W) {
            const double tol = 1e-13 * group_dmax<NM>(fmax(1.0, fabs(xu)));
            const double rone_c = CLOSED ? 1.0 / one_c : 0.0;
            double r[NM], v = x0;
            uint32_t done = 0;
            bool settled = false;
            for (int round = 0; round < 4 * NM + 4; ++round) {
                if (done == 0) {
                    // row `dot` of K (symmetric), identity beyond n, read
                    // afresh (the fence keeps the compiler from holding all
                    // of K in registers across the loop)
                    __asm__ volatile("" ::: "memory");
#pragma unroll
                    for (int q = 0; q < NM; ++q) {
                        double kv = (q == dot) ? 1.0 : 0.0;
                        if (q < n && is_dot) {
                            kv = sCdd[q * kMaxDot + dot];
                            if (CLOSED) kv -= (sc[q] * sc[dot]) * rone_c;
                        }
                        r[q] = kv;
                    }
                    v = x0;
                }
                if constexpr (NM == 16) {
                    // pivots in increasing dot order (as the shuffle form):
                    // dot k is pivoted by the groups that need it
                    const uint32_t todo = W & ~done;
                    static_for_dev<0, NM>([&](auto kc) {
                        constexpr int kp = decltype(kc)::value;
                        if (__ballot(todo >> kp & 1u) && (todo >> kp & 1u))
                            gj_pivot_row<NM, kp>(r, v, dot);
                    });
                } else {
                    for (uint32_t todo = W & ~done; todo; todo &= todo - 1)
                        gj_pivot<NM>(r, v, __ffs(todo) - 1, dot, base);
                }
                done = W;
                const bool in_w = W >> dot & 1u;
                x = in_w ? 0.0 : v;
                const bool keep = is_dot && (in_w ? (-v > -tol) : (v < -tol));
                const uint32_t Wn = group_ballot<NM>(keep);
                if (Wn == W) { settled = true; break; }
                if (W & ~Wn) done = 0;  // a dot leaves the active set: eliminate afresh
                W = Wn;
            }
            x = is_dot ? fmax(x, 0.0) : 0.0;
            flags = settled ? 1 : 3;
        }

        // candidate set (Sec. 3.2): base n0, free dots, closed: k raised free dots
        double t = t_in;
        bool freed = false;
        for (int iter = 0; iter < 80; ++iter) {
            // the box starts at floor(x* + 1e-9): a continuous minimum on an
            // integer keeps that integer as its floor whatever its last bit
            const double f = floor(x + 1e-9);
            const double fr = x - f;
            freed = is_dot && ((t >= 1.0) || (fabs(fr - 0.5) <= 0.5 * t));
            n0 = is_dot ? (int)f + ((!freed && fr > 0.5) ? 1 : 0) : 0;
            if (!CLOSED) break;
            const int sum0 = group_isum<NM>(n0);
            const int nfree = __popc(group_ballot<NM>(freed));
            const int need = nhat - sum0;
            if (need >= 0 && need <= nfree) { k = need; break; }
            if (t >= 1.0) {  // |sum x* - N_hat| < 1 makes this unreachable
                k = need < 0 ? 0 : nfree;
                cflags |= 2;
                break;
            }
            t = (t > 0.0) ? fmin(1.0, 2.0 * t) : 1.0;
            cflags |= 4;
        }
        fm = group_ballot<NM>(freed);
        if (!CLOSED) {
            gm = group_ballot<NM>(freed && x - (double)n0 >= 0.5);
        } else if (NM == 16) {
            // closed: the k free dots with the largest fractional parts (ties
            // to the lower index), an admissible state of the candidate set
            const double fr = freed ? x - (double)n0 : -1.0;
            int rank = 0;
            static_for_dev<0, NM>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                const double fq = group_bcast<NM, q>(fr, base);
                rank += ((fm >> q & 1u) && (fq > fr || (fq == fr && q < dot))) ? 1 : 0;
            });
            gm = group_ballot<NM>(freed && rank < k);
        }
    }
    __syncthreads();  // A from wave 0

    if (pixel_wave) {
        // g0 = A (n0 - x_u) and U(n0) = 1/2 (n0 - x_u)^T g0 (Eq. free_energy)
        const double z = is_dot ? (double)n0 - xu : 0.0;
        // column `dot` of A, all of it read before the first use (the loads
        // overlap instead of each waiting in turn)
        double acol[NM];
        static_for_dev<0, NM>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            acol[q] = sA[q * kMaxDot + dot];
        });
        const double aii = sA[dot * kMaxDot + dot];
        double g0 = 0.0;
        static_for_dev<0, NM>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            g0 += acol[q] * group_bcast<NM, q>(z, base);
        });
        const double u0 = 0.5 * group_dsum<NM>(z * g0);
        // energy of the guess state n0 + b (b = the bits gm) relative to
        // U(n0): b^T g0 + 1/2 b^T A b, with (A b)_dot the sum of the columns
        // of A that b raises
        double eg = 0.0;
        if (NM == 16 && n >= 13) {
            double ab = 0.0;
            static_for_dev<0, NM>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                ab += (gm >> q & 1u) ? acol[q] : 0.0;
            });
            eg = group_dsum<NM>((gm >> dot & 1u) ? g0 + 0.5 * ab : 0.0);
            if (!CLOSED) {
                // Open arrays: the rounding of x* takes the best single flip
                // of a free dot when it lowers the energy (flipping dot i of b
                // changes it by (1 - 2 b_i) (g0 + A b)_i + A_ii / 2).  The
                // guess stays a state of the candidate set; its lower energy
                // leaves fewer high parts for the scorer (on random sweeps
                // one flip reaches nearly all that a full descent does).
                const double gd = g0 + ab;
                const double de =
                    (fm >> dot & 1u) ? ((gm >> dot & 1u) ? -gd : gd) + 0.5 * aii : INFINITY;
                const double dmin = group_min<4>(de);
                const uint32_t at = group_ballot<NM>(de == dmin);
                if (dmin < 0.0 && at) {
                    gm ^= 1u << (__ffs(at) - 1);  // the lowest dot of the best flip
                    eg += dmin;
                }
            }
        }
        // terms of the lower bound of the bound-ordered scorer (N >= 13):
        // s = S z_hi and K = 1/2 z_hi^T s - U(n0) with S = (C_dd,HH)^{-1};
        // closed arrays also mu = -1^T A_LL^{-1} g0_lo
        double sv = 0.0, Kb = 0.0, mu = 0.0;
        if (NM == 16 && n >= 13) {
            const int hd = dot >= 8 ? dot : 8;
            double srow[8];
            static_for_dev<0, 8>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                srow[q] = sS[hd * kMaxDot + 8 + q];
            });
            static_for_dev<0, 8>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                sv += srow[q] * group_bcast<NM, (8 + q) & (NM - 1)>(z, base);
            });
            sv = dot >= 8 ? sv : 0.0;
            Kb = 0.5 * group_dsum<NM>(z * sv) - u0;
            if (CLOSED) {
                double qrow = 0.0;
                const int ld = dot < 8 ? dot : 0;
#pragma unroll
                for (int q = 0; q < 8; ++q) qrow += sS[ld * kMaxDot + q];
                mu = -group_dsum<NM>(dot < 8 ? qrow * g0 : 0.0);
            }
        }

        if (p < P) {
            PixRec *o = pr + p;
            for (int q = dot; q < kMaxDot; q += NM) {
                o->g0[q] = (q < NM) ? g0 : 0.0;
                o->n0[q] = (int16_t)((q < NM) ? n0 : 0);
            }
            if (dot >= 8) o->s[dot - 8] = (float)sv;
            if (dot == 0) {
                o->K = (float)Kb;
                o->mu = (float)mu;
                o->eg = (float)eg;
                o->u0 = u0;
                o->free = fm;
                o->k = k;
                o->flags = flags | cflags;
                o->guess = gm;
                if (flags_out) flags_out[p] = flags | (cflags & 4);
                if (cflags & 4) atomicAdd(&cnt[2], 1);
                if (flags & 1) atomicAdd(&cnt[1], 1);
                if (flags & 2) atomicAdd(&cnt[3], 1);
                atomicAdd(&cnt[0], 1);
            }
            if (x_out && is_dot) x_out[p * n + dot] = x;
        }
    }
    // per-block counts with plain stores (the host sums them): the counters
    // of this call are cleared by block 0 concurrently, so no atomics here
    __syncthreads();
    if (threadIdx.x < 4) bstats[blockIdx.x * 4 + threadIdx.x] = cnt[threadIdx.x];
    // the diagram's record for the next kernels: block 0 stores A and the
    // sums and clears the call's counters; the table entries are spread
    // over the waves of the grid (small grids) or were filled by wave 0
    // of the first 256 blocks
    if (blockIdx.x == 0) {
        prep_store_core(dr, sA, sc, red);
        if (counters)
            for (int i = threadIdx.x; i < kCounterWords; i += blockDim.x) counters[i] = 0;
    }
    if (gridDim.x < 256) prep_tables_spread(dr, sA, sS);
}

#define QA_DISPATCH_NM(n, CALL)                        \
    do {                                               \
        if ((n) <= 2) { constexpr int NM_ = 2; CALL; } \
        else if ((n) <= 4) { constexpr int NM_ = 4; CALL; } \
        else if ((n) <= 8) { constexpr int NM_ = 8; CALL; } \
        else { constexpr int NM_ = 16; CALL; }         \
    } while (0)

int64_t setup_blocks(int64_t P, int n_dot)
{
    int64_t b = 0;
    QA_DISPATCH_NM(n_dot, b = (P * NM_ + kSetupPixThreads - 1) / kSetupPixThreads);
    return b < 1 ? 1 : b;
}

hipError_t launch_setup(DiagRec *dr, const double *V, int64_t P, PixRec *pr, int64_t *counters,
                        int32_t *bstats, int n_dot, bool closed, hipStream_t s, double *x_out,
                        int32_t *flags_out, const VGrid *sweep)
{
    const dim3 grid((unsigned)setup_blocks(P, n_dot)), block(kSetupThreads);
    VGrid vg{};
    if (sweep) vg = *sweep;
    if (closed)
        QA_DISPATCH_NM(n_dot, hipLaunchKernelGGL((k_setup<NM_, true>), grid, block, 0, s, dr, V,
                                                 P, pr, counters, bstats, x_out, flags_out, vg));
    else
        QA_DISPATCH_NM(n_dot, hipLaunchKernelGGL((k_setup<NM_, false>), grid, block, 0, s, dr, V,
                                                 P, pr, counters, bstats, x_out, flags_out, vg));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K2 (FP64): T = 0 argmin and runner-up over the candidate set
// ---------------------------------------------------------------------------
template <int LG, int NM>
__global__ __launch_bounds__(256) void k_score_fp64(const DiagRec *__restrict__ dr,
                                                    const PixRec *__restrict__ pr, int64_t P,
                                                    int32_t *__restrict__ n_out,
                                                    int64_t *__restrict__ counters)
{
    constexpr int G = 1 << LG;
    __shared__ double sA[kMaxDot * kMaxDot];
    __shared__ unsigned long long sc[2];
    for (int i = threadIdx.x; i < kMaxDot * kMaxDot; i += blockDim.x) sA[i] = dr->A[i];
    if (threadIdx.x < 2) sc[threadIdx.x] = 0;
    __syncthreads();
    const int n = dr->n;
    const int lane = threadIdx.x & (G - 1);
    const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> LG;
    const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) >> LG;
    for (int64_t p = gid; p < P; p += ngroups) {
        const PixRec *r = pr + p;
        double g0[NM];
#pragma unroll
        for (int i = 0; i < NM; ++i) g0[i] = r->g0[i];
        const double u0 = r->u0;
        const uint32_t fm = r->free;
        const int k = r->k;
        const int m = __popc(fm);
        const uint64_t pos = free_positions(fm);
        const int chunk_log = m > LG ? m - LG : 0;
        const bool active = (m >= LG) || (lane < (1 << m));
        double e1 = INFINITY, e2 = INFINITY;
        uint32_t s1 = 0;
        int64_t scored = 0;
        if (active) {
            const uint32_t c0 = (uint32_t)lane << chunk_log;
            uint32_t s = pdep_mask(c0 ^ (c0 >> 1), fm);
            int pc = __popc(s);
            double y[NM];
            walk_start<NM>(sA, s, y);
            const int steps = 1 << chunk_log;
            for (int step = 0; step < steps; ++step) {
                if (step) walk_flip<NM>(sA, pos, step, s, pc, y);
                if (k < 0 || pc == k) {
                    const double e = walk_energy<NM>(g0, y, u0, s);
                    ++scored;
                    if (better(e, s, e1, s1)) { e2 = e1; e1 = e; s1 = s; }
                    else if (e < e2) e2 = e;
                }
            }
        }
        // group reduction of (e1, s1, e2)
#pragma unroll
        for (int off = G / 2; off >= 1; off >>= 1) {
            const double oe1 = __shfl_xor(e1, off, G);
            const double oe2 = __shfl_xor(e2, off, G);
            const uint32_t os1 = __shfl_xor(s1, off, G);
            if (better(oe1, os1, e1, s1)) { e2 = fmin(e1, oe2); e1 = oe1; s1 = os1; }
            else e2 = fmin(e2, oe1);
        }
        scored = (int64_t)group_sum<LG>((double)scored);
        if (lane == 0) {
            for (int i = 0; i < n; ++i) n_out[p * n + i] = (int32_t)r->n0[i] + (int32_t)(s1 >> i & 1u);
            if (e2 - e1 < 1e-9) atomicAdd(&sc[0], 1ull);
            atomicAdd(&sc[1], (unsigned long long)scored);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        block_add_counter(counters, C_GAP_1E9, (int64_t)sc[0]);
        block_add_counter(counters, C_CANDIDATES, (int64_t)sc[1]);
    }
}

#define QA_DISPATCH_GROUP(n, CALL)                                              \
    do {                                                                        \
        if ((n) == 1) { constexpr int LG_ = 1, NM_ = 2; CALL; }                 \
        else if ((n) == 2) { constexpr int LG_ = 2, NM_ = 2; CALL; }            \
        else if ((n) == 3) { constexpr int LG_ = 3, NM_ = 4; CALL; }            \
        else if ((n) == 4) { constexpr int LG_ = 4, NM_ = 4; CALL; }            \
        else if ((n) == 5) { constexpr int LG_ = 5, NM_ = 8; CALL; }            \
        else if ((n) <= 8) { constexpr int LG_ = 6, NM_ = 8; CALL; }            \
        else { constexpr int LG_ = 6, NM_ = 16; CALL; }                         \
    } while (0)

// table form (n <= 8): groups of up to 16 lanes, CPL candidates per lane
#define QA_DISPATCH_TAB(n, CALL)                                                 \
    do {                                                                         \
        if ((n) == 1) { constexpr int LG_ = 1, NM_ = 2, CPL_ = 1; CALL; }        \
        else if ((n) == 2) { constexpr int LG_ = 2, NM_ = 2, CPL_ = 1; CALL; }   \
        else if ((n) == 3) { constexpr int LG_ = 3, NM_ = 4, CPL_ = 1; CALL; }   \
        else if ((n) == 4) { constexpr int LG_ = 4, NM_ = 4, CPL_ = 1; CALL; }   \
        else if ((n) == 5) { constexpr int LG_ = 4, NM_ = 8, CPL_ = 2; CALL; }   \
        else if ((n) == 6) { constexpr int LG_ = 4, NM_ = 8, CPL_ = 4; CALL; }   \
        else if ((n) == 7) { constexpr int LG_ = 4, NM_ = 8, CPL_ = 8; CALL; }   \
        else { constexpr int LG_ = 4, NM_ = 8, CPL_ = 16; CALL; }                \
    } while (0)

static unsigned group_blocks(int64_t items, int lg, int64_t cap)
{
    const int64_t per_block = 256 >> lg;
    int64_t b = (items + per_block - 1) / per_block;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_score_fp64(const DiagRec *dr, const PixRec *pr, int64_t P, int32_t *n_out,
                             int64_t *counters, int n_dot, hipStream_t s)
{
    QA_DISPATCH_GROUP(n_dot, hipLaunchKernelGGL((k_score_fp64<LG_, NM_>),
                                                dim3(group_blocks(P, LG_, 8192)), dim3(256), 0, s,
                                                dr, pr, P, n_out, counters));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// softargmin (Sec. 4.2): pass 1 finds the smallest energy, pass 2 sums the
// Boltzmann weights exp(-(E - E_min)/kT) and the weighted offsets.
// ---------------------------------------------------------------------------
template <int LG, int NM>
__device__ __forceinline__ void soft_sums(const double *__restrict__ sA, const double (&g0)[NM],
                                          double u0, uint32_t fm, int k, int lane, double kT,
                                          double &emin, double &Z, double (&sv)[NM])
{
    const int m = __popc(fm);
    const uint64_t pos = free_positions(fm);
    const int chunk_log = m > LG ? m - LG : 0;
    const bool active = (m >= LG) || (lane < (1 << m));
    const uint32_t c0 = (uint32_t)lane << chunk_log;
    const int steps = 1 << chunk_log;
    double y[NM];
    double lmin = INFINITY;
    if (active) {
        uint32_t s = pdep_mask(c0 ^ (c0 >> 1), fm);
        int pc = __popc(s);
        walk_start<NM>(sA, s, y);
        for (int step = 0; step < steps; ++step) {
            if (step) walk_flip<NM>(sA, pos, step, s, pc, y);
            if (k < 0 || pc == k) lmin = fmin(lmin, walk_energy<NM>(g0, y, u0, s));
        }
    }
    emin = group_min<LG>(lmin);
    double z = 0.0;
#pragma unroll
    for (int i = 0; i < NM; ++i) sv[i] = 0.0;
    if (active) {
        uint32_t s = pdep_mask(c0 ^ (c0 >> 1), fm);
        int pc = __popc(s);
        walk_start<NM>(sA, s, y);
        for (int step = 0; step < steps; ++step) {
            if (step) walk_flip<NM>(sA, pos, step, s, pc, y);
            if (k < 0 || pc == k) {
                const double w = exp(-(walk_energy<NM>(g0, y, u0, s) - emin) / kT);
                z += w;
#pragma unroll
                for (int i = 0; i < NM; ++i)
                    if (s >> i & 1u) sv[i] += w;
            }
        }
    }
    Z = group_sum<LG>(z);
#pragma unroll
    for (int i = 0; i < NM; ++i) sv[i] = group_sum<LG>(sv[i]);
}

template <int LG, int NM>
__global__ __launch_bounds__(256) void k_soft_fwd(const DiagRec *__restrict__ dr,
                                                  const PixRec *__restrict__ pr, int64_t P,
                                                  double *__restrict__ nbar,
                                                  SavedRec *__restrict__ saved,
                                                  int64_t *__restrict__ counters)
{
    constexpr int G = 1 << LG;
    __shared__ double sA[kMaxDot * kMaxDot];
    for (int i = threadIdx.x; i < kMaxDot * kMaxDot; i += blockDim.x) sA[i] = dr->A[i];
    __syncthreads();
    const int n = dr->n;
    const double kT = dr->kT;
    const int lane = threadIdx.x & (G - 1);
    const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> LG;
    const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) >> LG;
    for (int64_t p = gid; p < P; p += ngroups) {
        const PixRec *r = pr + p;
        // g0: lane l of the group reads entry l mod NM, then broadcasts
        // within the group (one read per lane instead of NM)
        const double gl = r->g0[lane & (NM - 1)];
        double g0[NM], sv[NM];
        static_for_dev<0, NM>([&](auto ic) { g0[decltype(ic)::value] = lane_bcast<LG, decltype(ic)::value>(gl); });
        double emin, Z;
        soft_sums<LG, NM>(sA, g0, r->u0, r->free, r->k, lane, kT, emin, Z, sv);
        if (lane == 0) {
            for (int i = 0; i < n; ++i) {
                double v = 0.0;
#pragma unroll
                for (int j = 0; j < NM; ++j)
                    if (j == i) v = sv[j];
                nbar[p * n + i] = (double)r->n0[i] + v / Z;
            }
            if (saved) {
                SavedRec *o = saved + p;
                o->emin = emin;
                o->Z = Z;
#pragma unroll
                for (int i = 0; i < NM; ++i) o->nb[i] = sv[i] / Z;
                for (int i = NM; i < kMaxDot; ++i) o->nb[i] = 0.0;
                for (int i = 0; i < kMaxDot; ++i) o->n0[i] = r->n0[i];
                o->free = r->free;
                o->k = r->k;
            }
        }
    }
}

// Candidates of a pixel with n <= 8 dots in the table form: lane `lane` of
// a group of G takes compressed indices c = lane + G q, q < CPL, and
//   U(n0 + 1_s) = U(n0) + g0 . 1_s + h(s),  h(s) = 1/2 s^T A s,
// with h from the prologue's whole-box table (LDS).  Inadmissible slots
// (past the set, or the wrong closed popcount) get +inf.
template <int NM>
__device__ __forceinline__ double tab_energy(const double *__restrict__ sH, const double (&g0)[NM],
                                             double u0, uint32_t fm, int k, uint32_t c,
                                             uint32_t &sq)
{
    const uint32_t count = 1u << __popc(fm);
    const bool full = (fm & (fm + 1)) == 0;  // every dot free: s = c
    sq = full ? c : pdep_mask(c, fm);
    double E = INFINITY;
    if (c < count && (k < 0 || __popc(sq) == k)) {
        double L = u0;
#pragma unroll
        for (int i = 0; i < NM; ++i)
            if (sq >> i & 1u) L += g0[i];
        E = L + sH[sq];
    }
    return E;
}

// The same energies when every free dot is one of the low dots (fm = 2^m - 1,
// the usual case): candidate q of a lane is s = lane + q 2^LG, so the bits
// below LG come from the lane (summed once per pixel) and the rest from q,
// known at compile time once the loop is unrolled.
template <int LG, int NM, int CPL>
__device__ __forceinline__ void tab_energies_low(const double *__restrict__ sH,
                                                 const double (&g0)[NM], double u0,
                                                 uint32_t count, int k, int lane,
                                                 double (&e)[CPL])
{
    double lo = u0;
#pragma unroll
    for (int i = 0; i < LG; ++i)
        if (lane >> i & 1) lo += g0[i];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const uint32_t s = (uint32_t)lane + ((uint32_t)q << LG);
        double L = lo;
#pragma unroll
        for (int j = LG; j < NM; ++j)
            if ((q << LG) >> j & 1) L += g0[j];
        e[q] = (s < count && (k < 0 || __popc(s) == k)) ? L + sH[s] : INFINITY;
    }
}

template <int LG, int NM, int CPL>
__device__ __forceinline__ void tab_energies(const double *__restrict__ sH, const double (&g0)[NM],
                                             double u0, uint32_t fm, int k, int lane,
                                             double (&e)[CPL], uint32_t (&st)[CPL])
{
#pragma unroll
    for (int q = 0; q < CPL; ++q)
        e[q] = tab_energy<NM>(sH, g0, u0, fm, k, (uint32_t)(lane + (q << LG)), st[q]);
}

template <int LG, int NM, int CPL>
__global__ __launch_bounds__(256) void k_soft_fwd_tab(const DiagRec *__restrict__ dr,
                                                      const PixRec *__restrict__ pr, int64_t P,
                                                      double *__restrict__ nbar,
                                                      SavedRec *__restrict__ saved,
                                                      int64_t *__restrict__ counters)
{
    constexpr int G = 1 << LG;
    __shared__ double sH[256];
    // the scalars and the table entry of this thread (blocks of 256) read
    // together, one round trip before the pixel loop
    const int n = dr->n;
    const double kT = dr->kT;
    const double hs = dr->hs[threadIdx.x];
    sH[threadIdx.x] = hs;
    __syncthreads();
    const double ikT = 1.0 / kT;
    const int lane = threadIdx.x & (G - 1);
    const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> LG;
    const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) >> LG;
    for (int64_t p = gid; p < P; p += ngroups) {
        const PixRec *r = pr + p;
        // g0: lane l of the group reads entry l mod NM, then broadcasts
        // within the group (one read per lane instead of NM)
        const double gl = r->g0[lane & (NM - 1)];
        double g0[NM];
        static_for_dev<0, NM>([&](auto ic) { g0[decltype(ic)::value] = lane_bcast<LG, decltype(ic)::value>(gl); });
        double e[CPL];
        uint32_t st[CPL];
        const uint32_t fm = r->free;
        const bool low = (fm & (fm + 1)) == 0;
        if (low)
            tab_energies_low<LG, NM, CPL>(sH, g0, r->u0, 1u << __popc(fm), r->k, lane, e);
        else
            tab_energies<LG, NM, CPL>(sH, g0, r->u0, fm, r->k, lane, e, st);
        double lmin = e[0];
#pragma unroll
        for (int q = 1; q < CPL; ++q) lmin = fmin(lmin, e[q]);
        const double emin = group_min<LG>(lmin);
        double z = 0.0, sv[NM];
#pragma unroll
        for (int i = 0; i < NM; ++i) sv[i] = 0.0;
        if (low) {
            // dot i < LG is in every candidate of the lane or in none
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                if (e[q] < INFINITY) {
                    const double w = exp((emin - e[q]) * ikT);
                    z += w;
#pragma unroll
                    for (int j = LG; j < NM; ++j)
                        if ((q << LG) >> j & 1) sv[j] += w;
                }
            }
#pragma unroll
            for (int i = 0; i < LG; ++i) sv[i] = (lane >> i & 1) ? z : 0.0;
        } else {
#pragma unroll
            for (int q = 0; q < CPL; ++q) {
                if (e[q] < INFINITY) {
                    const double w = exp((emin - e[q]) * ikT);
                    z += w;
#pragma unroll
                    for (int i = 0; i < NM; ++i)
                        if (st[q] >> i & 1u) sv[i] += w;
                }
            }
        }
        const double Z = group_sum<LG>(z);
#pragma unroll
        for (int i = 0; i < NM; ++i) sv[i] = group_sum<LG>(sv[i]);
        // lane i < n writes dot i; lane 0 the rest of the saved record
        double svl = 0.0;
#pragma unroll
        for (int i = 0; i < NM; ++i)
            if (i == lane) svl = sv[i];
        if (lane < n) nbar[p * n + lane] = (double)r->n0[lane] + svl / Z;
        if (saved) {
            SavedRec *o = saved + p;
            if (lane < kMaxDot) {
                o->nb[lane] = (lane < n) ? svl / Z : 0.0;
                o->n0[lane] = r->n0[lane];
            }
            if (lane == 0) {
                o->emin = emin;
                o->Z = Z;
                o->free = r->free;
                o->k = r->k;
            }
        }
    }
}

// T = 0 argmin over the candidate set in the table form (n <= 8): the
// candidate energies U(n0 + s) = U(n0) + g0 . s + h(s), h(s) = 1/2 s^T A s from
// the whole-box table, CPL candidates per lane, groups of 2^LG lanes per
// pixel; the same minimum, tie-break and runner-up as k_score_fp64.
template <int LG, int NM, int CPL>
__global__ __launch_bounds__(256) void k_score_tab(const DiagRec *__restrict__ dr,
                                                   const PixRec *__restrict__ pr, int64_t P,
                                                   int32_t *__restrict__ n_out,
                                                   int64_t *__restrict__ counters)
{
    constexpr int G = 1 << LG;
    __shared__ double sH[256];
    __shared__ unsigned long long sc[2];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) sH[i] = dr->hs[i];
    if (threadIdx.x < 2) sc[threadIdx.x] = 0;
    __syncthreads();
    const int n = dr->n;
    const int lane = threadIdx.x & (G - 1);
    const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> LG;
    const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) >> LG;
    for (int64_t p = gid; p < P; p += ngroups) {
        const PixRec *r = pr + p;
        // g0: lane l of the group reads entry l mod NM, then broadcasts
        // within the group (one read per lane instead of NM)
        const double gl = r->g0[lane & (NM - 1)];
        double g0[NM];
        static_for_dev<0, NM>([&](auto ic) { g0[decltype(ic)::value] = lane_bcast<LG, decltype(ic)::value>(gl); });
        double e[CPL];
        uint32_t st[CPL];
        tab_energies<LG, NM, CPL>(sH, g0, r->u0, r->free, r->k, lane, e, st);
        double e1 = INFINITY, e2 = INFINITY;
        uint32_t s1 = 0;
        int scored = 0;
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            if (e[q] < INFINITY) ++scored;
            if (better(e[q], st[q], e1, s1)) { e2 = e1; e1 = e[q]; s1 = st[q]; }
            else if (e[q] < e2) e2 = e[q];
        }
#pragma unroll
        for (int off = G / 2; off >= 1; off >>= 1) {
            const double oe1 = __shfl_xor(e1, off, G);
            const double oe2 = __shfl_xor(e2, off, G);
            const uint32_t os1 = __shfl_xor(s1, off, G);
            if (better(oe1, os1, e1, s1)) { e2 = fmin(e1, oe2); e1 = oe1; s1 = os1; }
            else e2 = fmin(e2, oe1);
        }
        const int total = (int)group_sum<LG>((double)scored);
        if (lane < n) n_out[p * n + lane] = (int32_t)r->n0[lane] + (int32_t)(s1 >> lane & 1u);
        if (lane == 0) {
            if (e2 - e1 < 1e-9) atomicAdd(&sc[0], 1ull);
            atomicAdd(&sc[1], (unsigned long long)total);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        block_add_counter(counters, C_GAP_1E9, (int64_t)sc[0]);
        block_add_counter(counters, C_CANDIDATES, (int64_t)sc[1]);
    }
}

hipError_t launch_score_tab(const DiagRec *dr, const PixRec *pr, int64_t P, int32_t *n_out,
                            int64_t *counters, int n_dot, hipStream_t s)
{
    if (n_dot < 1 || n_dot > 8) return hipErrorInvalidValue;
    QA_DISPATCH_TAB(n_dot, hipLaunchKernelGGL((k_score_tab<LG_, NM_, CPL_>),
                                              dim3(group_blocks(P, LG_, 8192)), dim3(256), 0, s,
                                              dr, pr, P, n_out, counters));
    return hipGetLastError();
}

hipError_t launch_soft_fwd(const DiagRec *dr, const PixRec *pr, int64_t P, double *nbar,
                           SavedRec *saved, int64_t *counters, int n_dot, hipStream_t s)
{
    if (n_dot <= 8) {
        QA_DISPATCH_TAB(n_dot, hipLaunchKernelGGL((k_soft_fwd_tab<LG_, NM_, CPL_>),
                                                  dim3(group_blocks(P, LG_, 8192)), dim3(256), 0,
                                                  s, dr, pr, P, nbar, saved, counters));
    } else {
        hipLaunchKernelGGL((k_soft_fwd<6, 16>), dim3(group_blocks(P, 6, 8192)), dim3(256), 0, s,
                           dr, pr, P, nbar, saved, counters);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// adjoint of the softargmin.  With pi_s the normalised weight of candidate
// n0 + 1_s, nb = sum_s pi_s 1_s and Gbar = dL/d<n>:
//   dL/dE_s = ubar_s = -(pi_s / kT) (Gbar . 1_s - Gbar . nb)
//   m_p     = sum_s ubar_s 1_s,  z_p = n0 - x_u,  (sum_s ubar_s = 0)
//   dL/dA   = 1/2 sum_p (z_p m_p^T + m_p z_p^T) + 1/2 sum_s u_s 1_s 1_s^T,
//             u_s = sum_p ubar_ps
//   dL/dx_u,p = -A m_p,  dL/dC_gd = sum_p (dL/dx_u,p) V_p^T,
//   dL/dV_p = C_gd^T dL/dx_u,p,  dL/dC_dd = -A (dL/dA) A.
// ---------------------------------------------------------------------------
constexpr int kBwdMaxDot = 12;

// One pass over the candidates per pixel: the forward pass saved E_min, Z
// and nb, so the weights pi_s = exp(-(E_s - E_min)/kT) / Z follow from the
// recomputed energies (table form for n <= 8, CPL > 0; the Gray-code walk
// otherwise).  The per-pixel outer products go to block sums in LDS, spread
// over the lanes (lane i: row i of the dL/dA sum; lane j: gate column j of
// the dL/dC_gd sum); the u_s terms fold into the dL/dA block sum as superset
// sums, and the block sums reach HBM once per block, as atomic adds into one
// of kBwdReplicas copies.
// The table form is held to 168 VGPRs (three waves per SIMD, so that a
// 10^4-pixel launch is resident at once); the walk form would spill there.
template <int LG, int NM, int CPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CPL > 0 ? 3 : 1))) void k_soft_bwd(const DiagRec *__restrict__ dr,
                                                  const double *__restrict__ V, int64_t P,
                                                  const double *__restrict__ gbar,
                                                  const SavedRec *__restrict__ saved,
                                                  double *__restrict__ acc,
                                                  double *__restrict__ gradV,
                                                  const VGrid vg)
{
    constexpr int G = 1 << LG;
    constexpr int NU = 1 << (NM < kBwdMaxDot ? NM : kBwdMaxDot);
    __shared__ double sA[kMaxDot * kMaxDot];
    __shared__ double sCgd[kMaxDot * kMaxGate];
    __shared__ double sU[NU];
    __shared__ double sdA[kMaxDot * kMaxDot];
    __shared__ double sdG[kMaxDot * kMaxGate];
    __shared__ double sH[CPL > 0 ? 256 : 1];  // whole-box table h(s) (table form)
    static_assert(kMaxDot * kMaxDot == 256 && kMaxDot * kMaxGate == 512, "staging layout");
    // every staging read issued before the first LDS write (blocks of 256
    // threads: one A / table entry and two C_gd entries each), with the
    // scalars, so the staging is one round trip
    const int n = dr->n, g = dr->g;
    const double kT = dr->kT;
    {
        const int t = threadIdx.x;
        const double a = dr->A[t];
        const double h = CPL > 0 ? dr->hs[t] : 0.0;
        const double c0 = dr->Cgd[t], c1 = dr->Cgd[t + 256];
        sA[t] = a;
        sdA[t] = 0.0;
        if (CPL > 0) sH[t] = h;
        sCgd[t] = c0;
        sCgd[t + 256] = c1;
        sdG[t] = 0.0;
        sdG[t + 256] = 0.0;
    }
    for (int i = threadIdx.x; i < NU; i += blockDim.x) sU[i] = 0.0;
    __syncthreads();
    const double ikT = 1.0 / kT;
    const int lane = threadIdx.x & (G - 1);
    const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> LG;
    const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) >> LG;
    for (int64_t p = gid; p < P; p += ngroups) {
        // keep the reads of A in LDS inside the loop: hoisted, they would
        // hold N^2 doubles in registers for the whole kernel
        asm volatile("" ::: "memory");
        const SavedRec *sr = saved + p;
        // dot-wise quantities: lane d = lane mod NM computes dot d, then the
        // group gathers the vectors (G >= NM)
        const int d = lane & (NM - 1);
        // the pixel's sweep coordinates (sweep input)
        double va = 0.0, vb = 0.0;
        if (vg.on) grid_ab(vg, p, va, vb);
        auto volt = [&](int j) { return vg.on ? grid_v(vg, j, va, vb) : V[p * g + j]; };
        double zd = 0.0;
        if (d < n) {
            double s = 0.0;
            for (int j = 0; j < g; ++j) s += sCgd[d * kMaxGate + j] * volt(j);
            zd = (double)sr->n0[d] - s;
        }
        double z[NM], g0[NM], gb[NM];
        static_for_dev<0, NM>([&](auto I) { z[I] = lane_bcast<LG, I>(zd); });
        // dL/d<n> and <n> - n0 of the pixel: lane d reads entry d, then
        // broadcasts within the group (one read each per lane instead of NM)
        const double gbd = d < n ? gbar[p * n + d] : 0.0;
        const double gnd = gbd * sr->nb[d];
        double gnb = 0.0;
        static_for_dev<0, NM>([&](auto I) {
            gb[I] = lane_bcast<LG, I>(gbd);
            gnb += lane_bcast<LG, I>(gnd);
        });
        // g0 = A z, U(n0) = 1/2 z^T g0
        double gd = 0.0;
#pragma unroll
        for (int j = 0; j < NM; ++j) gd += sA[d * kMaxDot + j] * z[j];
        double u0 = 0.0;
        static_for_dev<0, NM>([&](auto I) { g0[I] = lane_bcast<LG, I>(gd); });
#pragma unroll
        for (int i = 0; i < NM; ++i) u0 += z[i] * g0[i];
        u0 *= 0.5;
        const uint32_t fm = sr->free;
        const int k = sr->k;
        const double emin = sr->emin, Z = sr->Z;
        // ubar_s, m_p and u_s
        double mv[NM];
#pragma unroll
        for (int i = 0; i < NM; ++i) mv[i] = 0.0;
        const double iZ = 1.0 / Z;
        auto add_candidate = [&](uint32_t s, double E) {
            const double pi = exp((emin - E) * ikT) * iZ;
            double gs = 0.0;
#pragma unroll
            for (int i = 0; i < NM; ++i)
                if (s >> i & 1u) gs += gb[i];
            const double ub = -(pi * ikT) * (gs - gnb);
#pragma unroll
            for (int i = 0; i < NM; ++i)
                if (s >> i & 1u) mv[i] += ub;
            atomicAdd(&sU[s], ub);
        };
        if constexpr (CPL > 0) {
            if ((fm & (fm + 1)) == 0) {
                // free dots 0..m-1: the same split of s = lane + q 2^LG as
                // the forward, so dots below LG take the lane's total
                double e[CPL];
                tab_energies_low<LG, NM, CPL>(sH, g0, u0, 1u << __popc(fm), k, lane, e);
                double glo = -gnb;
#pragma unroll
                for (int i = 0; i < LG; ++i)
                    if (lane >> i & 1) glo += gb[i];
                double tsum = 0.0;
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    if (e[q] < INFINITY) {
                        double gs = glo;
#pragma unroll
                        for (int j = LG; j < NM; ++j)
                            if ((q << LG) >> j & 1) gs += gb[j];
                        const double ub = -(exp((emin - e[q]) * ikT) * iZ * ikT) * gs;
                        tsum += ub;
#pragma unroll
                        for (int j = LG; j < NM; ++j)
                            if ((q << LG) >> j & 1) mv[j] += ub;
                        atomicAdd(&sU[lane + (q << LG)], ub);
                    }
                }
#pragma unroll
                for (int i = 0; i < LG; ++i)
                    if (lane >> i & 1) mv[i] += tsum;
            } else {
#pragma unroll 2
                for (int q = 0; q < CPL; ++q) {
                    uint32_t sq;
                    const double E =
                        tab_energy<NM>(sH, g0, u0, fm, k, (uint32_t)(lane + (q << LG)), sq);
                    if (E < INFINITY) add_candidate(sq, E);
                }
            }
        }
        const int m = __popc(fm);
        const uint64_t pos = free_positions(fm);
        const int chunk_log = m > LG ? m - LG : 0;
        const bool active = CPL == 0 && ((m >= LG) || (lane < (1 << m)));
        const uint32_t c0 = (uint32_t)lane << chunk_log;
        const int steps = 1 << chunk_log;
        double y[NM];
        if (active) {
            uint32_t s = pdep_mask(c0 ^ (c0 >> 1), fm);
            int pc = __popc(s);
            walk_start<NM>(sA, s, y);
            for (int step = 0; step < steps; ++step) {
                if (step) walk_flip<NM>(sA, pos, step, s, pc, y);
                if (k < 0 || pc == k) add_candidate(s, walk_energy<NM>(g0, y, u0, s));
            }
        }
#pragma unroll
        for (int i = 0; i < NM; ++i) mv[i] = group_sum<LG>(mv[i]);
        // dL/dx_u = -A m
        double dd = 0.0;
#pragma unroll
        for (int j = 0; j < NM; ++j) dd -= sA[d * kMaxDot + j] * mv[j];
        double dx[NM];
        static_for_dev<0, NM>([&](auto I) { dx[I] = lane_bcast<LG, I>(dd); });
        // lane i < n: row i of 1/2 (z m^T + m z^T)
        double zi = 0.0, mi = 0.0;
#pragma unroll
        for (int i = 0; i < NM; ++i)
            if (i == lane) { zi = z[i]; mi = mv[i]; }
        if (lane < n) {
#pragma unroll
            for (int j = 0; j < NM; ++j)
                if (j < n) atomicAdd(&sdA[lane * kMaxDot + j], 0.5 * (zi * mv[j] + mi * z[j]));
        }
        // gate column j: dL/dC_gd += dx V_j, dL/dV_j = sum_i C_gd,ij dx_i
        for (int j = lane; j < g; j += G) {
            const double vj = volt(j);
            double gv = 0.0;
#pragma unroll
            for (int i = 0; i < NM; ++i) {
                if (i < n) atomicAdd(&sdG[i * kMaxGate + j], dx[i] * vj);
                gv += sCgd[i * kMaxGate + j] * dx[i];
            }
            if (gradV) gradV[p * g + j] = gv;
        }
    }
    __syncthreads();
    // dL/dA_ij also takes 1/2 sum_s u_s [i in s][j in s] = 1/2 F({i, j}), F the
    // superset sums of the block's u_s (one dot per pass, in place: a pass
    // writes only entries without its dot and reads only entries with it)
    const int nu = 1 << n;
    for (int b = 0; b < n; ++b) {
        for (int s = threadIdx.x; s < nu; s += blockDim.x)
            if (!(s >> b & 1)) sU[s] += sU[s | (1 << b)];
        __syncthreads();
    }
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        sdA[i * kMaxDot + j] += 0.5 * sU[(1 << i) | (1 << j)];
    }
    __syncthreads();
    double *accA = acc + (blockIdx.x & (kBwdReplicas - 1)) * kBwdAccWords;
    double *accG = accA + kMaxDot * kMaxDot;
    for (int i = threadIdx.x; i < kMaxDot * kMaxDot; i += blockDim.x)
        if (sdA[i] != 0.0) atomicAdd(&accA[i], sdA[i]);
    for (int i = threadIdx.x; i < kMaxDot * kMaxGate; i += blockDim.x)
        if (sdG[i] != 0.0) atomicAdd(&accG[i], sdG[i]);
}

__global__ __launch_bounds__(256) void k_soft_bwd_final(const DiagRec *__restrict__ dr,
                                                        double *__restrict__ acc,
                                                        double *__restrict__ grad_cdd,
                                                        double *__restrict__ grad_cgd)
{
    __shared__ double sA[kMaxDot * kMaxDot];
    __shared__ double dA[kMaxDot * kMaxDot];
    __shared__ double T[kMaxDot * kMaxDot];
    __shared__ double dG[kMaxDot * kMaxGate];
    const int n = dr->n, g = dr->g;
    const int tid = threadIdx.x;
    auto total = [&](int e) {  // the copies' sum of accumulator word e
        double v = 0.0;
#pragma unroll
        for (int r = 0; r < kBwdReplicas; ++r) v += acc[r * kBwdAccWords + e];
        return v;
    };
    // every global read up front, in one round trip
    for (int e = tid; e < kMaxDot * kMaxDot; e += blockDim.x) {
        sA[e] = dr->A[e];
        dA[e] = total(e);
    }
    for (int e = tid; e < n * g; e += blockDim.x) {
        const int i = e / g, j = e % g;
        dG[e] = total(kMaxDot * kMaxDot + i * kMaxGate + j);
    }
    __syncthreads();
    // leave the accumulators zero for the next backward pass
    for (int e = tid; e < kBwdReplicas * kBwdAccWords; e += blockDim.x) acc[e] = 0.0;
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        double v = 0.0;
        for (int a = 0; a < n; ++a) v += dA[i * kMaxDot + a] * sA[a * kMaxDot + j];
        T[i * kMaxDot + j] = v;  // (dL/dA) A
    }
    for (int e = tid; e < n * g; e += blockDim.x) grad_cgd[e] = dG[e];
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        double v = 0.0;
        for (int a = 0; a < n; ++a) v += sA[i * kMaxDot + a] * T[a * kMaxDot + j];
        grad_cdd[e] = -v;
    }
}

hipError_t launch_soft_bwd(const DiagRec *dr, const double *V, int64_t P, const double *gbar,
                           const SavedRec *saved, double *acc, double *gradV, int n_dot,
                           hipStream_t s, const VGrid *sweep)
{
    VGrid vg{};
    if (sweep) vg = *sweep;
    // acc: zeroed by the caller's prologue launch or left zero by the last
    // final kernel
    if (n_dot <= 8) {
        QA_DISPATCH_TAB(n_dot, hipLaunchKernelGGL((k_soft_bwd<LG_, NM_, CPL_>),
                                                  dim3(group_blocks(P, LG_, 2048)), dim3(256), 0,
                                                  s, dr, V, P, gbar, saved, acc, gradV, vg));
    } else {
        hipLaunchKernelGGL((k_soft_bwd<6, 16, 0>), dim3(group_blocks(P, 6, 2048)), dim3(256), 0,
                           s, dr, V, P, gbar, saved, acc, gradV, vg);
    }
    return hipGetLastError();
}

hipError_t launch_soft_bwd_final(const DiagRec *dr, double *acc, double *grad_cdd,
                                 double *grad_cgd, hipStream_t s)
{
    hipLaunchKernelGGL(k_soft_bwd_final, dim3(1), dim3(256), 0, s, dr, acc, grad_cdd, grad_cgd);
    return hipGetLastError();
}

}  // namespace qa
