// qa_device.h -- device helpers shared by the kernels of libqarray:
// candidate sets (Sec. 3.2), the exact QP of Sec. 3.1.2, and the Gray-code
// walk over a candidate set with FP64 energies (Eq. free_energy).
#pragma once
#include "qa_internal.h"

#include <math.h>
#include <type_traits>

namespace qa {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pdep_mask(uint32_t c, uint32_t mask)
{
    // scatter the low bits of c onto the set bits of mask, in order
    uint32_t s = 0;
    for (int j = 0; mask; ++j) {
        const uint32_t low = mask & (0u - mask);
        if (c >> j & 1u) s |= low;
        mask ^= low;
    }
    return s;
}

__device__ __forceinline__ bool better(double e, uint32_t s, double e1, uint32_t s1)
{
    // smaller energy; equal energies resolve to the lexicographically
    // smallest charge vector (dot 0 most significant)
    return e < e1 || (e == e1 && __brev(s) < __brev(s1));
}


// Candidate set of Sec. 3.2 for the continuous minimum x: base state n0,
// mask of dots that take both roundings and, for closed arrays, the number k
// of those dots raised by one (k = -1 for open arrays).  Returns the flags
// (bit1: no admissible state even at t = 1, bit2: the threshold doubled).
template <int NM>
__device__ __forceinline__ int candidate_set(const DiagRec *__restrict__ dr, bool closed,
                                             const double (&x)[NM], int (&n0)[NM],
                                             uint32_t &fm, int &k)
{
    const int n = dr->n;
    double t = dr->t;
    int flags = 0;
    k = -1;
    for (int iter = 0; iter < 80; ++iter) {
        fm = 0;
        int sum0 = 0;
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            n0[i] = 0;
            if (i < n) {
                // the box starts at floor(x* + 1e-9): a continuous minimum on
                // an integer (an active bound, a whole free charge) keeps that
                // integer as its floor whatever its last rounded bit
                const double f = floor(x[i] + 1e-9);
                const double fr = x[i] - f;
                const bool freed = (t >= 1.0) || (fabs(fr - 0.5) <= 0.5 * t);
                n0[i] = (int)f + ((!freed && fr > 0.5) ? 1 : 0);
                if (freed) fm |= 1u << i;
                sum0 += n0[i];
            }
        }
        if (!closed) break;
        const int need = dr->nhat - sum0;
        if (need >= 0 && need <= __popc(fm)) { k = need; break; }
        if (t >= 1.0) {  // |sum x* - N_hat| < 1 makes this unreachable
            k = need < 0 ? 0 : __popc(fm);
            flags |= 2;
            break;
        }
        t = (t > 0.0) ? fmin(1.0, 2.0 * t) : 1.0;
        flags |= 4;
    }
    return flags;
}

// g0 = A (n0 - x_u) and U(n0) = 1/2 (n0 - x_u)^T g0 (Eq. free_energy)
template <int NM>
__device__ __forceinline__ double base_state(const double *__restrict__ A, int n,
                                             const int (&n0)[NM], const double (&xu)[NM],
                                             double (&g0)[NM])
{
    double z[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) z[i] = (i < n) ? (double)n0[i] - xu[i] : 0.0;
    double u0 = 0.0;
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NM; ++j) s += A[i * kMaxDot + j] * z[j];
        g0[i] = s;
        u0 += z[i] * s;
    }
    return 0.5 * u0;
}

// 1/sqrt(a) for the Cholesky pivots: the hardware estimate refined by two
// Newton steps r <- r (3/2 - a r^2 / 2) (each squares the relative error),
// within an ulp for the positive normal pivots of a definite system.
__device__ __forceinline__ double rsqrt_nr(double a)
{
    double r = __builtin_amdgcn_rsq(a);
    const double h = 0.5 * a;
    r = r * fma(-h * r, r, 1.5);
    return r * fma(-h * r, r, 1.5);
}

// Cholesky solve of an SPD system held as a packed lower triangle, M fixed.
// The factor's diagonal is kept as its reciprocal, so the factorisation and
// both substitutions multiply where they would divide (no square root, no
// division).  On return a holds L below the diagonal and 1 / L_jj on it.
template <int M>
__device__ __forceinline__ void chol_solve(double (&a)[M * (M + 1) / 2], double (&b)[M])
{
#define LIDX(i, j) ((i) * ((i) + 1) / 2 + (j))
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double d = a[LIDX(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= a[LIDX(j, k)] * a[LIDX(j, k)];
        const double inv = rsqrt_nr(d);
        a[LIDX(j, j)] = inv;
#pragma unroll
        for (int i = j + 1; i < M; ++i) {
            double s = a[LIDX(i, j)];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= a[LIDX(i, k)] * a[LIDX(j, k)];
            a[LIDX(i, j)] = s * inv;
        }
    }
#pragma unroll
    for (int i = 0; i < M; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= a[LIDX(i, k)] * b[k];
        b[i] = s * a[LIDX(i, i)];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        double s = b[i];
#pragma unroll
        for (int k = i + 1; k < M; ++k) s -= a[LIDX(k, i)] * b[k];
        b[i] = s * a[LIDX(i, i)];
    }
#undef LIDX
}

// The QP of Sec. 3.1.2, min U(x) s.t. x >= 0 [and 1^T x = N_hat], in its KKT
// form x = x_u + C_dd mu + lambda C_dd 1, mu >= 0, x >= 0, mu_i x_i = 0.
// For an active set W (x_W = 0, mu zero off W) the unknowns (mu_W, lambda)
// solve  [C_WW  c_W; c_W^T  1^T c] [mu_W; lambda] = [-x_u,W; N_hat - 1^T x_u]
// (open arrays: the C_WW block alone).  The system is embedded in a fixed
// (NM [+1])-size SPD matrix with identity rows for dots outside W, so all
// indexing is static.  Primal-dual active-set update (Hintermueller, Ito and
// Kunisch, SIAM J. Optim. 13, 2003): keep dots with mu > 0, add dots with
// x < 0; stop when W repeats.  For open arrays C_dd is an M-matrix and W only
// grows (Chandrasekaran's method), at most N rounds.  Returns false when the
// iteration did not settle (x is then the last iterate, clipped at 0).
template <int NM, bool CLOSED>
__device__ bool qp_solve(const DiagRec *__restrict__ dr, const double (&xu)[NM], double (&x)[NM])
{
    constexpr int M = NM + (CLOSED ? 1 : 0);
    const int n = dr->n;
    double sx = 0.0, scale = 1.0, mu[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        sx += xu[i];
        scale = fmax(scale, fabs(xu[i]));
    }
    const double tol = 1e-13 * scale;
    const double lam0 = CLOSED ? ((double)dr->nhat - sx) / dr->one_c : 0.0;
    uint32_t W = 0;
#pragma unroll
    for (int i = 0; i < NM; ++i)
        if (i < n && xu[i] + lam0 * dr->c[i] < 0.0) W |= 1u << i;
    bool converged = false;
    for (int round = 0; round < 4 * NM + 4; ++round) {
        double a[M * (M + 1) / 2], b[M];
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            const bool wi = W >> i & 1u;
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                const bool wj = W >> j & 1u;
                double v = (wi && wj) ? dr->Cdd[i * kMaxDot + j] : 0.0;
                if (i == j && !wi) v = 1.0;
                a[i * (i + 1) / 2 + j] = v;
            }
            b[i] = wi ? -xu[i] : 0.0;
        }
        if (CLOSED) {
#pragma unroll
            for (int j = 0; j < NM; ++j)
                a[NM * (NM + 1) / 2 + j] = (W >> j & 1u) ? dr->c[j] : 0.0;
            a[NM * (NM + 1) / 2 + NM] = dr->one_c;
            b[M - 1] = (double)dr->nhat - sx;
        }
        chol_solve<M>(a, b);
        const double lam = CLOSED ? b[M - 1] : 0.0;
        uint32_t Wn = 0;
#pragma unroll
        for (int i = 0; i < NM; ++i) mu[i] = (W >> i & 1u) ? b[i] : 0.0;
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            double s = xu[i] + lam * dr->c[i];
#pragma unroll
            for (int j = 0; j < NM; ++j) s += dr->Cdd[i * kMaxDot + j] * mu[j];
            x[i] = (W >> i & 1u) ? 0.0 : s;
            if (i < n) {
                if (W >> i & 1u) {
                    if (mu[i] > -tol) Wn |= 1u << i;
                } else if (x[i] < -tol) {
                    Wn |= 1u << i;
                }
            }
        }
        if (Wn == W) { converged = true; break; }
        W = Wn;
    }
#pragma unroll
    for (int i = 0; i < NM; ++i) x[i] = (i < n) ? fmax(x[i], 0.0) : 0.0;
    return converged;
}

// ---------------------------------------------------------------------------
// candidate walk shared by the FP64 kernels.
//
// A pixel's candidates are n0 + 1_s for s within its free mask (m dots);
// a group of G = 2^LG lanes splits the 2^m compressed indices into chunks of
// consecutive integers and walks each chunk in Gray-code order, so that one
// dot flips per step and the flipped dot is the same in every lane of the
// group.  With y = A 1_s maintained incrementally,
//   U(n0 + 1_s) = U(n0) + sum_{i in s} (g0_i + y_i / 2)      (Eq. free_energy)
// ---------------------------------------------------------------------------
struct WalkState {
    uint32_t s;
    int pc;
};

template <int NM>
__device__ __forceinline__ double walk_energy(const double (&g0)[NM], const double (&y)[NM],
                                              double u0, uint32_t s)
{
    double e = u0;
#pragma unroll
    for (int i = 0; i < NM; ++i)
        if (s >> i & 1u) e += g0[i] + 0.5 * y[i];
    return e;
}

template <int NM>
__device__ __forceinline__ void walk_start(const double *__restrict__ sA, uint32_t s,
                                           double (&y)[NM])
{
#pragma unroll
    for (int i = 0; i < NM; ++i) y[i] = 0.0;
#pragma unroll
    for (int j = 0; j < NM; ++j)
        if (s >> j & 1u) {
#pragma unroll
            for (int i = 0; i < NM; ++i) y[i] += sA[j * kMaxDot + i];
        }
}

template <int NM>
__device__ __forceinline__ void walk_flip(const double *__restrict__ sA, uint64_t pos, int step,
                                          uint32_t &s, int &pc, double (&y)[NM])
{
    const int j = __ffs(step) - 1;
    const int d = (int)((pos >> (4 * j)) & 15u);
    const uint32_t bit = 1u << d;
    const double sg = (s & bit) ? -1.0 : 1.0;
    s ^= bit;
    pc += (s & bit) ? 1 : -1;
#pragma unroll
    for (int i = 0; i < NM; ++i) y[i] += sg * sA[d * kMaxDot + i];
}

__device__ __forceinline__ uint64_t free_positions(uint32_t fm)
{
    uint64_t pos = 0;
    for (int j = 0; fm; ++j) {
        pos |= (uint64_t)(__ffs(fm) - 1) << (4 * j);
        fm &= fm - 1;
    }
    return pos;
}

// All-reductions over aligned groups of 2^LG lanes.  A group of at most 16
// lanes lies inside one DPP row and takes the first LG of the row steps (each
// an involution, so every lane ends with the same bits); wider groups use
// LDS permutes.
template <int LG>
__device__ __forceinline__ double group_min(double v)
{
    if constexpr (LG <= 4) {
        if constexpr (LG >= 1) v = fmin(v, dppd<kDppXor1>(v));
        if constexpr (LG >= 2) v = fmin(v, dppd<kDppXor2>(v));
        if constexpr (LG >= 3) v = fmin(v, dppd<kDppHalfMirror>(v));
        if constexpr (LG >= 4) v = fmin(v, dppd<kDppMirror>(v));
    } else {
#pragma unroll
        for (int off = (1 << LG) / 2; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 1 << LG));
    }
    return v;
}

template <int LG>
__device__ __forceinline__ double group_sum(double v)
{
    if constexpr (LG <= 4) {
        if constexpr (LG >= 1) v += dppd<kDppXor1>(v);
        if constexpr (LG >= 2) v += dppd<kDppXor2>(v);
        if constexpr (LG >= 3) v += dppd<kDppHalfMirror>(v);
        if constexpr (LG >= 4) v += dppd<kDppMirror>(v);
    } else {
#pragma unroll
        for (int off = (1 << LG) / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 1 << LG);
    }
    return v;
}

// lane Q of each aligned group of 2^LG lanes to the whole group (a DPP row
// broadcast when the group is one row)
template <int LG, int Q>
__device__ __forceinline__ double lane_bcast(double v)
{
    if constexpr (LG == 4)
        return dppd<kDppRowBcast0 + Q>(v);
    else
        return __shfl(v, Q, 1 << LG);
}

// ---------------------------------------------------------------------------
// K0: per-diagram prologue
// ---------------------------------------------------------------------------
constexpr int kPrepThreads = 256;  // one thread per element of a 16 x 16 matrix

// Prologue of one diagram, run by one 256-thread block (thread t owns element
// (t / 16, t % 16)).  prep_inverse leaves in LDS the symmetric A = C_dd^{-1}
// (M, 256 doubles), C_dd 1 (cvec, 16 doubles), 1^T C_dd 1 (red[4]) and
// sum|A|/2 (red[5]); prep_store writes them and the pixel-independent energy
// tables to the diagram record.
//
// The inverse is an in-place Gauss-Jordan elimination of the positive
// definite C_dd without pivoting (every pivot is a diagonal entry of a
// Schur complement of a positive definite matrix, hence positive; the host
// has checked definiteness by Cholesky).  Pivot k maps
//   m_kk -> 1/p,  m_kj -> m_kj/p,  m_ik -> -m_ik/p,  m_ij -> m_ij - m_ik m_kj/p,
// and after the n pivots M = C_dd^{-1}.  Dots beyond n stay identity rows.
// sCdd: C_dd (kMaxDot x kMaxDot, row-major) already in LDS.  The caller
// has passed a barrier after filling it.
__device__ __forceinline__ void prep_inverse(const double *sCdd, int n, double *M, double *cvec,
                                             double *red)
{
    const int tid = threadIdx.x;
    if (tid < kWave) {
        // wave 0 eliminates in registers: lane l holds row l / 4, columns
        // 4 (l % 4) .. 4 (l % 4) + 3; the pivot row, the pivot column and the
        // pivot come from the owning lanes by shuffles (no barriers)
        const int i = tid >> 2, j0 = 4 * (tid & 3);
        double m[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j0 + q;
            m[q] = (i < n && j < n) ? sCdd[i * kMaxDot + j] : (i == j ? 1.0 : 0.0);
        }
#pragma unroll
        for (int k = 0; k < kMaxDot; ++k) {
            if (k < n) {
                const double mik = __shfl(m[k & 3], (i << 2) | (k >> 2));
                const double piv = __shfl(m[k & 3], (k << 2) | (k >> 2));
                double mk[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) mk[q] = __shfl(m[q], (k << 2) | (tid & 3));
                const double r = recip_nr(piv);
                const double mr = -mik * r;  // the new column k
                // branch-free selects (the four cases of the pivot map)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = j0 + q;
                    const double t1 = mk[q] * r;
                    const double t2 = fma(-mik, t1, m[q]);
                    const double v = (i == k) ? t1 : t2;
                    m[q] = (j == k) ? ((i == k) ? r : mr) : v;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) M[i * kMaxDot + j0 + q] = m[q];
    } else if (tid < kWave + kMaxDot) {
        // meanwhile, 16 lanes of wave 1: C_dd 1 and 1^T C_dd 1
        const int r = tid - kWave;
        double c = 0.0;
        if (r < n)
            for (int q = 0; q < n; ++q) c += sCdd[r * kMaxDot + q];
        cvec[r] = c;
        double oc = c;
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) oc += __shfl_xor(oc, off, 16);
        if (r == 0) red[4] = oc;
    }
    __syncthreads();
    const int i = tid >> 4, j = tid & 15;
    const double m = M[tid];
    // exactly symmetric A (the energy tables and every kernel read this copy)
    const double a = (i < n && j < n) ? 0.5 * (m + M[j * kMaxDot + i]) : 0.0;
    __syncthreads();
    M[tid] = a;
    // sum |A_ij| / 2: wave sums, then the four partial sums
    double sa = fabs(a);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) sa += __shfl_xor(sa, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = sa;
    __syncthreads();
    if (tid == 0) red[5] = 0.5 * (red[0] + red[1] + red[2] + red[3]);
    __syncthreads();
}

// compile-time loop: f(std::integral_constant<int, Q>) for Q in [Q0, Q1)
template <int Q0, int Q1, typename F>
__device__ __forceinline__ void static_for_dev(F &&f)
{
    if constexpr (Q0 < Q1) {
        f(std::integral_constant<int, Q0>{});
        static_for_dev<Q0 + 1, Q1>(f);
    }
}

// DPP row B (16 lanes) of x copied to all four rows, lane by lane: the
// 16-lane swap pairs rows (0, 1) and (2, 3), the 32-lane swap the halves
template <int B>
__device__ __forceinline__ uint32_t row_bcast_block32(uint32_t x)
{
    const auto p = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    const uint32_t y = (B & 1) ? p[1] : p[0];
    const auto h = __builtin_amdgcn_permlane32_swap(y, y, false, false);
    return (B & 2) ? h[1] : h[0];
}
template <int B>
__device__ __forceinline__ double row_bcast_block(double x)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t r = (uint64_t)row_bcast_block32<B>((uint32_t)u) |
                       ((uint64_t)row_bcast_block32<B>((uint32_t)(u >> 32)) << 32);
    return __longlong_as_double((long long)r);
}

// Wave 0 alone (no block barrier): the symmetric A = C_dd^{-1} into M and
// sum|A|/2 into red[5], by the same elimination as prep_inverse.  The other
// waves of the block may be doing anything meanwhile; the caller's next
// block barrier publishes M.
//
// The pivots run over the high dots 8..n-1 first, then 0..7: after the high
// pivots the working matrix holds (C_dd,HH)^{-1} in its high block, the Schur
// complement C_LL - C_LH C_HH^{-1} C_HL = (A_LL)^{-1} in its low block and
// C_HH^{-1} C_HL in its high-low block; the whole 16 x 16 matrix is copied to
// S when S is given (identity rows and columns past n).
__device__ __forceinline__ void prep_inverse_wave(const double (&m0)[4], int n, double *M,
                                                  double *red, double *S = nullptr)
{
    // lane = 16 b + j: column j of rows 4 b .. 4 b + 3 (a DPP row of the
    // wave holds four matrix rows), so the pivot column of a lane's rows is a
    // broadcast within its DPP row and the pivot row a broadcast of one DPP
    // row to the others (the gfx950 row swaps); no LDS round trip per pivot.
    // m0: the caller's C_dd in that layout, identity rows and columns past n.
    const int tid = threadIdx.x;
    const int j = tid & 15, b = tid >> 4;
    double m[4] = {m0[0], m0[1], m0[2], m0[3]};
    static_for_dev<0, kMaxDot>([&](auto kc) {
        constexpr int kk = decltype(kc)::value;
        constexpr int k = (kk + 8) & (kMaxDot - 1);
        if (kk == 8 && S) {
#pragma unroll
            for (int q = 0; q < 4; ++q) S[(4 * b + q) * kMaxDot + j] = m[q];
        }
        if (k < n) {
            // M[k][j] (pivot row) and M[4 b + q][k] (pivot column)
            // the pivot M[k][k] straight from its lane (16 (k / 4) + k,
            // element k % 4), so its reciprocal starts while the pivot row
            // is still being broadcast
            const uint64_t pu = (uint64_t)__double_as_longlong(m[k & 3]);
            constexpr int lk = 16 * (k >> 2) + k;
            const double piv = __longlong_as_double(
                (long long)((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)pu, lk) |
                            ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(pu >> 32), lk)
                             << 32)));
            const double r = recip_nr(piv);
            const double rowk = row_bcast_block<(k >> 2)>(m[k & 3]);
            double mik[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) mik[q] = dppd<kDppRowBcast0 + k>(m[q]);
            const double t1 = rowk * r;
            // branch-free selects (the four cases of the pivot map)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 4 * b + q;
                const double t2 = fma(-mik[q], t1, m[q]);
                const double v = (i == k) ? t1 : t2;
                m[q] = (j == k) ? ((i == k) ? r : -mik[q] * r) : v;
            }
        }
    });
#pragma unroll
    for (int q = 0; q < 4; ++q) M[(4 * b + q) * kMaxDot + j] = m[q];
    // exactly symmetric A: each lane reads the transposed entries (LDS
    // requests of one wave are served in order, so every lane's read of the
    // first pass precedes every write of the second)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double a[4], sa = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = 4 * b + q;
        a[q] = (i < n && j < n) ? 0.5 * (m[q] + M[j * kMaxDot + i]) : 0.0;
        sa += fabs(a[q]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int q = 0; q < 4; ++q) M[(4 * b + q) * kMaxDot + j] = a[q];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) sa += __shfl_xor(sa, off, 64);
    if (tid == 0) red[5] = 0.5 * sa;
}

// A, C_dd 1, 1^T C_dd 1 and sum|A|/2 into the record (one block)
__device__ __forceinline__ void prep_store_core(DiagRec *dr, const double *M, const double *cvec,
                                       const double *red)
{
    const int tid = threadIdx.x;
    for (int e = tid; e < kMaxDot * kMaxDot; e += blockDim.x) dr->A[e] = M[e];
    if (tid < kMaxDot) dr->c[tid] = cvec[tid];
    if (tid == 0) {
        dr->one_c = red[4];
        dr->sumabs = (float)red[5];
    }
}

// The energy tables from A in LDS, spread over the waves of a grid: entry e
// (of 256) goes to global wave e mod (number of waves), whose 64 lanes take
// the 8 x 8 products b_x b_y A_xy and sum them.
//
// With first/stride the caller picks the entries of this wave (default: the
// global wave index and the number of waves of the grid).
__device__ __forceinline__ void prep_tables_spread(DiagRec *dr, const double *M,
                                                   const double *S = nullptr, int first = -1,
                                                   int stride = 0, int n_dots = -1)
{
    const int n = n_dots >= 0 ? n_dots : dr->n;
    const int lane = threadIdx.x & (kWave - 1);
    const int gw = first >= 0 ? first : blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int nw = first >= 0 ? stride : gridDim.x * (blockDim.x / kWave);
    const int x = lane >> 3, y = lane & 7;
    const int nh = n - 8;
    for (int e = gw; e < 256; e += nw) {
        const bool both = (e >> x & 1) && (e >> y & 1);
        double hl = 0.0, hh = 0.0, hs = 0.0, sa = 0.0;
        if (n >= 9) {
            hl = both ? M[x * kMaxDot + y] : 0.0;
            hh = (both && x < nh && y < nh) ? M[(8 + x) * kMaxDot + 8 + y] : 0.0;
            if (S && x < nh && y < nh) {
                const double sxy = S[(8 + x) * kMaxDot + 8 + y];
                hs = both ? sxy : 0.0;
                sa = fabs(sxy);
            }
        } else if (e < (1 << n)) {
            hl = both ? M[x * kMaxDot + y] : 0.0;
        }
        hl = wave_sum(hl);
        hh = wave_sum(hh);
        if (S && n >= 9) {
            hs = wave_sum(hs);
            if (e == 0) sa = wave_sum(sa);
        }
        if (lane == 0) {
            if (n >= 9 && S) {
                dr->Hs[e] = (e < (1 << nh)) ? (float)(0.5 * hs) : 1e30f;
                if (e == 0) {
                    dr->sabsS = (float)(0.5 * sa);
                    // closed-array terms: w = C_HH^{-1} C_HL 1, gamma = 1^T A_LL^{-1} 1
                    double gam = 0.0;
                    for (int i = 0; i < 8; ++i)
                        for (int jj = 0; jj < 8; ++jj) gam += S[i * kMaxDot + jj];
                    for (int jj = 0; jj < 8; ++jj) {
                        double w = 0.0;
                        for (int i = 0; i < 8; ++i) w += S[(8 + jj) * kMaxDot + i];
                        dr->wB[jj] = (jj < nh) ? (float)w : 0.0f;
                    }
                    dr->inv2g = (float)(0.5 / gam);
                }
            }
            if (n >= 9) {
                dr->hlo[e] = (float)(0.5 * hl);
                dr->Hhi[e] = (e < (1 << nh)) ? (float)(0.5 * hh) : 1e30f;
                dr->hlod[e] = 0.5 * hl;
                dr->Hhid[e] = (e < (1 << nh)) ? 0.5 * hh : 1e300;
                if (e < 16 * 8) {
                    const int r = e >> 3, q = e & 7;
                    double t1 = 0.0, t2 = 0.0;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        if ((r >> b & 1) && b < nh) t1 += M[q * kMaxDot + 8 + b];
                        if ((r >> b & 1) && b + 4 < nh) t2 += M[q * kMaxDot + 12 + b];
                    }
                    dr->T1[r][q] = (float)t1;
                    dr->T2[r][q] = (float)t2;
                    dr->T1d[r][q] = t1;
                    dr->T2d[r][q] = t2;
                }
            } else {
                dr->hs[e] = 0.5 * hl;
            }
        }
    }
}

// everything the prologue stores, by one block
__device__ __forceinline__ void prep_store(DiagRec *dr, const double *M, const double *cvec,
                                  const double *red)
{
    const int n = dr->n;
    const int tid = threadIdx.x;
    prep_store_core(dr, M, cvec, red);
    // tables of the matrix-core scorer: low part = dots 0..7, high = 8..n-1
    if (n >= 9) {
        const int nh = n - 8;
        if (tid < 16 * 8) {
            const int r = tid >> 3, q = tid & 7;
            double t1 = 0.0, t2 = 0.0;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                if ((r >> b & 1) && b < nh) t1 += M[q * kMaxDot + 8 + b];
                if ((r >> b & 1) && b + 4 < nh) t2 += M[q * kMaxDot + 12 + b];
            }
            dr->T1[r][q] = (float)t1;
            dr->T2[r][q] = (float)t2;
            dr->T1d[r][q] = t1;
            dr->T2d[r][q] = t2;
        }
        double hh = 0.0, hl = 0.0;
#pragma unroll
        for (int x = 0; x < 8; ++x)
#pragma unroll
            for (int y = 0; y < 8; ++y) {
                if ((tid >> x & 1) && (tid >> y & 1)) {
                    hl += M[x * kMaxDot + y];
                    if (x < nh && y < nh) hh += M[(8 + x) * kMaxDot + 8 + y];
                }
            }
        dr->hlo[tid] = (float)(0.5 * hl);
        dr->Hhi[tid] = (tid < (1 << nh)) ? (float)(0.5 * hh) : 1e30f;
        dr->hlod[tid] = 0.5 * hl;
        dr->Hhid[tid] = (tid < (1 << nh)) ? 0.5 * hh : 1e300;
    } else {
        // whole-box table of the lane walk: h(s) = 1/2 s^T A s, s < 2^n
        double h = 0.0;
        if (tid < (1 << n)) {
#pragma unroll
            for (int x = 0; x < 8; ++x)
#pragma unroll
                for (int y = 0; y < 8; ++y)
                    if ((tid >> x & 1) && (tid >> y & 1)) h += M[x * kMaxDot + y];
        }
        dr->hs[tid] = 0.5 * h;
    }
}

// the whole prologue of one diagram by one block; sCdd is 256 doubles of LDS
__device__ __forceinline__ void prep_body(DiagRec *dr, double *sCdd, double *M, double *cvec,
                                          double *red)
{
    sCdd[threadIdx.x] = dr->Cdd[threadIdx.x];
    __syncthreads();
    prep_inverse(sCdd, dr->n, M, cvec, red);
    prep_store(dr, M, cvec, red);
}

}  // namespace qa
