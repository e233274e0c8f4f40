// qa_kernels.hip -- gfx950 kernels of the constant-capacitance ground-state
// path (van Straaten et al., arXiv 2404.04994), except the matrix-core
// scorer (qa_mfma.hip).
//
//   k_prep      per diagram: A = C_dd^{-1} (FP64 Cholesky), C_dd 1, the
//               pixel-independent energy tables (Sec. 2, Eq. free_energy).
//   k_setup     per pixel (lane = pixel): x_u = C_gd V, the analytic
//               continuous minimum (Sec. 3.1.1, App. C/D); pixels where it is
//               negative go to a list for k_qp; others get their candidate set
//               (Sec. 3.2) and the base-state gradient.
//   k_qp        per listed pixel: the constrained minimum of Sec. 3.1.2 in FP64
//               by a primal-dual active-set iteration whose linear systems are
//               solved by Cholesky in registers.
//   k_score_fp64  T = 0 argmin (Eq. argmin) over each pixel's candidate set,
//               FP64, a group of lanes per pixel walking a Gray code.
//   k_soft_fwd  kT > 0 softargmin (Sec. 4.2, Eq. softargmin), FP64.
//   k_soft_bwd  its adjoint with respect to C_dd, C_gd and V.
#include "qa_internal.h"

#include <math.h>

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

__global__ void k_zero_f64(double *p, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// ---------------------------------------------------------------------------
// K0: per-diagram prologue, one 64-thread block per diagram
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_prep(DiagRec *dr_all)
{
    DiagRec *dr = dr_all + blockIdx.x;
    __shared__ double L[kMaxDot * kMaxDot];
    __shared__ double Ainv[kMaxDot * kMaxDot];
    const int n = dr->n;
    const int tid = threadIdx.x;
    if (tid == 0) {
        // Cholesky C_dd = L L^T (the host has checked positive definiteness)
        for (int j = 0; j < n; ++j) {
            double d = dr->Cdd[j * kMaxDot + j];
            for (int k = 0; k < j; ++k) d -= L[j * kMaxDot + k] * L[j * kMaxDot + k];
            const double ljj = sqrt(d);
            L[j * kMaxDot + j] = ljj;
            for (int i = j + 1; i < n; ++i) {
                double s = dr->Cdd[i * kMaxDot + j];
                for (int k = 0; k < j; ++k) s -= L[i * kMaxDot + k] * L[j * kMaxDot + k];
                L[i * kMaxDot + j] = s / ljj;
            }
        }
    }
    __syncthreads();
    if (tid < n) {
        // column tid of A: L y = e_tid, then L^T a = y
        double y[kMaxDot], a[kMaxDot];
        for (int i = 0; i < n; ++i) {
            double s = (i == tid) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[i * kMaxDot + k] * y[k];
            y[i] = s / L[i * kMaxDot + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < n; ++k) s -= L[k * kMaxDot + i] * a[k];
            a[i] = s / L[i * kMaxDot + i];
        }
        for (int i = 0; i < n; ++i) Ainv[i * kMaxDot + tid] = a[i];
    }
    __syncthreads();
    for (int e = tid; e < kMaxDot * kMaxDot; e += blockDim.x) {
        const int i = e / kMaxDot, j = e % kMaxDot;
        double v = 0.0;
        if (i < n && j < n) v = 0.5 * (Ainv[i * kMaxDot + j] + Ainv[j * kMaxDot + i]);
        dr->A[e] = v;
        Ainv[e] = v;  // exactly symmetric copy for the tables below
    }
    __syncthreads();
    if (tid < kMaxDot) {
        double s = 0.0;
        if (tid < n)
            for (int j = 0; j < n; ++j) s += dr->Cdd[tid * kMaxDot + j];
        dr->c[tid] = s;
    }
    if (tid == 0) {
        double s = 0.0, sa = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                s += dr->Cdd[i * kMaxDot + j];
                sa += fabs(Ainv[i * kMaxDot + j]);
            }
        dr->one_c = s;
        dr->sumabs = (float)(0.5 * sa);
    }
    // tables of the matrix-core scorer: low part = dots 0..7, high = 8..n-1
    if (n >= 9) {
        const int nh = n - 8;
        for (int e = tid; e < 16 * 8; e += blockDim.x) {
            const int r = e / 8, i = e % 8;
            double t1 = 0.0, t2 = 0.0;
            for (int j = 0; j < 4; ++j) {
                if ((r >> j & 1) && j < nh) t1 += Ainv[i * kMaxDot + 8 + j];
                if ((r >> j & 1) && j + 4 < nh) t2 += Ainv[i * kMaxDot + 12 + j];
            }
            dr->T1[r][i] = (float)t1;
            dr->T2[r][i] = (float)t2;
        }
        for (int e = tid; e < 256; e += blockDim.x) {
            double hh = 0.0, hl = 0.0;
            for (int a = 0; a < 8; ++a)
                for (int b = 0; b < 8; ++b) {
                    if ((e >> a & 1) && (e >> b & 1)) {
                        hl += Ainv[a * kMaxDot + b];
                        if (a < nh && b < nh) hh += Ainv[(8 + a) * kMaxDot + 8 + b];
                    }
                }
            dr->hlo[e] = (float)(0.5 * hl);
            dr->Hhi[e] = (e < (1 << nh)) ? (float)(0.5 * hh) : 1e30f;
        }
    }
}

hipError_t launch_prep(DiagRec *dr, int n_diag, hipStream_t s)
{
    hipLaunchKernelGGL(k_prep, dim3(n_diag), dim3(64), 0, s, dr);
    return hipGetLastError();
}

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

__device__ __forceinline__ void block_add_counter(int64_t *counters, int which, int64_t v)
{
    if (v) atomicAdd((unsigned long long *)&counters[which], (unsigned long long)v);
}

// ---------------------------------------------------------------------------
// K1: candidate set and base-state gradient of one pixel
// ---------------------------------------------------------------------------
template <int NM, bool CLOSED>
__device__ void finish_pixel(const DiagRec *__restrict__ dr, const double (&x)[NM],
                             const double (&xu)[NM], int flags, PixRec *__restrict__ out,
                             int *doubled)
{
    const int n = dr->n;
    double t = dr->t;
    int n0[NM];
    uint32_t fm = 0;
    int k = -1;
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
        if (!CLOSED) break;
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
    *doubled = (flags & 4) ? 1 : 0;
    double z[NM], g0[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) z[i] = (i < n) ? (double)n0[i] - xu[i] : 0.0;
    double u0 = 0.0;
#pragma unroll
    for (int i = 0; i < NM; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NM; ++j) s += dr->A[i * kMaxDot + j] * z[j];
        g0[i] = s;
        u0 += z[i] * s;
    }
#pragma unroll
    for (int i = 0; i < kMaxDot; ++i) {
        out->g0[i] = (i < NM) ? g0[i] : 0.0;
        out->n0[i] = (i < NM) ? (int16_t)n0[i] : (int16_t)0;
    }
    out->u0 = 0.5 * u0;
    out->free = fm;
    out->k = k;
    out->flags = flags;
}

template <int NM, bool CLOSED>
__global__ __launch_bounds__(256) void k_setup(const DiagRec *__restrict__ dr,
                                               const double *__restrict__ V, int64_t P,
                                               PixRec *__restrict__ pr,
                                               int32_t *__restrict__ qp_list,
                                               int64_t *__restrict__ counters)
{
    __shared__ int64_t sc[3];
    if (threadIdx.x < 3) sc[threadIdx.x] = 0;
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) {
        const int n = dr->n, g = dr->g;
        double xu[NM], x[NM];
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            double s = 0.0;
            if (i < n)
                for (int j = 0; j < g; ++j) s += dr->Cgd[i * kMaxGate + j] * V[p * g + j];
            xu[i] = s;
        }
        // analytic minimum: open x = x_u; closed adds (N_hat - 1^T x_u) C_dd 1 / (1^T C_dd 1)
        double lam = 0.0;
        if (CLOSED) {
            double sx = 0.0;
#pragma unroll
            for (int i = 0; i < NM; ++i) sx += xu[i];
            lam = ((double)dr->nhat - sx) / dr->one_c;
        }
        bool feasible = true;
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            x[i] = (i < n) ? xu[i] + lam * dr->c[i] : 0.0;
            feasible &= x[i] >= 0.0;
        }
        bool solved_qp = false;
        if (CLOSED && dr->nhat == 0) {
            // x = 0 is the only admissible point of a closed empty array, so
            // it is the QP's solution whenever the analytic one is negative
            solved_qp = !feasible;
#pragma unroll
            for (int i = 0; i < NM; ++i) x[i] = 0.0;
            feasible = true;
        }
        if (feasible) {
            int dbl = 0;
            finish_pixel<NM, CLOSED>(dr, x, xu, solved_qp ? 1 : 0, pr + p, &dbl);
            if (dbl) atomicAdd((unsigned long long *)&sc[2], 1ull);
            if (solved_qp) atomicAdd((unsigned long long *)&sc[1], 1ull);
        } else {
            const unsigned long long slot =
                atomicAdd((unsigned long long *)&counters[C_QP_LIST], 1ull);
            qp_list[slot] = (int32_t)p;
            atomicAdd((unsigned long long *)&sc[1], 1ull);
        }
        atomicAdd((unsigned long long *)&sc[0], 1ull);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        block_add_counter(counters, C_PIXELS, sc[0]);
        block_add_counter(counters, C_QP, sc[1]);
        block_add_counter(counters, C_DOUBLED, sc[2]);
    }
}

// Cholesky solve of an SPD system held as a packed lower triangle, M fixed.
template <int M>
__device__ __forceinline__ void chol_solve(double (&a)[M * (M + 1) / 2], double (&b)[M])
{
#define LIDX(i, j) ((i) * ((i) + 1) / 2 + (j))
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double d = a[LIDX(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= a[LIDX(j, k)] * a[LIDX(j, k)];
        d = sqrt(d);
        a[LIDX(j, j)] = d;
        const double inv = 1.0 / d;
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
        b[i] = s / a[LIDX(i, i)];
    }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        double s = b[i];
#pragma unroll
        for (int k = i + 1; k < M; ++k) s -= a[LIDX(k, i)] * b[k];
        b[i] = s / a[LIDX(i, i)];
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
// grows (Chandrasekaran's method), at most N rounds.
template <int NM, bool CLOSED>
__global__ __launch_bounds__(64) void k_qp(const DiagRec *__restrict__ dr,
                                           const double *__restrict__ V, int64_t P,
                                           PixRec *__restrict__ pr,
                                           const int32_t *__restrict__ qp_list,
                                           int64_t *__restrict__ counters)
{
    constexpr int M = NM + (CLOSED ? 1 : 0);
    const int64_t count = counters[C_QP_LIST];
    const int n = dr->n, g = dr->g;
    int64_t fails = 0, dbls = 0;
    for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < count;
         it += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = qp_list[it];
        double xu[NM], x[NM], mu[NM];
        double sx = 0.0, scale = 1.0;
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            double s = 0.0;
            if (i < n)
                for (int j = 0; j < g; ++j) s += dr->Cgd[i * kMaxGate + j] * V[p * g + j];
            xu[i] = s;
            sx += s;
            scale = fmax(scale, fabs(s));
        }
        const double tol = 1e-13 * scale;
        double lam0 = CLOSED ? ((double)dr->nhat - sx) / dr->one_c : 0.0;
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
            for (int i = 0; i < NM; ++i) {
                mu[i] = (W >> i & 1u) ? b[i] : 0.0;
            }
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
        int dbl = 0;
        finish_pixel<NM, CLOSED>(dr, x, xu, 1 | (converged ? 0 : 2), pr + p, &dbl);
        fails += converged ? 0 : 1;
        dbls += dbl;
    }
    if (fails) atomicAdd((unsigned long long *)&counters[C_QP_FAIL], (unsigned long long)fails);
    if (dbls) atomicAdd((unsigned long long *)&counters[C_DOUBLED], (unsigned long long)dbls);
}

#define QA_DISPATCH_NM(n, CALL)                        \
    do {                                               \
        if ((n) <= 2) { constexpr int NM_ = 2; CALL; } \
        else if ((n) <= 4) { constexpr int NM_ = 4; CALL; } \
        else if ((n) <= 8) { constexpr int NM_ = 8; CALL; } \
        else { constexpr int NM_ = 16; CALL; }         \
    } while (0)

hipError_t launch_setup(const DiagRec *dr, const double *V, int64_t P, PixRec *pr,
                        int32_t *qp_list, int64_t *counters, int n_dot, bool closed,
                        hipStream_t s)
{
    const dim3 grid((unsigned)((P + 255) / 256)), block(256);
    if (closed)
        QA_DISPATCH_NM(n_dot, hipLaunchKernelGGL((k_setup<NM_, true>), grid, block, 0, s, dr, V, P,
                                                 pr, qp_list, counters));
    else
        QA_DISPATCH_NM(n_dot, hipLaunchKernelGGL((k_setup<NM_, false>), grid, block, 0, s, dr, V,
                                                 P, pr, qp_list, counters));
    return hipGetLastError();
}

hipError_t launch_qp(const DiagRec *dr, const double *V, int64_t P, PixRec *pr,
                     const int32_t *qp_list, int64_t *counters, int n_dot, bool closed,
                     hipStream_t s)
{
    // grid-stride over the list, whose length is only known on the device
    int64_t blocks = (P + 63) / 64;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    const dim3 grid((unsigned)blocks), block(64);
    if (closed)
        QA_DISPATCH_NM(n_dot, hipLaunchKernelGGL((k_qp<NM_, true>), grid, block, 0, s, dr, V, P, pr,
                                                 qp_list, counters));
    else
        QA_DISPATCH_NM(n_dot, hipLaunchKernelGGL((k_qp<NM_, false>), grid, block, 0, s, dr, V, P, pr,
                                                 qp_list, counters));
    return hipGetLastError();
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

template <int LG>
__device__ __forceinline__ double group_min(double v)
{
#pragma unroll
    for (int off = (1 << LG) / 2; off >= 1; off >>= 1) v = fmin(v, __shfl_xor(v, off, 1 << LG));
    return v;
}

template <int LG>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int off = (1 << LG) / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 1 << LG);
    return v;
}

// ---------------------------------------------------------------------------
// K2 (FP64): T = 0 argmin and runner-up over the candidate set
// ---------------------------------------------------------------------------
template <int LG, int NM>
__global__ __launch_bounds__(256) void k_score_fp64(const DiagRec *__restrict__ dr,
                                                    const PixRec *__restrict__ pr, int64_t P,
                                                    const int32_t *__restrict__ list,
                                                    const int64_t *__restrict__ list_count,
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
    const int64_t count = list ? *list_count : P;
    for (int64_t it = gid; it < count; it += ngroups) {
        const int64_t p = list ? list[it] : it;
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
        if (!list) block_add_counter(counters, C_CANDIDATES, (int64_t)sc[1]);
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

static unsigned group_blocks(int64_t items, int lg, int64_t cap)
{
    const int64_t per_block = 256 >> lg;
    int64_t b = (items + per_block - 1) / per_block;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_score_fp64(const DiagRec *dr, const PixRec *pr, int64_t P,
                             const int32_t *list, const int64_t *list_count, int32_t *n_out,
                             int64_t *counters, int n_dot, hipStream_t s)
{
    QA_DISPATCH_GROUP(n_dot, hipLaunchKernelGGL((k_score_fp64<LG_, NM_>),
                                                dim3(group_blocks(P, LG_, 8192)), dim3(256), 0, s,
                                                dr, pr, P, list, list_count, n_out, counters));
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
        double g0[NM], sv[NM];
#pragma unroll
        for (int i = 0; i < NM; ++i) g0[i] = r->g0[i];
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
                o->logZ = log(Z);
                for (int i = 0; i < kMaxDot; ++i) o->n0[i] = r->n0[i];
                o->free = r->free;
                o->k = r->k;
            }
        }
    }
}

hipError_t launch_soft_fwd(const DiagRec *dr, const PixRec *pr, int64_t P, double *nbar,
                           SavedRec *saved, int64_t *counters, int n_dot, hipStream_t s)
{
    QA_DISPATCH_GROUP(n_dot, hipLaunchKernelGGL((k_soft_fwd<LG_, NM_>),
                                                dim3(group_blocks(P, LG_, 8192)), dim3(256), 0, s,
                                                dr, pr, P, nbar, saved, counters));
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

template <int LG, int NM>
__global__ __launch_bounds__(256) void k_soft_bwd(const DiagRec *__restrict__ dr,
                                                  const double *__restrict__ V, int64_t P,
                                                  const double *__restrict__ gbar,
                                                  const SavedRec *__restrict__ saved,
                                                  double *__restrict__ accA,
                                                  double *__restrict__ accG,
                                                  double *__restrict__ accU,
                                                  double *__restrict__ gradV)
{
    constexpr int G = 1 << LG;
    constexpr int NU = 1 << (NM < kBwdMaxDot ? NM : kBwdMaxDot);
    __shared__ double sA[kMaxDot * kMaxDot];
    __shared__ double sU[NU];
    __shared__ double sdA[kMaxDot * kMaxDot];
    __shared__ double sdG[kMaxDot * kMaxGate];
    for (int i = threadIdx.x; i < kMaxDot * kMaxDot; i += blockDim.x) {
        sA[i] = dr->A[i];
        sdA[i] = 0.0;
    }
    for (int i = threadIdx.x; i < NU; i += blockDim.x) sU[i] = 0.0;
    for (int i = threadIdx.x; i < kMaxDot * kMaxGate; i += blockDim.x) sdG[i] = 0.0;
    __syncthreads();
    const int n = dr->n, g = dr->g;
    const double kT = dr->kT;
    const int lane = threadIdx.x & (G - 1);
    const int64_t gid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> LG;
    const int64_t ngroups = ((int64_t)gridDim.x * blockDim.x) >> LG;
    for (int64_t p = gid; p < P; p += ngroups) {
        const SavedRec *sr = saved + p;
        double xu[NM], z[NM], g0[NM], gb[NM];
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            double s = 0.0;
            if (i < n)
                for (int j = 0; j < g; ++j) s += dr->Cgd[i * kMaxGate + j] * V[p * g + j];
            xu[i] = s;
            z[i] = (i < n) ? (double)sr->n0[i] - s : 0.0;
            gb[i] = (i < n) ? gbar[p * n + i] : 0.0;
        }
        double u0 = 0.0;
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < NM; ++j) s += sA[i * kMaxDot + j] * z[j];
            g0[i] = s;
            u0 += z[i] * s;
        }
        u0 *= 0.5;
        const uint32_t fm = sr->free;
        const int k = sr->k;
        const double emin = sr->emin;
        const int m = __popc(fm);
        const uint64_t pos = free_positions(fm);
        const int chunk_log = m > LG ? m - LG : 0;
        const bool active = (m >= LG) || (lane < (1 << m));
        const uint32_t c0 = (uint32_t)lane << chunk_log;
        const int steps = 1 << chunk_log;
        double y[NM];
        // pass 1: normaliser and mean offset
        double zsum = 0.0, nb[NM];
#pragma unroll
        for (int i = 0; i < NM; ++i) nb[i] = 0.0;
        if (active) {
            uint32_t s = pdep_mask(c0 ^ (c0 >> 1), fm);
            int pc = __popc(s);
            walk_start<NM>(sA, s, y);
            for (int step = 0; step < steps; ++step) {
                if (step) walk_flip<NM>(sA, pos, step, s, pc, y);
                if (k < 0 || pc == k) {
                    const double w = exp(-(walk_energy<NM>(g0, y, u0, s) - emin) / kT);
                    zsum += w;
#pragma unroll
                    for (int i = 0; i < NM; ++i)
                        if (s >> i & 1u) nb[i] += w;
                }
            }
        }
        const double Z = group_sum<LG>(zsum);
        double gnb = 0.0;
#pragma unroll
        for (int i = 0; i < NM; ++i) {
            nb[i] = group_sum<LG>(nb[i]) / Z;
            gnb += gb[i] * nb[i];
        }
        // pass 2: ubar_s, m_p and u_s
        double mv[NM];
#pragma unroll
        for (int i = 0; i < NM; ++i) mv[i] = 0.0;
        if (active) {
            uint32_t s = pdep_mask(c0 ^ (c0 >> 1), fm);
            int pc = __popc(s);
            walk_start<NM>(sA, s, y);
            for (int step = 0; step < steps; ++step) {
                if (step) walk_flip<NM>(sA, pos, step, s, pc, y);
                if (k < 0 || pc == k) {
                    const double pi = exp(-(walk_energy<NM>(g0, y, u0, s) - emin) / kT) / Z;
                    double gs = 0.0;
#pragma unroll
                    for (int i = 0; i < NM; ++i)
                        if (s >> i & 1u) gs += gb[i];
                    const double ub = -(pi / kT) * (gs - gnb);
#pragma unroll
                    for (int i = 0; i < NM; ++i)
                        if (s >> i & 1u) mv[i] += ub;
                    atomicAdd(&sU[s], ub);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < NM; ++i) mv[i] = group_sum<LG>(mv[i]);
        if (lane == 0) {
            double dx[NM];
#pragma unroll
            for (int i = 0; i < NM; ++i) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < NM; ++j) s += sA[i * kMaxDot + j] * mv[j];
                dx[i] = -s;
            }
#pragma unroll
            for (int i = 0; i < NM; ++i)
#pragma unroll
                for (int j = 0; j < NM; ++j)
                    if (i < n && j < n)
                        atomicAdd(&sdA[i * kMaxDot + j], 0.5 * (z[i] * mv[j] + mv[i] * z[j]));
            for (int j = 0; j < g; ++j) {
                const double vj = V[p * g + j];
                double gv = 0.0;
#pragma unroll
                for (int i = 0; i < NM; ++i) {
                    if (i < n) {
                        atomicAdd(&sdG[i * kMaxGate + j], dx[i] * vj);
                        gv += dr->Cgd[i * kMaxGate + j] * dx[i];
                    }
                }
                if (gradV) gradV[p * g + j] = gv;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kMaxDot * kMaxDot; i += blockDim.x)
        if (sdA[i] != 0.0) atomicAdd(&accA[i], sdA[i]);
    for (int i = threadIdx.x; i < kMaxDot * kMaxGate; i += blockDim.x)
        if (sdG[i] != 0.0) atomicAdd(&accG[i], sdG[i]);
    for (int i = threadIdx.x; i < NU; i += blockDim.x)
        if (sU[i] != 0.0) atomicAdd(&accU[i], sU[i]);
}

__global__ __launch_bounds__(256) void k_soft_bwd_final(const DiagRec *__restrict__ dr,
                                                        const double *__restrict__ accA,
                                                        const double *__restrict__ accG,
                                                        const double *__restrict__ accU,
                                                        double *__restrict__ grad_cdd,
                                                        double *__restrict__ grad_cgd)
{
    __shared__ double dA[kMaxDot * kMaxDot];
    __shared__ double T[kMaxDot * kMaxDot];
    const int n = dr->n, g = dr->g;
    const int tid = threadIdx.x;
    for (int e = tid; e < kMaxDot * kMaxDot; e += blockDim.x) {
        const int i = e / kMaxDot, j = e % kMaxDot;
        double v = accA[e];
        if (i < n && j < n) {
            // 1/2 sum_s u_s [i in s][j in s]
            const uint32_t need = (1u << i) | (1u << j);
            double q = 0.0;
            for (uint32_t s = 0; s < (1u << n); ++s)
                if ((s & need) == need) q += accU[s];
            v += 0.5 * q;
        }
        dA[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < kMaxDot * kMaxDot; e += blockDim.x) {
        const int i = e / kMaxDot, j = e % kMaxDot;
        double v = 0.0;
        for (int a = 0; a < n; ++a) v += dA[i * kMaxDot + a] * dr->A[a * kMaxDot + j];
        T[e] = v;  // (dL/dA) A
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += blockDim.x) {
        const int i = e / n, j = e % n;
        double v = 0.0;
        for (int a = 0; a < n; ++a) v += dr->A[i * kMaxDot + a] * T[a * kMaxDot + j];
        grad_cdd[e] = -v;
    }
    for (int e = tid; e < n * g; e += blockDim.x) {
        const int i = e / g, j = e % g;
        grad_cgd[e] = accG[i * kMaxGate + j];
    }
}

hipError_t launch_soft_bwd(const DiagRec *dr, const double *V, int64_t P, const double *gbar,
                           const SavedRec *saved, double *accA, double *accG, double *accU,
                           double *gradV, int n_dot, hipStream_t s)
{
    // accumulators: kMaxDot^2 + kMaxDot*kMaxGate + 2^n doubles, contiguous
    const int64_t nacc = (int64_t)kMaxDot * kMaxDot + (int64_t)kMaxDot * kMaxGate + (1 << n_dot);
    hipLaunchKernelGGL(k_zero_f64, dim3((unsigned)((nacc + 255) / 256)), dim3(256), 0, s, accA,
                       nacc);
    if (n_dot <= 8) {
        QA_DISPATCH_GROUP(n_dot, hipLaunchKernelGGL((k_soft_bwd<LG_, NM_>),
                                                    dim3(group_blocks(P, LG_, 2048)), dim3(256), 0,
                                                    s, dr, V, P, gbar, saved, accA, accG, accU,
                                                    gradV));
    } else {
        hipLaunchKernelGGL((k_soft_bwd<6, 16>), dim3(group_blocks(P, 6, 2048)), dim3(256), 0, s,
                           dr, V, P, gbar, saved, accA, accG, accU, gradV);
    }
    return hipGetLastError();
}

hipError_t launch_soft_bwd_final(const DiagRec *dr, const double *accA, const double *accG,
                                 const double *accU, double *grad_cdd, double *grad_cgd,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(k_soft_bwd_final, dim3(1), dim3(256), 0, s, dr, accA, accG, accU, grad_cdd,
                       grad_cgd);
    return hipGetLastError();
}

}  // namespace qa
