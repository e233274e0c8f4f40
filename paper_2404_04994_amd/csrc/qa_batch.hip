// qa_batch.hip -- a ragged batch of stability diagrams (different dot counts,
// open and closed arrays, different temperatures) in one persistent launch,
// the dataset-generation use the paper motivates (Sec. 1, Sec. 8).
//
//   k_prep_batch  one block per diagram: copies C_dd, C_gd and the solve
//                 mode into a DiagRec and runs the same prologue as a single
//                 diagram (A = C_dd^{-1} in FP64).
//   k_batch       persistent: each wave takes 64-pixel work items from a
//                 queue; a work item belongs to one diagram, so every lane of
//                 the wave shares its dot count and candidate layout.  Lane =
//                 pixel, and the whole path runs in registers: x_u = C_gd V,
//                 the analytic minimum or the exact QP (Sec. 3.1), the
//                 candidate set (Sec. 3.2), the argmin (Eq. argmin) and, when
//                 kT > 0, the softargmin (Eq. softargmin) over the set, all
//                 energies in FP64.  Nothing per pixel goes back to HBM except
//                 the results.
#include "qa_device.h"

namespace qa {

__global__ __launch_bounds__(kPrepThreads) void k_prep_batch(const BatchHdr *__restrict__ hdr,
                                                   const double *__restrict__ mats,
                                                   DiagRec *__restrict__ recs)
{
    __shared__ double sCdd[kMaxDot * kMaxDot];
    __shared__ double M[kMaxDot * kMaxDot];
    __shared__ double cvec[kMaxDot];
    __shared__ double red[8];
    const BatchHdr h = hdr[blockIdx.x];
    DiagRec *dr = recs + blockIdx.x;
    const int n = h.n, g = h.g;
    const double *cdd = mats + h.mat_off;
    const double *cgd = cdd + n * n;
    for (int e = threadIdx.x; e < kMaxDot * kMaxDot; e += blockDim.x) {
        const int i = e / kMaxDot, j = e % kMaxDot;
        dr->Cdd[e] = (i < n && j < n) ? cdd[i * n + j] : 0.0;
    }
    for (int e = threadIdx.x; e < kMaxDot * kMaxGate; e += blockDim.x) {
        const int i = e / kMaxGate, j = e % kMaxGate;
        dr->Cgd[e] = (i < n && j < g) ? cgd[i * g + j] : 0.0;
    }
    if (threadIdx.x == 0) {
        dr->n = n;
        dr->g = g;
        dr->closed = h.closed;
        dr->nhat = h.nhat;
        dr->kT = h.kT;
        dr->t = h.t;
        dr->prec = 0;
    }
    __syncthreads();
    prep_body(dr, sCdd, M, cvec, red);
}

hipError_t launch_prep_batch(const BatchHdr *hdr, const double *mats, DiagRec *recs, int n_diag,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_prep_batch, dim3(n_diag), dim3(kPrepThreads), 0, s, hdr, mats, recs);
    return hipGetLastError();
}

// Dense box of n <= 8 dots (every dot free), walked by one lane.  With s the
// raised dots and h(s) = 1/2 s^T A s from the diagram's table (LDS),
//     U(n0 + s) - U(n0) = s . g0 + h(s)                       (Eq. free_energy)
// The 2^n states are visited in blocks of sixteen Gray-code steps: inside a
// block only dots 0..3 flip, the flipped dot and (for dots 0..2) its new value
// are compile-time constants, and gray(16 o + k) = gray(16 o) ^ gray(k).
// Pass 1 finds the smallest energy; pass 2 finds the lexicographically
// smallest state at that energy (the rank brev(s)), the runner-up energy and,
// for kT > 0, the Boltzmann sums (weights by the hardware exp2 in FP32 of
// an FP64 argument, relative error below 3e-6 for every weight above e^-60;
// sums in FP64).
template <int NM>
__device__ __forceinline__ int64_t dense_small(const double *__restrict__ sh,
                                               const double (&g0)[NM], int n, int k, double kT,
                                               bool soft, double &e1out, double &e2out,
                                               uint32_t &s1out, double &Z, double (&sv)[NM])
{
    const int nb = n > 4 ? 1 << (n - 4) : 1;
    const int kmax = n >= 4 ? 16 : 1 << n;
    int64_t scored = 0;
    double e1 = INFINITY;
    for (int o = 0; o < nb; ++o) {
        const uint32_t sb = ((uint32_t)o << 4) ^ ((uint32_t)o << 3);
        const int par = o & 1;
        const int pchi = __popc(sb >> 4);
        double L = 0.0;
#pragma unroll
        for (int i = 0; i < NM; ++i)
            if (sb >> i & 1u) L += g0[i];
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const uint32_t gk = (uint32_t)(kk ^ (kk >> 1));
            if (kk > 0) {
                const int d = __builtin_ctz(kk);
                if (d < 3) L += ((gk >> d) & 1u) ? g0[d] : -g0[d];
                else L += par ? -g0[3] : g0[3];
            }
            if (kk < kmax) {
                const bool valid = k < 0 || pchi + __popc((gk ^ ((uint32_t)par << 3)) & 15u) == k;
                if (valid) {
                    e1 = fmin(e1, L + sh[sb ^ gk]);
                    ++scored;
                }
            }
        }
    }
    const double c = soft ? 1.4426950408889634 / kT : 0.0;
    uint32_t r1 = 0xFFFFFFFFu;
    int neq = 0;
    double e2 = INFINITY;
#pragma unroll
    for (int i = 0; i < NM; ++i) sv[i] = 0.0;
    Z = 0.0;
    for (int o = 0; o < nb; ++o) {
        const uint32_t sb = ((uint32_t)o << 4) ^ ((uint32_t)o << 3);
        const uint32_t rb = __brev(sb);
        const int par = o & 1;
        const int pchi = __popc(sb >> 4);
        double L = 0.0;
#pragma unroll
        for (int i = 0; i < NM; ++i)
            if (sb >> i & 1u) L += g0[i];
        float sblk = 0.0f, t0 = 0.0f, t1 = 0.0f, t2 = 0.0f, t3 = 0.0f;
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            const uint32_t gk = (uint32_t)(kk ^ (kk >> 1));
            if (kk > 0) {
                const int d = __builtin_ctz(kk);
                if (d < 3) L += ((gk >> d) & 1u) ? g0[d] : -g0[d];
                else L += par ? -g0[3] : g0[3];
            }
            if (kk < kmax) {
                const bool valid = k < 0 || pchi + __popc((gk ^ ((uint32_t)par << 3)) & 15u) == k;
                if (valid) {
                    const double e = L + sh[sb ^ gk];
                    if (e == e1) {
                        r1 = min(r1, rb ^ __brev(gk));
                        ++neq;
                    } else {
                        e2 = fmin(e2, e);
                    }
                    if (soft) {
                        const float w = __builtin_amdgcn_exp2f((float)((e1 - e) * c));
                        sblk += w;
                        if (gk & 1u) t0 += w;
                        if (gk & 2u) t1 += w;
                        if (gk & 4u) t2 += w;
                        if (gk & 8u) t3 += w;
                    }
                }
            }
        }
        if (soft) {
            Z += sblk;
            sv[0] += t0;
            if (NM > 1) sv[1] += t1;
            if (NM > 2) sv[2] += t2;
            if (NM > 3) sv[3] += par ? (double)(sblk - t3) : (double)t3;
#pragma unroll
            for (int i = 4; i < NM; ++i)
                if (sb >> i & 1u) sv[i] += sblk;
        }
    }
    e1out = e1;
    e2out = neq > 1 ? e1 : e2;
    s1out = __brev(r1);
    return scored;
}

// one pixel, lane-sequential: returns the number of candidates scored
// (volt(j): the pixel's voltage of gate j)
template <int NM, typename Volt>
__device__ __forceinline__ int64_t batch_pixel(const DiagRec *__restrict__ dr,
                                               const double *__restrict__ A,
                                               const double *__restrict__ hs, bool closed,
                                               Volt &&volt,
                                               int32_t *__restrict__ nout,
                                               double *__restrict__ nbout, int &qp, int &fail,
                                               int &dbl, int &gap)
{
    const int n = dr->n, g = dr->g;
    // x_u = C_gd V, gate by gate: each voltage is read (or formed) once,
    // and every x_u,i still sums over j in increasing order
    double xu[NM], x[NM];
#pragma unroll
    for (int i = 0; i < NM; ++i) xu[i] = 0.0;
    for (int j = 0; j < g; ++j) {
        const double vj = volt(j);
#pragma unroll
        for (int i = 0; i < NM; ++i)
            if (i < n) xu[i] += dr->Cgd[i * kMaxGate + j] * vj;
    }
    // analytic minimum first (Sec. 3.1.1), the QP only when it is negative
    double lam = 0.0;
    if (closed) {
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
    if (closed && dr->nhat == 0) {
        qp = !feasible;
#pragma unroll
        for (int i = 0; i < NM; ++i) x[i] = 0.0;
        feasible = true;
    }
    if (!feasible) {
        qp = 1;
        bool ok = false;
        if constexpr (NM <= 8) {
            // the QP at the diagram's own size (its factorisation is cubic in
            // the order; dots n.. of x are zero already).  The rest of the
            // path stays at NM: one copy of it per dot count made the kernel
            // too large for the instruction cache.
            static_for_dev<1, NM + 1>([&](auto kc) {
                constexpr int K = decltype(kc)::value;
                if (n == K) {
                    const double(&xk)[K] = *reinterpret_cast<const double(*)[K]>(&xu[0]);
                    double(&yk)[K] = *reinterpret_cast<double(*)[K]>(&x[0]);
                    ok = closed ? qp_solve<K, true>(dr, xk, yk) : qp_solve<K, false>(dr, xk, yk);
                }
            });
        } else {
            ok = closed ? qp_solve<NM, true>(dr, xu, x) : qp_solve<NM, false>(dr, xu, x);
        }
        fail = ok ? 0 : 1;
    }
    int n0[NM];
    uint32_t fm;
    int k;
    const int flags = candidate_set<NM>(dr, closed, x, n0, fm, k);
    dbl = (flags & 4) ? 1 : 0;
    double g0[NM];
    double u0 = 0.0;
    if constexpr (NM <= 8) {
        // at the diagram's own size too (quadratic in it; the padding of A
        // adds zeros only)
#pragma unroll
        for (int i = 0; i < NM; ++i) g0[i] = 0.0;
        static_for_dev<1, NM + 1>([&](auto kc) {
            constexpr int K = decltype(kc)::value;
            if (n == K)
                u0 = base_state<K>(A, n, *reinterpret_cast<const int(*)[K]>(&n0[0]),
                                   *reinterpret_cast<const double(*)[K]>(&xu[0]),
                                   *reinterpret_cast<double(*)[K]>(&g0[0]));
        });
    } else {
        u0 = base_state<NM>(A, n, n0, xu, g0);
    }
    if (NM <= 8 && fm == (1u << n) - 1u) {
        // dense box: table-driven walk
        const bool soft = nbout != nullptr && dr->kT > 0.0;
        double e1, e2, Z, sv[NM];
        uint32_t s1;
        const int64_t scored = dense_small<NM>(hs, g0, n, k, dr->kT, soft, e1, e2, s1, Z, sv);
        gap = (e2 - e1 < 1e-9) ? 1 : 0;
#pragma unroll
        for (int i = 0; i < NM; ++i)
            if (i < n) nout[i] = n0[i] + (int)(s1 >> i & 1u);
        if (nbout) {
#pragma unroll
            for (int i = 0; i < NM; ++i)
                if (i < n)
                    nbout[i] = soft ? (double)n0[i] + sv[i] / Z
                                    : (double)(n0[i] + (int)(s1 >> i & 1u));
        }
        return scored;
    }
    // any other set: argmin and runner-up with the y = A 1_s walk
    const int m = __popc(fm);
    const uint64_t pos = free_positions(fm);
    const int steps = 1 << m;
    double y[NM];
    double e1 = INFINITY, e2 = INFINITY;
    uint32_t s1 = 0;
    int64_t scored = 0;
    {
        uint32_t s = 0;
        int pc = 0;
        walk_start<NM>(A, s, y);
        for (int step = 0; step < steps; ++step) {
            if (step) walk_flip<NM>(A, pos, step, s, pc, y);
            if (k < 0 || pc == k) {
                const double e = walk_energy<NM>(g0, y, u0, s);
                ++scored;
                if (better(e, s, e1, s1)) { e2 = e1; e1 = e; s1 = s; }
                else if (e < e2) e2 = e;
            }
        }
    }
    gap = (e2 - e1 < 1e-9) ? 1 : 0;
#pragma unroll
    for (int i = 0; i < NM; ++i)
        if (i < n) nout[i] = n0[i] + (int)(s1 >> i & 1u);
    if (nbout) {
        const double kT = dr->kT;
        if (kT > 0.0) {
            double Z = 0.0, sv[NM];
#pragma unroll
            for (int i = 0; i < NM; ++i) sv[i] = 0.0;
            uint32_t s = 0;
            int pc = 0;
            walk_start<NM>(A, s, y);
            for (int step = 0; step < steps; ++step) {
                if (step) walk_flip<NM>(A, pos, step, s, pc, y);
                if (k < 0 || pc == k) {
                    const double w = exp(-(walk_energy<NM>(g0, y, u0, s) - e1) / kT);
                    Z += w;
#pragma unroll
                    for (int i = 0; i < NM; ++i)
                        if (s >> i & 1u) sv[i] += w;
                }
            }
#pragma unroll
            for (int i = 0; i < NM; ++i)
                if (i < n) nbout[i] = (double)n0[i] + sv[i] / Z;
        } else {
#pragma unroll
            for (int i = 0; i < NM; ++i)
                if (i < n) nbout[i] = (double)(n0[i] + (int)(s1 >> i & 1u));
        }
    }
    return scored;
}

// Up to 8 dots: three waves per SIMD (168 registers, a few spilled) hide
// more of each lane's FP64 chains than two at full register use.
template <int NM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NM <= 8 ? 3 : 1))) void k_batch(const BatchHdr *__restrict__ hdr,
                                              const DiagRec *__restrict__ recs,
                                              const double *__restrict__ mats, int n_diag,
                                              int64_t tiles, const double *__restrict__ V,
                                              int32_t *__restrict__ n_out,
                                              double *__restrict__ nbar,
                                              int64_t *__restrict__ counters)
{
    __shared__ double sA[kMaxDot * kMaxDot];
    __shared__ double sh[256];
    __shared__ int64_t sitem;
    const int lane = threadIdx.x;
    int64_t npix = 0, nqp = 0, nfail = 0, ndbl = 0, ngap = 0, ncand = 0;
    // The work queue is sharded over the kCounterSlots counter lines: slot s
    // hands out items s, s + kCounterSlots, ... (each shard keeps the plan's
    // largest-first order).  A block drains its home slot, then takes what
    // is left in the others, moving on once its count on a shard runs past
    // the end, so no single address sees every block's atomics.
    const int home = blockIdx.x & (kCounterSlots - 1);
    int shard = 0;
    // lane 0: an atomic on the current shard (its raw count; -1 once every
    // shard is exhausted), and the work item such a count stands for (the
    // next shards are tried when it is past the end)
    auto issue = [&]() -> int64_t {
        if (shard >= kCounterSlots) return -1;
        const int sl = (home + shard) & (kCounterSlots - 1);
        return (int64_t)atomicAdd((unsigned long long *)&counters[sl * C_NUM + C_WORK], 1ull);
    };
    auto take = [&](int64_t raw) -> int64_t {
        while (raw >= 0) {
            const int64_t it = (int64_t)((home + shard) & (kCounterSlots - 1)) + kCounterSlots * raw;
            if (it < tiles) return it;
            ++shard;
            raw = issue();
        }
        return tiles;
    };
    // The next item's atomic is issued when an item starts and read when it
    // ends, so its latency hides behind the item's work.  The diagram's A
    // and table stay in LDS while the items come from the same diagram (its
    // items are consecutive in a shard), and the search over the headers
    // runs only when an item leaves the current diagram.
    if (lane == 0) sitem = take(issue());
    int d = -1;
    int64_t d_lo = 0, d_hi = 0;  // items [d_lo, d_hi) belong to diagram d
    BatchHdr h{};
    for (;;) {
        __syncthreads();
        const int64_t item = sitem;
        if (item >= tiles) break;
        int64_t raw = -1;
        if (lane == 0) raw = issue();
        if (item < d_lo || item >= d_hi) {
            // the diagram of this work item: last d with tile0 <= item
            int lo = 0, hi = n_diag - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (hdr[mid].tile0 <= item) lo = mid;
                else hi = mid - 1;
            }
            d = lo;
            h = hdr[d];
            d_lo = h.tile0;
            d_hi = d + 1 < n_diag ? hdr[d + 1].tile0 : tiles;
            const DiagRec *dn = recs + d;
            for (int e = lane; e < kMaxDot * kMaxDot; e += 64) sA[e] = dn->A[e];
            if (NM <= 8)
                for (int e = lane; e < 256; e += 64) sh[e] = dn->hs[e];
            __syncthreads();
        }
        const DiagRec *dr = recs + d;
        const int64_t p = (item - h.tile0) * 64 + lane;
        if (p < h.P) {
            int qp = 0, fail = 0, dbl = 0, gap = 0;
            // the voltages: read, or formed from the diagram's sweep
            const double *Vp = V + h.v_off + p * h.g;
            const double *gv = mats + h.grid_off;
            double va = 0.0, vb = 0.0;
            if (h.nx > 0) {
                const double *sc = gv + 3 * h.g;  // a0, da, a1, b0, db, b1
                va = lin_point(p % h.nx, h.nx, sc[0], sc[1], sc[2]);
                vb = lin_point(p / h.nx, h.ny, sc[3], sc[4], sc[5]);
            }
            auto volt = [&](int j) {
                return h.nx > 0 ? sweep_volt(gv[j], gv[h.g + j], gv[2 * h.g + j], va, vb) : Vp[j];
            };
            ncand += batch_pixel<NM>(dr, sA, sh, h.closed != 0, volt,
                                     n_out + h.out_off + p * h.n,
                                     nbar ? nbar + h.out_off + p * h.n : nullptr, qp, fail, dbl,
                                     gap);
            ++npix;
            nqp += qp;
            nfail += fail;
            ndbl += dbl;
            ngap += gap;
        }
        __syncthreads();  // sA and sitem are rewritten for the next item
        if (lane == 0) sitem = take(raw);
    }
    // wave totals -> counters
    npix = (int64_t)group_sum<6>((double)npix);
    nqp = (int64_t)group_sum<6>((double)nqp);
    nfail = (int64_t)group_sum<6>((double)nfail);
    ndbl = (int64_t)group_sum<6>((double)ndbl);
    ngap = (int64_t)group_sum<6>((double)ngap);
    ncand = (int64_t)group_sum<6>((double)ncand);
    if (lane == 0) {
        block_add_counter(counters, C_PIXELS, npix);
        block_add_counter(counters, C_QP, nqp);
        block_add_counter(counters, C_QP_FAIL, nfail);
        block_add_counter(counters, C_DOUBLED, ndbl);
        block_add_counter(counters, C_GAP_1E9, ngap);
        block_add_counter(counters, C_CANDIDATES, ncand);
    }
}

hipError_t launch_batch(const BatchHdr *hdr, const DiagRec *recs, const double *mats, int n_diag,
                        int64_t tiles, const double *V, int32_t *n_out, double *nbar,
                        int64_t *counters, int max_dot, int blocks, hipStream_t s)
{
    if (blocks < 1) blocks = 1;
    if (max_dot <= 4)
        hipLaunchKernelGGL(k_batch<4>, dim3(blocks), dim3(64), 0, s, hdr, recs, mats, n_diag, tiles, V,
                           n_out, nbar, counters);
    else if (max_dot <= 8)
        hipLaunchKernelGGL(k_batch<8>, dim3(blocks), dim3(64), 0, s, hdr, recs, mats, n_diag, tiles, V,
                           n_out, nbar, counters);
    else
        hipLaunchKernelGGL(k_batch<16>, dim3(blocks), dim3(64), 0, s, hdr, recs, mats, n_diag, tiles, V,
                           n_out, nbar, counters);
    return hipGetLastError();
}

}  // namespace qa
