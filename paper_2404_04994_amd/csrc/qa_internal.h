// qa_internal.h -- device-side records and launch wrappers of libqarray.
//
// Layout in HBM (one call = one diagram unless batched):
//   DiagRec  : per diagram, written by the prologue kernel (k_prep):
//              C_dd, A = C_dd^{-1} (FP64, symmetric), C_gd, C_dd 1, sums,
//              and the FP32 / split-BF16 tables the matrix-core scorer reads.
//   PixRec   : per pixel, written by the setup kernel (k_setup):
//              the candidate description (n0, free mask, k) and the FP64
//              gradient g0 = A (n0 - x_u) and energy U(n0) at the base state.
//   SavedRec : per pixel, the softargmin state the adjoint needs (the
//              caller-owned "saved" buffer of qa_soft_charge): candidate
//              set, smallest energy, normaliser and mean offset; no energies.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace qa {

constexpr int kMaxDot = 16;
constexpr int kMaxGate = 32;
constexpr int kWave = 64;

// counters (int64) kept in the workspace, mirrored into qa_stats.  Atomics
// on one address from every block serialise at the memory side, so the
// statistics are spread over kCounterSlots cache lines ([slot][C_NUM], a
// block adds to slot blockIdx mod kCounterSlots) and summed by the host.
// C_WORK is the cursor of one shard of the batched kernel's work queue in
// every slot.
constexpr int kCounterSlots = 64;
enum Counter {
    C_PIXELS = 0,
    C_QP = 1,
    C_QP_FAIL = 2,
    C_DOUBLED = 3,
    C_NEAR_TIE = 4,
    C_GAP_1E9 = 5,
    C_CANDIDATES = 6,
    C_SCORED = 7,       // states whose approximate energy a scorer computed
    C_UNUSED8 = 8,
    C_UNUSED9 = 9,
    C_WORK = 10,        // work-queue shard cursor of the batched kernel
    C_NUM = 16
};
constexpr int kCounterWords = kCounterSlots * C_NUM;

// add a block's partial count to its counter slot
__device__ __forceinline__ void block_add_counter(int64_t *counters, int which, int64_t v)
{
    if (v)
        atomicAdd((unsigned long long *)&counters[(blockIdx.x & (kCounterSlots - 1)) * C_NUM + which],
                  (unsigned long long)v);
}

// Cross-lane all-reductions without LDS: DPP within each 16-lane row
// (exchange with lane ^ 1, lane ^ 2, then the mirror images within 8 and 16
// lanes, each an involution, so after four steps every lane of a row holds
// the row's result), then the row swaps of gfx950 for 16 and 32 lanes.
// Every pattern used here (quad permutations, row mirrors, row broadcasts) has
// a valid source lane for every lane, so the move needs no "old" value: the
// plain DPP move, not the update form, whose old operand costs a v_mov per
// use.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dppf(float x)
{
    return __uint_as_float(dpp32<CTRL>(__float_as_uint(x)));
}
template <int CTRL>
__device__ __forceinline__ double dppd(double x)
{
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint64_t r = (uint64_t)dpp32<CTRL>((uint32_t)u) |
                       ((uint64_t)dpp32<CTRL>((uint32_t)(u >> 32)) << 32);
    return __longlong_as_double((long long)r);
}
// 1/a for the pivots of the eliminations: the hardware estimate refined by
// two Newton steps r <- r + r (1 - a r) (each squares the relative error),
// within an ulp of the rounded quotient for the normal, finite pivots of a
// positive definite elimination; five dependent operations instead of the
// ten of the correctly rounded division.
__device__ __forceinline__ double recip_nr(double a)
{
    double r = __builtin_amdgcn_rcp(a);
    double e = fma(-a, r, 1.0);
    r = fma(r, e, r);
    e = fma(-a, r, 1.0);
    return fma(r, e, r);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
// lane i of every 16-lane row to the whole row
constexpr int kDppRowBcast0 = 0x150;
__device__ __forceinline__ float row_min(float x)
{
    x = fminf(x, dppf<kDppXor1>(x));
    x = fminf(x, dppf<kDppXor2>(x));
    x = fminf(x, dppf<kDppHalfMirror>(x));
    return fminf(x, dppf<kDppMirror>(x));
}
__device__ __forceinline__ double row_sum(double x)
{
    x += dppd<kDppXor1>(x);
    x += dppd<kDppXor2>(x);
    x += dppd<kDppHalfMirror>(x);
    return x + dppd<kDppMirror>(x);
}
// minimum over the four rows of a value that is uniform within each row
__device__ __forceinline__ float rows_min(float x)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = fminf(__uint_as_float(r[0]), __uint_as_float(r[1]));
    const auto t = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return fminf(__uint_as_float(t[0]), __uint_as_float(t[1]));
}
__device__ __forceinline__ float wave_min(float x) { return rows_min(row_min(x)); }
// sum over the 64 lanes (every lane gets it): the row sums, then the row swaps
__device__ __forceinline__ double wave_sum(double x)
{
    x = row_sum(x);
    auto swap_add = [&](auto swap) {
        const uint64_t u = (uint64_t)__double_as_longlong(x);
        const auto lo = swap((uint32_t)u), hi = swap((uint32_t)(u >> 32));
        const double a = __longlong_as_double((long long)((uint64_t)lo[0] | ((uint64_t)hi[0] << 32)));
        const double b = __longlong_as_double((long long)((uint64_t)lo[1] | ((uint64_t)hi[1] << 32)));
        x = a + b;
    };
    swap_add([](uint32_t v) { return __builtin_amdgcn_permlane16_swap(v, v, false, false); });
    swap_add([](uint32_t v) { return __builtin_amdgcn_permlane32_swap(v, v, false, false); });
    return x;
}

struct alignas(16) DiagRec {
    // inputs (written by the host, or by k_prep_batch): everything up to Cgd
    int32_t n, g, closed, nhat;
    double kT, t;
    int32_t prec, pad0;
    double Cdd[kMaxDot * kMaxDot];
    double Cgd[kMaxDot * kMaxGate];
    // computed by the prologue
    double one_c;                 // 1^T C_dd 1
    double c[kMaxDot];            // C_dd 1
    double A[kMaxDot * kMaxDot];  // C_dd^{-1}
    // matrix-core tables (dense box, n >= 9): low part = dots 0..7,
    // high part = dots 8..n-1; see qa_mfma.hip
    float T1[16][8];              // A_LH b_hi for the 4 row bits of the high index
    float T2[16][8];              // A_LH b_hi for the next 4 bits of the high index
    float Hhi[256];               // 1/2 b_hi^T A_HH b_hi
    float hlo[256];               // 1/2 b_lo^T A_LL b_lo
    float sumabs;                 // sum |A_ij| / 2, bound used by the error band
    float pad1[3];
    double hs[256];               // n <= 8: 1/2 s^T A s for every s in {0,1}^n
    // FP64 copies of the matrix-core tables (the near-tie re-score)
    double T1d[16][8], T2d[16][8];
    double Hhid[256], hlod[256];
    // bound-ordered search (N >= 9): with S = (C_dd,HH)^{-1}, the Schur
    // complement of the low block in A, Hs = 1/2 b_hi^T S b_hi (1e30 past
    // 2^(N-8))
    float Hs[256];
    float sabsS;                  // sum |S_ij| / 2
    // closed arrays: the low part's sum is fixed, which adds
    // (m - mu - w^T b_hi)^2 / (2 gamma) to the bound (m = k - popc(b_hi)),
    // w = S C_HL 1, gamma = 1^T A_LL^{-1} 1
    float wB[8];
    float inv2g;                  // 1 / (2 gamma)
    float pad2[2];
};

// bytes of a DiagRec the host uploads (the inputs)
constexpr size_t kDiagInputBytes = offsetof(DiagRec, one_c);

struct alignas(8) PixRec {
    double g0[kMaxDot];   // A (n0 - x_u)
    double u0;            // U(n0)
    int16_t n0[kMaxDot];  // base state of the candidate set
    uint32_t free;        // dots that take both roundings
    int32_t k;            // closed: number of raised free dots; -1 open
    int32_t flags;        // bit0 QP path, bit1 QP failure, bit2 threshold doubled
    uint32_t guess;       // a state of the candidate set: the free dots whose x* rounds up,
                          // then the best single flip of a free dot if it lowers the energy
                          // (closed: the k free dots with the largest fractional parts)
    // lower bound of the states of a high part b_hi (N >= 13, open):
    // K + b_hi^T s + 1/2 b_hi^T S b_hi, s = S (n0 - x_u)_hi
    float s[8];
    float K;
    float mu;             // closed: -1^T A_LL^{-1} g_lo (the low sum of the free minimiser)
    float eg;             // N = 16 lanes: U(n0 + guess) - U(n0), from FP64
};

struct alignas(8) SavedRec {
    double emin;          // smallest candidate energy
    double Z;             // sum exp(-(E - emin)/kT) (>= 1)
    double nb[kMaxDot];   // <n> - n0 = sum_s pi_s 1_s (zero beyond n)
    int16_t n0[kMaxDot];
    uint32_t free;
    int32_t k;
};

// one diagram of a ragged batch, as uploaded by the host (work order)
struct alignas(8) BatchHdr {
    int32_t n, g, closed, nhat;
    double kT, t;
    int64_t v_off;    // element offset of the diagram's P x G voltages
    int64_t out_off;  // element offset of its P x N outputs
    int64_t P;        // pixels
    int64_t mat_off;  // offset of C_dd (n x n) then C_gd (n x g) in the matrix buffer
    int64_t tile0;    // first 64-pixel work item of the diagram
    // swept diagrams (nx > 0): the voltages are formed from the sweep at
    // grid_off in the matrix buffer: v0, e1, e2 (g each), then a0, da, a1,
    // b0, db, b1 (see VGrid); P = nx * ny
    int64_t grid_off;
    int32_t nx, ny;
};

// An affine sweep of the gate voltages over a raster of nx x ny pixels,
// pixel p = j nx + i:  V(i, j) = (v0 + a_i e1) + b_j e2 with a_i = i da + a0
// (the last a_i is a1 itself) and b_j alike.  These are the values that
// numpy's linspace and broadcast arithmetic give, rounded the same way (no
// fused multiply-add), so a sweep and the explicit voltages it describes
// give bitwise identical results.  on = 0: explicit voltages instead.
struct VGrid {
    double v0[kMaxGate], e1[kMaxGate], e2[kMaxGate];
    double a0, da, a1, b0, db, b1;
    int64_t nx, ny;
    int32_t on, pad;
};

// point i of num equally spaced points from start to stop (step = (stop -
// start) / (num - 1), 0 for one point), as numpy's linspace forms it
// (contraction into fused multiply-adds is off in both: each product and
// sum is rounded on its own)
__device__ __forceinline__ double lin_point(int64_t i, int64_t num, double start, double step,
                                            double stop)
{
#pragma clang fp contract(off)
    const double t = (double)i * step;
    return (num > 1 && i == num - 1) ? stop : t + start;
}
// v0_k + a e1_k + b e2_k, each operation rounded on its own
__device__ __forceinline__ double sweep_volt(double v0, double e1, double e2, double a, double b)
{
#pragma clang fp contract(off)
    const double s = v0 + a * e1;
    return s + b * e2;
}
// the sweep coordinates (a, b) of pixel p
__device__ __forceinline__ void grid_ab(const VGrid &G, int64_t p, double &a, double &b)
{
    a = lin_point(p % G.nx, G.nx, G.a0, G.da, G.a1);
    b = lin_point(p / G.nx, G.ny, G.b0, G.db, G.b1);
}
// gate k's voltage at sweep coordinates (a, b)
__device__ __forceinline__ double grid_v(const VGrid &G, int k, double a, double b)
{
    return sweep_volt(G.v0[k], G.e1[k], G.e2[k], a, b);
}

// The inputs of a DiagRec carried in a kernel's arguments (no host staging
// buffer and no copy call): part 0 writes the header and C_dd, part 1 rows
// [row0, row1) of C_gd; entries past the problem's n x n and n x g are
// written as zeros, so the record's padding is the same whatever an earlier
// call left there.  A chunk holds at most kChunkDoubles matrix entries.
constexpr int kChunkDoubles = 256;
struct InputChunk {
    int32_t n, g, closed, nhat;
    double kT, t;
    int32_t prec;
    int32_t part;        // 0: header and C_dd; 1: C_gd rows [row0, row1)
    int32_t row0, row1;  // part 1: rows of the padded C_gd written by this chunk
    double v[kChunkDoubles];  // part 0: C_dd, n x n; part 1: rows row0.. of C_gd, each g long
};

// the setup kernel: one wave for the prologue, seven for the pixels
constexpr int kSetupPixThreads = 7 * kWave;
// its grid is largest for 16-lane pixel groups
constexpr int64_t setup_blocks_max(int64_t P)
{
    return P < 1 ? 1 : (P * kMaxDot + kSetupPixThreads - 1) / kSetupPixThreads;
}

// -------------------------------------------------------------------------
// launch wrappers (qa_kernels.hip); all enqueue on `s` and return the HIP
// error of the launch.
// -------------------------------------------------------------------------
hipError_t launch_zero_i64(int64_t *p, int n, hipStream_t s);
// one chunk of a diagram's inputs into dr
hipError_t launch_put_inputs(DiagRec *dr, const InputChunk &c, hipStream_t s);
// prologue of n_diag diagrams; also zeroes the kCounterWords counters and
// the nzero doubles at zero when given
hipError_t launch_prep(DiagRec *dr, int n_diag, int64_t *counters, hipStream_t s,
                       double *zero = nullptr, int64_t nzero = 0);
// prologue (every block; block 0 also stores A and the tables into dr and
// clears the kCounterWords counters) and setup of every pixel; the per-block
// counts {pixels, QP, doubled, QP failures} go to bstats[4 * block] for
// setup_blocks(P, n_dot) blocks; x_out (P x N) / flags_out (P) are optional
// copies of x*; grid, when given and on, replaces the voltages V.  P >= 1.
int64_t setup_blocks(int64_t P, int n_dot);
hipError_t launch_setup(DiagRec *dr, const double *V, int64_t P, PixRec *pr, int64_t *counters,
                        int32_t *bstats, int n_dot, bool closed, hipStream_t s,
                        double *x_out = nullptr, int32_t *flags_out = nullptr,
                        const VGrid *grid = nullptr);
// T = 0 argmin in FP64 over the candidate set of every pixel
hipError_t launch_score_fp64(const DiagRec *dr, const PixRec *pr, int64_t P, int32_t *n_out,
                             int64_t *counters, int n_dot, hipStream_t s);
// the same in the table form (n_dot <= 8; the whole-box table from the setup)
hipError_t launch_score_tab(const DiagRec *dr, const PixRec *pr, int64_t P, int32_t *n_out,
                            int64_t *counters, int n_dot, hipStream_t s);
// matrix-core scorer at T = 0; mode 0: the dense box, 1: the sub-box of each
// pixel's free dots (thresholded), 2: closed arrays (subsets of the free
// dots with k raised); near ties re-scored in FP64 inside the kernel.  For
// N >= 13 dots the candidate sets are searched in bound order unless exhaustive.
hipError_t launch_score_mfma(const DiagRec *dr, const PixRec *pr, int64_t P, int prec, int mode,
                             bool exhaustive, int32_t *n_out, int64_t *counters, int n_dot,
                             hipStream_t s);
hipError_t launch_soft_fwd(const DiagRec *dr, const PixRec *pr, int64_t P, double *nbar,
                           SavedRec *saved, int64_t *counters, int n_dot, hipStream_t s);
// adjoint partial sums: kBwdReplicas copies of (dL/dA, kMaxDot^2; dL/dC_gd,
// kMaxDot x kMaxGate), block b adding into copy b mod kBwdReplicas, so that
// fewer blocks contend for one address; zero on entry, and left zero by the
// final kernel, which adds the copies up
constexpr int kBwdReplicas = 8;
constexpr int kBwdAccWords = kMaxDot * kMaxDot + kMaxDot * kMaxGate;
hipError_t launch_soft_bwd(const DiagRec *dr, const double *V, int64_t P,
                           const double *gbar, const SavedRec *saved, double *acc,
                           double *gradV, int n_dot, hipStream_t s, const VGrid *grid = nullptr);
hipError_t launch_soft_bwd_final(const DiagRec *dr, double *acc, double *grad_cdd,
                                 double *grad_cgd, hipStream_t s);
// charge-sensor response (qa_sensor.hip): the last n_sensor dots of dr are
// sensors; array charges from n_int or n_dbl (P x (n - n_sensor)); noise
// draws optional (NULL: none); signal P x n_sensor
hipError_t launch_sensor(const DiagRec *dr, int n_sensor, int shape, double gamma, const double *V,
                         int64_t P, const int32_t *n_int, const double *n_dbl,
                         const double *white_draws, double white, const double *pink_draws,
                         double pink, int octaves, double *signal, hipStream_t s);
hipError_t launch_sensor_jumps(int64_t P, int n_sensor, const double *u, double rate, double amp,
                               double *signal, hipStream_t s);
// ragged batch (qa_batch.hip): prologue of every diagram, then one persistent
// kernel over all 64-pixel work items
hipError_t launch_prep_batch(const BatchHdr *hdr, const double *mats, DiagRec *recs, int n_diag,
                             hipStream_t s);
hipError_t launch_batch(const BatchHdr *hdr, const DiagRec *recs, const double *mats, int n_diag,
                        int64_t tiles, const double *V, int32_t *n_out, double *nbar,
                        int64_t *counters, int max_dot, int blocks, hipStream_t s);

}  // namespace qa
