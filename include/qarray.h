/*
 * qarray.h -- C ABI of the MI355X constant-capacitance ground-state library
 * (libqarray.so, hand-written HIP for gfx950).
 *
 * The problem is the one stated in van Straaten et al., "QArray: a
 * GPU-accelerated constant capacitance model simulator for large quantum dot
 * arrays" (arXiv 2404.04994):
 *
 *   For every pixel p (a vector V_p of gate voltages), with A = C_dd^{-1} and
 *   x_u = C_gd V_p (the open continuous minimum, Sec. 3.1.1), find the dot
 *   charge vector n that minimises the free energy (Sec. 2, Eq. free_energy)
 *       U(n) = 1/2 (n - x_u)^T A (n - x_u)
 *   over integer n >= 0 (open array), additionally with sum(n) = N_hat
 *   (closed array, constraint iii of Sec. 2).  The library implements the
 *   paper's two-stage method (Sec. 3): the constrained continuous minimum x*
 *   (analytic solution of Sec. 3.1.1 / App. C-D, else the QP of Sec. 3.1.2),
 *   then the candidate states around it -- the 2^N floor/ceil box of
 *   Sec. 3.2.1 (threshold t = 1) or the thresholded subset of Sec. 3.2.2
 *   (t < 1, closed arrays double t when no admissible state is left) -- and
 *   finally the argmin (Eq. argmin, T = 0) or the Boltzmann softargmin
 *   (Sec. 4.2, Eq. softargmin, kT > 0) over those candidates.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units: e = 1, so kT is in the energy units of U (Sec. 6).  Charges are
 *   holes as written in Sec. 2; for electrons pass -V (U is invariant under
 *   n -> -n, V -> -V up to a constant).
 * Layout: all matrices are row-major FP64.  V is P x G, one row per pixel.
 *   Outputs are P x N, one row per pixel.
 * Candidate set: f = floor(x*), the candidates are f + b with b in {0,1}^N
 *   (also when x*_i is an exact integer); thresholded dots with
 *   |frac(x*_i) - 1/2| > t/2 are rounded to nearest instead; ties in energy
 *   resolve to the lexicographically smallest n (dot 0 most significant).
 * Memory: every buffer is owned by the caller.  "_dev" arguments are device
 *   pointers on the current HIP device; problem matrices are host pointers
 *   that are read before the call returns.  The library keeps a private
 *   workspace per (device, stream), grown on demand with hipMalloc and freed
 *   by qa_release(); it never keeps caller pointers after returning.
 * Streams: work is enqueued on `hip_stream` (a hipStream_t; NULL = the null
 *   stream) and the call returns without waiting, unless `stats` is non-NULL,
 *   in which case the call waits for the stream to copy the counters back.
 *   Calls on the same stream run in order; concurrent calls on different
 *   streams use different workspaces.
 * Errors: every entry point returns a qa_status; nothing is thrown or
 *   aborted across the ABI.  Validation (FP64, on the host) happens before any
 *   device work: on error nothing is enqueued and no output is written.
 *   qa_last_error() describes the last failure on the calling thread.
 */
#ifndef QARRAY_H
#define QARRAY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QA_MAX_DOT 16  /* largest n_dot the kernels are built for */
#define QA_MAX_GATE 32 /* largest n_gate */

typedef enum {
    QA_OK = 0,
    QA_E_NULL = 1,          /* a required pointer is NULL */
    QA_E_SHAPE = 2,         /* n_dot/n_gate/P out of range */
    QA_E_NOT_SYMMETRIC = 3, /* C_dd not symmetric to 1e-12 relative */
    QA_E_NOT_PD = 4,        /* C_dd not positive definite (App. B) */
    QA_E_RANGE = 5,         /* t not in [0,1], kT < 0 or not finite, N_hat < 0,
                               non-finite matrix entry, bad enum value */
    QA_E_UNSUPPORTED = 6,   /* valid input outside what this build handles */
    QA_E_WORKSPACE = 7,     /* device allocation failed */
    QA_E_DEVICE = 8         /* a HIP call failed (launch, copy, fault) */
} qa_status;

typedef enum { QA_OPEN = 0, QA_CLOSED = 1 } qa_mode;

/* Arithmetic used to score the candidate states.
 *  QA_PREC_FP64   : every candidate energy in FP64 on the vector ALUs.
 *  QA_PREC_FP32   : b^T g on FP32 matrix cores, FP64 re-score of near ties.
 *  QA_PREC_BF16X3 : b^T g on BF16 matrix cores with g split exactly into
 *                   three BF16 parts (FP32 accumulation), FP64 re-score of
 *                   near ties.
 *  QA_PREC_BF16X2 : as BF16X3 with two parts (g rounded to 16 significant
 *                   bits), FP64 re-score of near ties.
 * The integer result is the same for all four: the near-tie re-score
 * replaces the approximate argmin by the FP64 one whenever the approximate
 * runner-up lies within the certified error band.  The matrix-core forms are
 * used at T = 0 with n_dot >= 9: for open arrays over the dense box (t = 1)
 * or the thresholded sub-box of each pixel (t < 1, Sec. 3.2.2), for closed
 * arrays over the subsets of the free dots that raise the charge to N_hat
 * (Sec. 3.2); elsewhere the FP64 form runs regardless of the request. */
typedef enum {
    QA_PREC_FP64 = 0,
    QA_PREC_FP32 = 1,
    QA_PREC_BF16X3 = 2,
    QA_PREC_BF16X2 = 3
} qa_precision;

typedef struct {
    int32_t n_dot;       /* N, 1..QA_MAX_DOT */
    int32_t n_gate;      /* G, 1..QA_MAX_GATE */
    const double *cdd;   /* host, N x N Maxwell dot-dot block (Sec. 2):
                            diagonal = total capacitance, off-diagonal =
                            minus the coupling; symmetric positive definite */
    const double *cgd;   /* host, N x G gate-dot coupling (x_u = C_gd V) */
    int32_t mode;        /* qa_mode */
    int32_t n_charge;    /* N_hat >= 0 for QA_CLOSED, ignored for QA_OPEN */
    double kT;           /* >= 0; used by qa_soft_charge* only */
    double threshold;    /* t in [0,1]; 1 = the default 2^N box */
    int32_t precision;   /* qa_precision */
    int32_t flags;       /* QA_FLAG_* bits, 0 for the defaults */
} qa_problem;

/* qa_problem.flags.
 *  QA_FLAG_EXHAUSTIVE : the matrix-core scorer computes the energy of every
 *      state of the candidate set.  By default the candidate sets of N >= 13
 *      dots (the dense box, the thresholded sub-boxes and the closed subsets)
 *      are searched in bound order: a lower bound of the 256 states that
 *      share a high part (the low part minimised over the reals, whose value
 *      is the Schur complement of the low block of C_dd^{-1}, i.e. the inverse
 *      of the high block of C_dd; closed arrays with the low part's sum fixed)
 *      discards high parts that cannot hold the argmin or a state of the
 *      near-tie band.  Both give the argmin over the whole candidate set
 *      (Sec. 3.2); qa_stats.scored tells how many energies were computed. */
#define QA_FLAG_EXHAUSTIVE 1

typedef struct {
    int64_t pixels;            /* pixels processed */
    int64_t qp_pixels;         /* analytic minimum infeasible -> QP solved */
    int64_t qp_failures;       /* QP did not reach a KKT point (should be 0) */
    int64_t doubled_pixels;    /* closed thresholded pixels whose t doubled */
    int64_t near_tie_pixels;   /* approximate scoring flagged -> FP64 re-score */
    int64_t fp64_gap_below_1e9;/* pixels whose FP64 best/runner-up gap < 1e-9 */
    int64_t candidates;        /* states of the candidate sets (Sec. 3.2) */
    int64_t scored;            /* states whose energy the scorer computed */
} qa_stats;

/* Ground state at T = 0 (Sec. 3, Eq. argmin) of P pixels.
 *   V_dev     : device, P x G FP64 gate voltages.
 *   P         : number of pixels, >= 0 (0 is a no-op).
 *   n_out_dev : device, P x N int32, receives n* per pixel.
 *   stats     : host, may be NULL (then the call does not wait). */
qa_status qa_ground_state(const qa_problem *prob, const double *V_dev, int64_t P,
                          int32_t *n_out_dev, qa_stats *stats, void *hip_stream);

/* An affine two-dimensional sweep of the gate voltages: the raster scans of
 * Sec. 5 (the gate-voltage composer's two-gate and do2d sweeps), and sweeps
 * of two virtual gates (Fig. 1(b); Sec. 5.3, App. I: e1, e2 the columns of
 * the virtual-gate matrix).  nx x ny pixels, pixel p = j * nx + i (the row is
 * the second swept coordinate), with
 *     a_i = linspace(a0, a1, nx)[i],  b_j = linspace(b0, b1, ny)[j],
 *     V(i, j) = (v0 + a_i e1) + b_j e2,
 * each operation rounded to FP64 on its own (no fused multiply-add) and a_i
 * formed as numpy's linspace forms it (i * step + a0, the last point a1):
 * the results are bitwise those of the explicit voltages numpy computes
 * from the same description.  The voltages are formed inside the kernels
 * and never stored.
 *   v0, e1, e2 : host, n_gate doubles each, read before the call returns.
 *   nx, ny     : >= 1, nx * ny < 2^31 (QA_E_SHAPE).  Non-finite values:
 *                QA_E_RANGE; NULL pointers: QA_E_NULL. */
typedef struct {
    const double *v0, *e1, *e2;
    double a0, a1;   /* first swept coordinate (columns of the raster) */
    double b0, b1;   /* second swept coordinate (rows) */
    int32_t nx, ny;
} qa_grid;

/* qa_ground_state over a sweep: P = nx * ny pixels, n_out_dev P x N int32
 * (row-major in p).  Launches directly (never as a graph replay). */
qa_status qa_ground_state_grid(const qa_problem *prob, const qa_grid *grid, int32_t *n_out_dev,
                               qa_stats *stats, void *hip_stream);

/* qa_ground_state for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same problem, inputs, output and result as qa_ground_state,
 * but the call allocates nothing (no hipMalloc, hipHostMalloc or hipFree,
 * no host heap) and issues no copy: the problem's inputs travel as kernel
 * arguments, and every intermediate (diagram record, per-pixel records,
 * counters) lives in a static device array of about 15 MB that each GPU the
 * library runs on holds until the process ends.
 *   P : 0..QA_NOALLOC_MAX_PIXELS; larger P returns QA_E_SHAPE (nothing is
 *       enqueued).  Split larger sweeps into several calls.
 * No statistics and no stage timing.  Every call on one GPU uses that GPU's
 * one scratch array and leaves the last call's contents in it: calls that
 * overlap on one GPU (different streams, or different threads without
 * ordering) race and give wrong results, so order them on one stream.
 * The call enqueues on hip_stream and returns without waiting. */
#define QA_NOALLOC_MAX_PIXELS 65536
qa_status qa_ground_state_noalloc(const qa_problem *prob, const double *V_dev, int64_t P,
                                  int32_t *n_out_dev, void *hip_stream);

/* Constrained continuous minimum of every pixel (Sec. 3.1): x* = the
 * analytic minimum (Sec. 3.1.1; App. C for open, App. D for closed arrays)
 * when it is non-negative, otherwise the exact solution of the QP of
 * Sec. 3.1.2 (x >= 0, and sum x = N_hat for closed arrays) in FP64.
 *   x_out_dev     : device, P x N FP64, receives x*.
 *   flags_out_dev : device, P int32, or NULL; bit0 = the QP was solved,
 *                   bit1 = the QP iteration did not settle (x* is then its
 *                   last iterate), bit2 = the threshold doubled when the
 *                   candidate set was formed (closed, t < 1).
 * This is the first stage of qa_ground_state and qa_soft_charge, exposed so
 * that the continuous minimum can be checked and reused on its own. */
qa_status qa_continuous_min(const qa_problem *prob, const double *V_dev, int64_t P,
                            double *x_out_dev, int32_t *flags_out_dev, qa_stats *stats,
                            void *hip_stream);

/* Thermal softargmin (Sec. 4.2, Eq. softargmin) over the candidate set of
 * each pixel, in FP64.
 *   nbar_out_dev : device, P x N FP64, receives <n> per pixel.
 *   saved_dev    : device, qa_saved_bytes(P, N) bytes, or NULL; receives
 *                  what qa_soft_charge_backward needs (candidate set and
 *                  normaliser per pixel; the energies are not stored). */
qa_status qa_soft_charge(const qa_problem *prob, const double *V_dev, int64_t P,
                         double *nbar_out_dev, void *saved_dev, qa_stats *stats,
                         void *hip_stream);

/* Adjoint of qa_soft_charge.  Given grad_nbar = dL/d<n> (device, P x N
 * FP64) and the saved buffer of the forward call with the same problem and
 * V, writes
 *   grad_cdd_dev : device, N x N FP64, dL/dC_dd (every entry independent),
 *   grad_cgd_dev : device, N x G FP64, dL/dC_gd,
 *   grad_V_dev   : device, P x G FP64, dL/dV, or NULL to skip.
 * The candidate set is piecewise constant in the inputs, so only the
 * energies carry gradient; they are recomputed, not read back.  This is not
 * in the paper (which notes that the discrete model defeats autograd,
 * Sec. 6); it differentiates the softargmin exactly.  n_dot <= 12 (each
 * block keeps one FP64 sum per candidate state, 2^N of them, in its local
 * memory); larger problems return QA_E_UNSUPPORTED. */
qa_status qa_soft_charge_backward(const qa_problem *prob, const double *V_dev, int64_t P,
                                  const double *grad_nbar_dev, const void *saved_dev,
                                  double *grad_cdd_dev, double *grad_cgd_dev,
                                  double *grad_V_dev, void *hip_stream);

/* qa_soft_charge over a sweep (qa_grid): P = nx * ny pixels; nbar_out_dev
 * P x N FP64 and saved_dev qa_saved_bytes(P, N) as for qa_soft_charge. */
qa_status qa_soft_charge_grid(const qa_problem *prob, const qa_grid *grid, double *nbar_out_dev,
                              void *saved_dev, qa_stats *stats, void *hip_stream);

/* qa_soft_charge_backward over a sweep: the saved buffer of a
 * qa_soft_charge_grid call with the same problem and sweep.  grad_V_dev
 * (P x G FP64, or NULL) receives dL/dV of every pixel's voltages (the
 * sweep's derivatives follow from them by the chain rule). */
qa_status qa_soft_charge_backward_grid(const qa_problem *prob, const qa_grid *grid,
                                       const double *grad_nbar_dev, const void *saved_dev,
                                       double *grad_cdd_dev, double *grad_cgd_dev,
                                       double *grad_V_dev, void *hip_stream);

/* Bytes of the saved buffer for P pixels of an N-dot problem. */
size_t qa_saved_bytes(int64_t P, int32_t n_dot);

/* A batch of independent diagrams (the dataset-generation use of Sec. 1)
 * in one launch sequence (prologue of every diagram, one persistent
 * kernel over all pixels).  Diagram d has its own problem
 * probs[d] (N_d, G_d, mode, N_hat, kT, t; precision is ignored, every
 * energy is FP64) and its own P_d pixels.
 *   V_dev       : device FP64; diagram d's voltages are the P_d x G_d
 *                 row-major block starting at element v_offsets[d].
 *   v_offsets   : host, n_diag entries (elements, not bytes).
 *   pix_counts  : host, n_diag entries, P_d >= 0.
 *   out_offsets : host, n_diag entries; diagram d's outputs are the
 *                 P_d x N_d row-major block starting at element
 *                 out_offsets[d] of n_out_dev and of nbar_out_dev.
 *   n_out_dev   : device int32; the T = 0 ground state (argmin over the
 *                 candidate set) of every pixel of every diagram.
 *   nbar_out_dev: device FP64 or NULL; the softargmin of diagrams with
 *                 kT > 0 (for kT = 0 diagrams, n* converted to FP64).
 *   stats       : host or NULL; summed over the batch (waits for the stream).
 * Every problem is validated as for qa_ground_state before any device work;
 * blocks must lie inside the caller's buffers (not checked: device sizes
 * are unknown to the library).  Returns QA_E_SHAPE for n_diag < 0 or a
 * negative offset or count. */
qa_status qa_ground_state_batched(const qa_problem *probs, int32_t n_diag, const double *V_dev,
                                  const int64_t *v_offsets, const int64_t *pix_counts,
                                  const int64_t *out_offsets, int32_t *n_out_dev,
                                  double *nbar_out_dev, qa_stats *stats, void *hip_stream);

/* qa_ground_state_batched over sweeps: diagram d is the sweep grids[d]
 * (P_d = nx * ny pixels, validated as for qa_ground_state_grid); its
 * outputs are the P_d x N_d block at element out_offsets[d], as for the
 * explicit-voltage form.  The sweeps are uploaded with the matrices and the
 * voltages are formed inside the kernel. */
qa_status qa_ground_state_batched_grid(const qa_problem *probs, int32_t n_diag,
                                       const qa_grid *grids, const int64_t *out_offsets,
                                       int32_t *n_out_dev, double *nbar_out_dev, qa_stats *stats,
                                       void *hip_stream);

/* Stage timing (diagnostics).  While enabled, every ground-state call on a
 * stream records HIP events on that stream around its stages:
 *   stage 0: prologue, continuous minimum and candidate setup,
 *   stage 1: candidate scoring (the matrix-core or FP64 scorer, including
 *            the FP64 re-score of near ties),
 *   stage 2: work after the scorer (none in this build: 0).
 * qa_timing_reset() forgets earlier records of the stream;
 * qa_timing_sum() waits for the stream and writes the summed milliseconds
 * of each stage (ms_out[3]) over the calls recorded since the reset and the
 * number of calls (at most 4096 are kept).  Off by default. */
void qa_timing_enable(int on);

/* Launch mode.  Off (the default; QA_GRAPHS=1 in the environment starts
 * with it on), every kernel is launched directly on the caller's stream.
 * On, each call replays a hipGraph captured for its launch shape and
 * buffers (captured on first use; the per-call inputs are copied before the
 * replay).  Results are identical.  A call here is two or three kernels, and
 * on ROCm 7 a graph launch costs more host and device time than launching
 * them directly, so graphs are opt-in.  Stage timing always launches
 * directly. */
void qa_graphs_enable(int on);
void qa_timing_reset(void *hip_stream);
qa_status qa_timing_sum(void *hip_stream, double *ms_out, int64_t *calls_out);

/* Kernel timing (diagnostics).  Runs qa_ground_state's device work once
 * (n_out_dev receives the ground state), then on hip_stream: an event,
 * `reps` back-to-back launches of the setup kernel (prologue, continuous
 * minimum, candidate setup), an event, `reps` (setup, scorer) pairs, an
 * event.  Waits, and writes the mean milliseconds per launch: ms_out[0] the
 * setup kernel (first interval / reps), ms_out[1] the T = 0 scorer the
 * problem selects (second interval less the first, / reps), i.e. the
 * scorer as it runs in a call, right after the setup that wrote its inputs.
 * No events separate the launches, so each mean includes the dispatch gap
 * between back-to-back launches.  reps in [1, 100000]; P >= 1. */
qa_status qa_time_kernels(const qa_problem *prob, const double *V_dev, int64_t P,
                          int32_t *n_out_dev, int32_t reps, double *ms_out, void *hip_stream);

/* Charge sensors (Sec. 5.1).  The problem's last n_sensor dots are sensor
 * dots (prob: the whole system, n_dot = N_array + n_sensor).  The array
 * dots' charges are given: their ground state or softargmin computed by the
 * caller with the array block of C_dd (first N_array rows and columns) and
 * of C_gd (first N_array rows, every gate), i.e. the sensors left out but
 * the sensor gates' cross-talk kept.  Per pixel, with those charges fixed,
 * the sensors take the charges that minimise the electrostatic energy of
 * the whole system (the floor/ceil box around their continuous minimum,
 * clipped at zero; exact for one sensor), their potentials follow the
 * potential equation v = C_dd^{-1} (n - C_gd V), and the response of sensor
 * s is P(v_s + A_ss/2) + P(-v_s + A_ss/2) (A = C_dd^{-1}; the second term
 * only when the sensor is occupied): the energy to add or to remove one
 * carrier, each zero at a Coulomb-peak condition, under the peak profile P
 * (Lorentzian 1/(1 + (x/gamma)^2) or Gaussian exp(-x^2/(2 gamma^2)), peak 1).
 * Noise is added from draws the caller passes (noise_dev, device FP64):
 *   [0, P*S)           white: standard-normal, pixel-major (p * S + s)
 *   then, per sensor s and octave k < pink_octaves, ceil(P / 2^k)
 *                      standard-normal draws: 1/f noise by the
 *                      Voss-McCartney sum over the octaves / sqrt(K)
 *   then [.., + P*S)   uniform [0, 1) draws: telegraph jumps, the state
 *                      flips where a draw is below jump_rate (pixel order)
 * qa_sensor_noise_len(P, S, K) gives the total; noise_dev may be NULL when
 * white, pink and jump are all 0.
 *   n_array_dev     : device, P x N_array int32 (ground state), or NULL and
 *   nbar_array_dev  : device, P x N_array FP64 (softargmin).
 *   signal_dev      : device, P x n_sensor FP64. */
typedef enum { QA_SENSOR_LORENTZIAN = 0, QA_SENSOR_GAUSSIAN = 1 } qa_sensor_shape;
typedef struct {
    int32_t n_sensor;      /* 1..4 */
    int32_t shape;         /* qa_sensor_shape */
    double gamma;          /* peak width, > 0 (energy units of U) */
    double white;          /* white-noise amplitude, >= 0 */
    double pink;           /* 1/f-noise amplitude, >= 0 */
    int32_t pink_octaves;  /* K, 1..40 when pink > 0 */
    int32_t reserved;
    double jump;           /* telegraph-jump amplitude, >= 0 */
    double jump_rate;      /* flip probability per sample, [0, 1] */
} qa_sensor;

size_t qa_sensor_noise_len(int64_t P, int32_t n_sensor, int32_t pink_octaves);

qa_status qa_sensor_response(const qa_problem *prob, const qa_sensor *sensor, const double *V_dev,
                             int64_t P, const int32_t *n_array_dev, const double *nbar_array_dev,
                             const double *noise_dev, double *signal_dev, void *hip_stream);

/* Optimal gate voltages (Sec. 5.3, App. H): the V that minimises the free
 * energy of the fixed dot charges q, i.e. the least-squares solution of
 * R q = R C_gd V with R^T R = C_dd^{-1} (Cholesky), V = (R C_gd)^+ R q
 * (Moore-Penrose pseudo-inverse: exact when C_gd is square and invertible,
 * minimum-norm when there are more gates than dots, least squares when
 * fewer).  Host FP64; no device work.
 *   q     : host, N doubles (charges in units of e, holes positive).
 *   v_out : host, G doubles.
 * Uses n_dot, n_gate, cdd, cgd of prob (validated as for every entry point;
 * mode, kT, threshold and precision are ignored beyond validation). */
qa_status qa_optimal_gate_voltages(const qa_problem *prob, const double *q, double *v_out);

/* Virtual-gate matrix (Sec. 5.3, App. I): alpha = (C_dd^{-1} C_gd)^+, G x N
 * row-major into alpha_out (host).  The dot potentials move by
 * C_dd^{-1} C_gd dV (Eq. for the potential), so column i of alpha is the
 * gate-voltage change that moves dot i's potential by one unit and leaves
 * the others (exactly when C_dd^{-1} C_gd has full row rank, otherwise in
 * the least-squares sense with minimum norm).  Host FP64; no device work.
 * The paper's transposed product C_gd C_dd^{-1} is defined only for square
 * C_gd; this form is its general reading. */
qa_status qa_virtual_gate_matrix(const qa_problem *prob, double *alpha_out);

/* Description of the last error on the calling thread ("" if none). */
const char *qa_last_error(void);

/* Free the library workspace of `hip_stream` on the current device; call
 * after the stream's work has finished.  Safe to call more than once. */
void qa_release(void *hip_stream);

/* Library version string. */
const char *qa_version(void);

#ifdef __cplusplus
}
#endif
#endif /* QARRAY_H */
