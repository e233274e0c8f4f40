// qa_api.hip -- host side of the C ABI declared in include/qarray.h:
// validation (FP64, before any device work), the per-(device, stream)
// workspace, and the launch sequence of the ground-state path.
#include "../../include/qarray.h"
#include "qa_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <array>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

using namespace qa;

namespace {

// message of the last failure on this thread (a fixed buffer: recording an
// error allocates nothing)
thread_local char g_err[512];

void clear_error() { g_err[0] = '\0'; }

qa_status fail(qa_status s, const char *fmt, ...)
{
    char buf[sizeof g_err];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::memcpy(g_err, buf, sizeof g_err);
    return s;
}

#define QA_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(QA_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct Workspace {
    hipStream_t stream = nullptr;
    DiagRec *dr = nullptr;
    int64_t dr_cap = 0;
    PixRec *pr = nullptr;
    int64_t pr_cap = 0;
    int32_t *bstats = nullptr;          // per-block counts of the setup kernel
    int64_t bstats_cap = 0;
    int64_t bstats_used = 0;            // blocks of the last single-diagram setup
    int64_t *counters = nullptr;
    double *acc = nullptr;
    int64_t acc_cap = 0;
    // stage timing: event sets {start, after setup, after scoring, after re-score}
    std::vector<std::array<hipEvent_t, 4>> ev;
    int64_t ev_used = 0;
    // ragged batch
    BatchHdr *bhdr = nullptr;
    int64_t bhdr_cap = 0;
    double *bmats = nullptr;
    int64_t bmats_cap = 0;
    DiagRec *brecs = nullptr;
    int64_t brecs_cap = 0;
    // pinned staging of the batch plan (headers, then matrices), two slots
    // used in turn; a slot is rewritten only after its last copy has run
    unsigned char *bstage[2] = {};
    size_t bstage_cap[2] = {};
    hipEvent_t bstage_ev[2] = {};
    int bstage_next = 0;
    std::vector<unsigned char> bplan_inputs;  // the plan last copied to bhdr / bmats
    hipStream_t cap_stream = nullptr;   // private stream used for graph capture
    hipGraphExec_t graph = nullptr;
    std::vector<int64_t> graph_key;
    // single-diagram calls: pinned staging ring for the uploaded inputs and
    // the graphs of recent launch shapes
    static constexpr int kRing = 8;
    DiagRec *stage = nullptr;           // kRing pinned host records
    hipEvent_t stage_ev[kRing] = {};
    int stage_next = 0;
    // the inputs last copied into dr (a call with the same problem reuses them)
    std::vector<unsigned char> dr_inputs;
    // w->dr also holds the prologue's outputs (A, sums, tables) for the
    // inputs in dr_inputs: a setup or prologue launch has been enqueued since
    // they were uploaded
    bool dr_derived = false;
    // the adjoint's accumulators are zero (the final adjoint kernel leaves
    // them so; fresh allocations are cleared once)
    bool acc_zero = false;
    std::map<std::vector<int64_t>, hipGraphExec_t> graphs;
};

// autotuned launch shape of the batched kernel, per batch signature
struct BatchTune {
    int blocks;
    bool by_size;  // work order: diagrams with more candidates first
};
std::map<std::vector<int64_t>, BatchTune> g_tune;
bool g_autotune_env_read = false, g_autotune = true, g_graphs = false;

void read_env()
{
    if (g_autotune_env_read) return;
    g_autotune_env_read = true;
    if (const char *e = getenv("QA_AUTOTUNE")) g_autotune = atoi(e) != 0;
    if (const char *e = getenv("QA_GRAPHS")) g_graphs = atoi(e) != 0;
}

constexpr int64_t kMaxTimedCalls = 4096;
bool g_timing = false;

// returns the event set of this call, or nullptr when timing is off/full
std::array<hipEvent_t, 4> *timing_slot(Workspace *w)
{
    if (!g_timing || w->ev_used >= kMaxTimedCalls) return nullptr;
    if (w->ev_used >= (int64_t)w->ev.size()) {
        std::array<hipEvent_t, 4> e{};
        for (auto &x : e)
            if (hipEventCreate(&x) != hipSuccess) return nullptr;
        w->ev.push_back(e);
    }
    return &w->ev[w->ev_used++];
}

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

template <typename T>
qa_status grow(Workspace *w, T *&ptr, int64_t &cap, int64_t need)
{
    if (need <= cap && ptr) return QA_OK;
    if (ptr) {
        QA_HIP(hipStreamSynchronize(w->stream));
        QA_HIP(hipFree(ptr));
        ptr = nullptr;
        cap = 0;
    }
    int64_t n = need < 1 ? 1 : need;
    if (hipMalloc((void **)&ptr, sizeof(T) * (size_t)n) != hipSuccess) {
        ptr = nullptr;
        return fail(QA_E_WORKSPACE, "hipMalloc of %lld bytes failed",
                    (long long)(sizeof(T) * (size_t)n));
    }
    cap = n;
    return QA_OK;
}

qa_status get_ws(hipStream_t stream, Workspace **out)
{
    read_env();
    int dev = 0;
    QA_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, stream);
    auto it = g_ws.find(key);
    if (it == g_ws.end()) {
        Workspace *w = new Workspace();
        w->stream = stream;
        if (hipMalloc((void **)&w->counters, sizeof(int64_t) * kCounterWords) != hipSuccess) {
            delete w;
            return fail(QA_E_WORKSPACE, "hipMalloc of the counters failed");
        }
        it = g_ws.emplace(key, w).first;
    }
    *out = it->second;
    return QA_OK;
}

// ---------------------------------------------------------------------------
// validation (FP64 on the host, before any device work)
// ---------------------------------------------------------------------------
qa_status validate(const qa_problem *pb, bool need_kT)
{
    if (!pb) return fail(QA_E_NULL, "problem is NULL");
    if (pb->n_dot < 1 || pb->n_dot > QA_MAX_DOT)
        return fail(QA_E_SHAPE, "n_dot=%d outside [1, %d]", pb->n_dot, QA_MAX_DOT);
    if (pb->n_gate < 1 || pb->n_gate > QA_MAX_GATE)
        return fail(QA_E_SHAPE, "n_gate=%d outside [1, %d]", pb->n_gate, QA_MAX_GATE);
    if (!pb->cdd || !pb->cgd) return fail(QA_E_NULL, "cdd or cgd is NULL");
    const int n = pb->n_dot, g = pb->n_gate;
    double amax = 0.0;
    for (int i = 0; i < n * n; ++i) {
        if (!std::isfinite(pb->cdd[i])) return fail(QA_E_RANGE, "cdd[%d] is not finite", i);
        amax = std::fmax(amax, std::fabs(pb->cdd[i]));
    }
    for (int i = 0; i < n * g; ++i)
        if (!std::isfinite(pb->cgd[i])) return fail(QA_E_RANGE, "cgd[%d] is not finite", i);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j)
            if (std::fabs(pb->cdd[i * n + j] - pb->cdd[j * n + i]) > 1e-12 * amax)
                return fail(QA_E_NOT_SYMMETRIC, "cdd[%d][%d] != cdd[%d][%d]", i, j, j, i);
    // positive definiteness by Cholesky (App. B: the Maxwell block is PD)
    double L[QA_MAX_DOT * QA_MAX_DOT] = {0};
    for (int j = 0; j < n; ++j) {
        double d = pb->cdd[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return fail(QA_E_NOT_PD, "cdd is not positive definite (pivot %d)", j);
        L[j * n + j] = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double s = pb->cdd[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / L[j * n + j];
        }
    }
    if (pb->mode != QA_OPEN && pb->mode != QA_CLOSED)
        return fail(QA_E_RANGE, "mode=%d is not QA_OPEN or QA_CLOSED", pb->mode);
    if (pb->mode == QA_CLOSED && (pb->n_charge < 0 || pb->n_charge > 1000000))
        return fail(QA_E_RANGE, "n_charge=%d outside [0, 1e6]", pb->n_charge);
    if (!std::isfinite(pb->threshold) || pb->threshold < 0.0 || pb->threshold > 1.0)
        return fail(QA_E_RANGE, "threshold=%g outside [0, 1]", pb->threshold);
    if (!std::isfinite(pb->kT) || pb->kT < 0.0)
        return fail(QA_E_RANGE, "kT=%g is negative or not finite", pb->kT);
    if (need_kT && !(pb->kT > 0.0))
        return fail(QA_E_RANGE, "the softargmin needs kT > 0 (got %g)", pb->kT);
    if (pb->precision < QA_PREC_FP64 || pb->precision > QA_PREC_BF16X2)
        return fail(QA_E_RANGE, "precision=%d unknown", pb->precision);
    if (pb->flags & ~QA_FLAG_EXHAUSTIVE)
        return fail(QA_E_RANGE, "flags=0x%x has unknown bits", (unsigned)pb->flags);
    return QA_OK;
}

// Validate a sweep descriptor for a problem with n_gate gates and fill the
// device form; P receives nx * ny.
qa_status fill_grid(const qa_grid *gd, int n_gate, VGrid *vg, int64_t *P)
{
    if (!gd) return fail(QA_E_NULL, "grid is NULL");
    if (!gd->v0 || !gd->e1 || !gd->e2) return fail(QA_E_NULL, "grid v0, e1 or e2 is NULL");
    if (gd->nx < 1 || gd->ny < 1 || (int64_t)gd->nx * gd->ny > INT32_MAX)
        return fail(QA_E_SHAPE, "grid nx=%d, ny=%d: each >= 1, nx * ny < 2^31", gd->nx, gd->ny);
    const double ends[4] = {gd->a0, gd->a1, gd->b0, gd->b1};
    for (double e : ends)
        if (!std::isfinite(e)) return fail(QA_E_RANGE, "grid range is not finite");
    std::memset(vg, 0, sizeof *vg);
    for (int k = 0; k < n_gate; ++k) {
        if (!std::isfinite(gd->v0[k]) || !std::isfinite(gd->e1[k]) || !std::isfinite(gd->e2[k]))
            return fail(QA_E_RANGE, "grid vector entry %d is not finite", k);
        vg->v0[k] = gd->v0[k];
        vg->e1[k] = gd->e1[k];
        vg->e2[k] = gd->e2[k];
    }
    // linspace: the step (stop - start) / (num - 1); a single point is start
    vg->a0 = gd->a0;
    vg->a1 = gd->a1;
    vg->da = gd->nx > 1 ? (gd->a1 - gd->a0) / (double)(gd->nx - 1) : 0.0;
    vg->b0 = gd->b0;
    vg->b1 = gd->b1;
    vg->db = gd->ny > 1 ? (gd->b1 - gd->b0) / (double)(gd->ny - 1) : 0.0;
    vg->nx = gd->nx;
    vg->ny = gd->ny;
    vg->on = 1;
    *P = (int64_t)gd->nx * gd->ny;
    return QA_OK;
}

void fill_diag(const qa_problem *pb, DiagRec *h)
{
    std::memset(h, 0, sizeof(DiagRec));
    const int n = pb->n_dot, g = pb->n_gate;
    h->n = n;
    h->g = g;
    h->closed = pb->mode == QA_CLOSED;
    h->nhat = pb->mode == QA_CLOSED ? pb->n_charge : 0;
    h->kT = pb->kT;
    h->t = pb->threshold;
    h->prec = pb->precision;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) h->Cdd[i * kMaxDot + j] = pb->cdd[i * n + j];
        for (int j = 0; j < g; ++j) h->Cgd[i * kMaxGate + j] = pb->cgd[i * g + j];
    }
}

// Upload the inputs of a diagram (header, C_dd, C_gd) through a ring of
// pinned host records, so the copy is asynchronous and the host record is
// not reused before its copy has run.
qa_status upload_diag(Workspace *w, const qa_problem *pb)
{
    if (!w->stage) {
        if (hipHostMalloc((void **)&w->stage, sizeof(DiagRec) * Workspace::kRing) != hipSuccess) {
            w->stage = nullptr;
            return fail(QA_E_WORKSPACE, "hipHostMalloc of the staging ring failed");
        }
        for (auto &e : w->stage_ev) QA_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    const int slot = w->stage_next;
    w->stage_next = (slot + 1) % Workspace::kRing;
    QA_HIP(hipEventSynchronize(w->stage_ev[slot]));
    fill_diag(pb, &w->stage[slot]);
    // the same problem as the previous call on this stream: its inputs are
    // still in w->dr (only the prologue's outputs follow them there)
    if (w->dr_inputs.size() == kDiagInputBytes &&
        std::memcmp(w->dr_inputs.data(), &w->stage[slot], kDiagInputBytes) == 0)
        return QA_OK;
    QA_HIP(hipMemcpyAsync(w->dr, &w->stage[slot], kDiagInputBytes, hipMemcpyHostToDevice,
                          w->stream));
    QA_HIP(hipEventRecord(w->stage_ev[slot], w->stream));
    w->dr_derived = false;
    const unsigned char *b = reinterpret_cast<const unsigned char *>(&w->stage[slot]);
    w->dr_inputs.assign(b, b + kDiagInputBytes);
    return QA_OK;
}

qa_status grow_single(Workspace *w, int64_t P)
{
    qa_status st;
    DiagRec *dr0 = w->dr;
    if ((st = grow(w, w->dr, w->dr_cap, 1))) return st;
    if (w->dr != dr0) w->dr_inputs.clear();
    if ((st = grow(w, w->pr, w->pr_cap, P))) return st;
    // four counts per setup block; N = 16 has the most blocks
    if ((st = grow(w, w->bstats, w->bstats_cap, 4 * setup_blocks(P, kMaxDot)))) return st;
    return QA_OK;
}

bool use_matrix_cores(const qa_problem *pb)
{
    return pb->precision != QA_PREC_FP64 && pb->n_dot >= 9;
}

// candidate family of the matrix-core scorer: dense box, thresholded
// sub-box, or closed subsets
int scorer_mode(const qa_problem *pb)
{
    return pb->mode == QA_CLOSED ? 2 : (pb->threshold < 1.0 ? 1 : 0);
}

// the T = 0 scorer of the problem's candidate family and precision
hipError_t launch_scorer(const DiagRec *dr, const PixRec *pr, int64_t *counters,
                         const qa_problem *pb, int64_t P, int32_t *n_out, hipStream_t s)
{
    if (use_matrix_cores(pb))
        return launch_score_mfma(dr, pr, P, pb->precision, scorer_mode(pb),
                                 (pb->flags & QA_FLAG_EXHAUSTIVE) != 0, n_out, counters,
                                 pb->n_dot, s);
    if (pb->n_dot <= 8) return launch_score_tab(dr, pr, P, n_out, counters, pb->n_dot, s);
    return launch_score_fp64(dr, pr, P, n_out, counters, pb->n_dot, s);
}

// The device work of one single-diagram call on stream s, with the inputs
// already in dr: prologue, setup and QP in one kernel, then either the T = 0
// scoring (n_out) or the softargmin (nbar, saved).  pr holds P pixel records,
// bstats 4 * setup_blocks(P, n_dot) counts.  ev: optional stage events.
qa_status enqueue_path(DiagRec *dr, PixRec *pr, int64_t *counters, int32_t *bstats, hipStream_t s,
                       const qa_problem *pb, const double *V, int64_t P, int32_t *n_out,
                       double *nbar, SavedRec *saved, std::array<hipEvent_t, 4> *ev,
                       const VGrid *sweep = nullptr)
{
    const bool closed = pb->mode == QA_CLOSED;
    if (ev) QA_HIP(hipEventRecord((*ev)[0], s));
    QA_HIP(launch_setup(dr, V, P, pr, counters, bstats, pb->n_dot, closed, s, nullptr, nullptr,
                        sweep));
    if (ev) QA_HIP(hipEventRecord((*ev)[1], s));
    if (nbar)
        QA_HIP(launch_soft_fwd(dr, pr, P, nbar, saved, counters, pb->n_dot, s));
    else
        QA_HIP(launch_scorer(dr, pr, counters, pb, P, n_out, s));
    if (ev) QA_HIP(hipEventRecord((*ev)[2], s));
    if (ev) QA_HIP(hipEventRecord((*ev)[3], s));
    return QA_OK;
}

// the same on a workspace's buffers
qa_status enqueue_single(Workspace *w, hipStream_t s, const qa_problem *pb, const double *V,
                         int64_t P, int32_t *n_out, double *nbar, SavedRec *saved,
                         std::array<hipEvent_t, 4> *ev, const VGrid *sweep = nullptr)
{
    qa_status st = enqueue_path(w->dr, w->pr, w->counters, w->bstats, s, pb, V, P, n_out, nbar,
                                saved, ev, sweep);
    if (!st) w->dr_derived = true;
    return st;
}

// Run a single-diagram call: with stage timing on, or with a sweep (whose
// values travel in the kernel arguments), direct launches; otherwise replay
// (or capture) the graph of this launch shape.
qa_status run_single(Workspace *w, const qa_problem *pb, const double *V, int64_t P,
                     int32_t *n_out, double *nbar, SavedRec *saved, const VGrid *sweep = nullptr)
{
    qa_status st;
    if ((st = grow_single(w, P))) return st;
    if ((st = upload_diag(w, pb))) return st;
    w->bstats_used = setup_blocks(P, pb->n_dot);
    std::array<hipEvent_t, 4> *ev = timing_slot(w);
    if (ev || !g_graphs || sweep)
        return enqueue_single(w, w->stream, pb, V, P, n_out, nbar, saved, ev, sweep);
    const int path = nbar ? 2 : (use_matrix_cores(pb) ? 10 + 3 * pb->precision + scorer_mode(pb) : 1);
    std::vector<int64_t> key = {pb->n_dot, pb->mode, path, pb->flags, P, (int64_t)(uintptr_t)V,
                                (int64_t)(uintptr_t)n_out, (int64_t)(uintptr_t)nbar,
                                (int64_t)(uintptr_t)saved, (int64_t)(uintptr_t)w->dr,
                                (int64_t)(uintptr_t)w->pr,
                                (int64_t)(uintptr_t)w->bstats};
    auto it = w->graphs.find(key);
    if (it == w->graphs.end()) {
        if (w->graphs.size() >= 16) {
            QA_HIP(hipStreamSynchronize(w->stream));
            for (auto &kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
            w->graphs.clear();
        }
        if (!w->cap_stream) QA_HIP(hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking));
        hipGraph_t g;
        QA_HIP(hipStreamBeginCapture(w->cap_stream, hipStreamCaptureModeThreadLocal));
        st = enqueue_single(w, w->cap_stream, pb, V, P, n_out, nbar, saved, nullptr);
        hipError_t ec = hipStreamEndCapture(w->cap_stream, &g);
        if (st) return st;
        if (ec != hipSuccess)
            return fail(QA_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
        hipGraphExec_t exec;
        ec = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ec != hipSuccess)
            return fail(QA_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ec));
        it = w->graphs.emplace(key, exec).first;
    }
    QA_HIP(hipGraphLaunch(it->second, w->stream));
    return QA_OK;
}

qa_status read_stats(Workspace *w, qa_stats *stats)
{
    if (!stats) return QA_OK;
    std::vector<int64_t> all(kCounterWords);
    QA_HIP(hipMemcpyAsync(all.data(), w->counters, sizeof(int64_t) * kCounterWords,
                          hipMemcpyDeviceToHost, w->stream));
    QA_HIP(hipStreamSynchronize(w->stream));
    std::vector<int32_t> blk(4 * w->bstats_used);
    if (w->bstats_used)
        QA_HIP(hipMemcpyAsync(blk.data(), w->bstats, sizeof(int32_t) * blk.size(),
                              hipMemcpyDeviceToHost, w->stream));
    QA_HIP(hipStreamSynchronize(w->stream));
    int64_t c[C_NUM] = {};
    for (int slot = 0; slot < kCounterSlots; ++slot)
        for (int i = 0; i < C_NUM; ++i) c[i] += all[slot * C_NUM + i];
    // counts of the single-diagram setup kernel, per block
    const int which[4] = {C_PIXELS, C_QP, C_DOUBLED, C_QP_FAIL};
    for (int64_t b = 0; b < w->bstats_used; ++b)
        for (int k = 0; k < 4; ++k) c[which[k]] += blk[4 * b + k];
    stats->pixels = c[C_PIXELS];
    stats->qp_pixels = c[C_QP];
    stats->qp_failures = c[C_QP_FAIL];
    stats->doubled_pixels = c[C_DOUBLED];
    stats->near_tie_pixels = c[C_NEAR_TIE];
    stats->fp64_gap_below_1e9 = c[C_GAP_1E9];
    stats->candidates = c[C_CANDIDATES];
    // only the bound-ordered search skips candidates; the other scorers
    // compute every energy of the candidate set
    stats->scored = c[C_SCORED] ? c[C_SCORED] : c[C_CANDIDATES];
    return QA_OK;
}

// The adjoint's device work (validated problem; voltages V or the sweep vg)
qa_status backward(const qa_problem *prob, const double *V_dev, const VGrid *vg, int64_t P,
                   const double *grad_nbar_dev, const void *saved_dev, double *grad_cdd_dev,
                   double *grad_cgd_dev, double *grad_V_dev, void *hip_stream)
{
    qa_status st;
    if (prob->n_dot > 12)
        return fail(QA_E_UNSUPPORTED, "the adjoint is built for n_dot <= 12 (got %d)", prob->n_dot);
    if (!grad_cdd_dev || !grad_cgd_dev) return fail(QA_E_NULL, "gradient output is NULL");
    if (P > 0 && (!grad_nbar_dev || !saved_dev))
        return fail(QA_E_NULL, "grad_nbar_dev or saved_dev is NULL");
    Workspace *w;
    if ((st = get_ws((hipStream_t)hip_stream, &w))) return st;
    DiagRec *dr0 = w->dr;
    if ((st = grow(w, w->dr, w->dr_cap, 1))) return st;
    if (w->dr != dr0) w->dr_inputs.clear();
    const int64_t nacc = (int64_t)kBwdReplicas * kBwdAccWords;
    double *acc0 = w->acc;
    if ((st = grow(w, w->acc, w->acc_cap, nacc))) return st;
    if (w->acc != acc0) w->acc_zero = false;
    if ((st = upload_diag(w, prob))) return st;
    // the prologue (A, C_dd 1, tables) only when the record does not already
    // hold it for these inputs (the usual case after the forward call);
    // it also clears the accumulators when they are not known to be zero
    const int64_t nzero = w->acc_zero ? 0 : nacc;
    if (!w->dr_derived) {
        QA_HIP(launch_prep(w->dr, 1, nullptr, w->stream, nzero ? w->acc : nullptr, nzero));
        w->dr_derived = true;
    } else if (nzero) {
        QA_HIP(launch_zero_i64(reinterpret_cast<int64_t *>(w->acc), (int)nzero, w->stream));
    }
    w->acc_zero = false;  // until the final kernel below is enqueued
    QA_HIP(launch_soft_bwd(w->dr, V_dev, P, grad_nbar_dev, (const SavedRec *)saved_dev, w->acc,
                           grad_V_dev, prob->n_dot, w->stream, vg));
    QA_HIP(launch_soft_bwd_final(w->dr, w->acc, grad_cdd_dev, grad_cgd_dev, w->stream));
    w->acc_zero = true;
    return QA_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Library-owned device scratch of qa_ground_state_noalloc: the diagram
// record, the counters, the setup kernel's per-block counts and one record
// per pixel, for at most QA_NOALLOC_MAX_PIXELS pixels.  Every device the
// library runs on holds its own copy for the life of the process.  In host
// code `scratch` names a host-side stand-in: kernels get the device address
// that hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kScrDiag = 0;
constexpr size_t kScrCounters = kScrDiag + align256(sizeof(DiagRec));
constexpr size_t kScrBstats = kScrCounters + align256(sizeof(int64_t) * kCounterWords);
constexpr int64_t kScrBstatsWords = 4 * setup_blocks_max(QA_NOALLOC_MAX_PIXELS);
constexpr size_t kScrPix = kScrBstats + align256(sizeof(int32_t) * kScrBstatsWords);
constexpr size_t kScratchBytes = kScrPix + sizeof(PixRec) * (size_t)QA_NOALLOC_MAX_PIXELS;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_dev[kMaxDevices] = {};

// device address of the current device's scratch, looked up once per device
qa_status scratch_address(unsigned char **out)
{
    int dev = 0;
    QA_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(QA_E_DEVICE, "device %d beyond the %d this build tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(QA_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return QA_OK;
}

// a diagram's inputs into dr as kernel arguments: the header and C_dd in one
// chunk, C_gd in chunks of whole rows (at most two for n_gate <= 32)
qa_status put_inputs(DiagRec *dr, const qa_problem *pb, hipStream_t s)
{
    InputChunk c;
    std::memset(&c, 0, sizeof c);
    const int n = pb->n_dot, g = pb->n_gate;
    c.n = n;
    c.g = g;
    c.closed = pb->mode == QA_CLOSED;
    c.nhat = pb->mode == QA_CLOSED ? pb->n_charge : 0;
    c.kT = pb->kT;
    c.t = pb->threshold;
    c.prec = pb->precision;
    c.part = 0;
    std::memcpy(c.v, pb->cdd, sizeof(double) * n * n);
    QA_HIP(launch_put_inputs(dr, c, s));
    c.part = 1;
    const int rows_per_chunk = kChunkDoubles / g;
    for (int r0 = 0; r0 < kMaxDot; r0 += rows_per_chunk) {
        const int r1 = std::min(r0 + rows_per_chunk, n);
        c.row0 = r0;
        // the last chunk also writes the zero rows past n
        c.row1 = r1 >= n ? kMaxDot : r1;
        std::memset(c.v, 0, sizeof c.v);
        if (r1 > r0) std::memcpy(c.v, pb->cgd + (size_t)r0 * g, sizeof(double) * (r1 - r0) * g);
        QA_HIP(launch_put_inputs(dr, c, s));
        if (c.row1 == kMaxDot) break;
    }
    return QA_OK;
}

}  // namespace

extern "C" {

qa_status qa_ground_state(const qa_problem *prob, const double *V_dev, int64_t P,
                          int32_t *n_out_dev, qa_stats *stats, void *hip_stream)
{
    clear_error();
    qa_status st = validate(prob, false);
    if (st) return st;
    if (P < 0 || P > INT32_MAX) return fail(QA_E_SHAPE, "P=%lld outside [0, 2^31)", (long long)P);
    if (P == 0) {
        if (stats) std::memset(stats, 0, sizeof *stats);
        return QA_OK;
    }
    if (!V_dev || !n_out_dev) return fail(QA_E_NULL, "V_dev or n_out_dev is NULL");
    Workspace *w;
    if ((st = get_ws((hipStream_t)hip_stream, &w))) return st;
    if ((st = run_single(w, prob, V_dev, P, n_out_dev, nullptr, nullptr))) return st;
    return read_stats(w, stats);
}

qa_status qa_ground_state_noalloc(const qa_problem *prob, const double *V_dev, int64_t P,
                                  int32_t *n_out_dev, void *hip_stream)
{
    clear_error();
    qa_status st = validate(prob, false);
    if (st) return st;
    if (P < 0 || P > QA_NOALLOC_MAX_PIXELS)
        return fail(QA_E_SHAPE, "P=%lld outside [0, %d], the pixels the static scratch holds",
                    (long long)P, QA_NOALLOC_MAX_PIXELS);
    if (P == 0) return QA_OK;
    if (!V_dev || !n_out_dev) return fail(QA_E_NULL, "V_dev or n_out_dev is NULL");
    if (4 * setup_blocks(P, prob->n_dot) > kScrBstatsWords)
        return fail(QA_E_SHAPE, "P=%lld needs more setup blocks than the scratch counts",
                    (long long)P);
    unsigned char *base;
    if ((st = scratch_address(&base))) return st;
    DiagRec *dr = reinterpret_cast<DiagRec *>(base + kScrDiag);
    int64_t *counters = reinterpret_cast<int64_t *>(base + kScrCounters);
    int32_t *bstats = reinterpret_cast<int32_t *>(base + kScrBstats);
    PixRec *pr = reinterpret_cast<PixRec *>(base + kScrPix);
    hipStream_t s = (hipStream_t)hip_stream;
    if ((st = put_inputs(dr, prob, s))) return st;
    return enqueue_path(dr, pr, counters, bstats, s, prob, V_dev, P, n_out_dev, nullptr, nullptr,
                        nullptr);
}

qa_status qa_ground_state_grid(const qa_problem *prob, const qa_grid *grid, int32_t *n_out_dev,
                               qa_stats *stats, void *hip_stream)
{
    clear_error();
    qa_status st = validate(prob, false);
    if (st) return st;
    VGrid vg;
    int64_t P = 0;
    if ((st = fill_grid(grid, prob->n_gate, &vg, &P))) return st;
    if (!n_out_dev) return fail(QA_E_NULL, "n_out_dev is NULL");
    Workspace *w;
    if ((st = get_ws((hipStream_t)hip_stream, &w))) return st;
    if ((st = run_single(w, prob, nullptr, P, n_out_dev, nullptr, nullptr, &vg))) return st;
    return read_stats(w, stats);
}

qa_status qa_continuous_min(const qa_problem *prob, const double *V_dev, int64_t P,
                            double *x_out_dev, int32_t *flags_out_dev, qa_stats *stats,
                            void *hip_stream)
{
    clear_error();
    qa_status st = validate(prob, false);
    if (st) return st;
    if (P < 0 || P > INT32_MAX) return fail(QA_E_SHAPE, "P=%lld outside [0, 2^31)", (long long)P);
    if (P == 0) {
        if (stats) std::memset(stats, 0, sizeof *stats);
        return QA_OK;
    }
    if (!V_dev || !x_out_dev) return fail(QA_E_NULL, "V_dev or x_out_dev is NULL");
    Workspace *w;
    if ((st = get_ws((hipStream_t)hip_stream, &w))) return st;
    if ((st = grow_single(w, P))) return st;
    if ((st = upload_diag(w, prob))) return st;
    QA_HIP(launch_setup(w->dr, V_dev, P, w->pr, w->counters, w->bstats, prob->n_dot,
                        prob->mode == QA_CLOSED, w->stream, x_out_dev, flags_out_dev));
    w->bstats_used = setup_blocks(P, prob->n_dot);
    return read_stats(w, stats);
}

size_t qa_saved_bytes(int64_t P, int32_t n_dot)
{
    (void)n_dot;
    return P <= 0 ? 0 : (size_t)P * sizeof(SavedRec);
}

qa_status qa_soft_charge(const qa_problem *prob, const double *V_dev, int64_t P,
                         double *nbar_out_dev, void *saved_dev, qa_stats *stats, void *hip_stream)
{
    clear_error();
    qa_status st = validate(prob, true);
    if (st) return st;
    if (P < 0 || P > INT32_MAX) return fail(QA_E_SHAPE, "P=%lld outside [0, 2^31)", (long long)P);
    if (P == 0) {
        if (stats) std::memset(stats, 0, sizeof *stats);
        return QA_OK;
    }
    if (!V_dev || !nbar_out_dev) return fail(QA_E_NULL, "V_dev or nbar_out_dev is NULL");
    Workspace *w;
    if ((st = get_ws((hipStream_t)hip_stream, &w))) return st;
    if ((st = run_single(w, prob, V_dev, P, nullptr, nbar_out_dev, (SavedRec *)saved_dev)))
        return st;
    return read_stats(w, stats);
}

qa_status qa_soft_charge_grid(const qa_problem *prob, const qa_grid *grid, double *nbar_out_dev,
                              void *saved_dev, qa_stats *stats, void *hip_stream)
{
    clear_error();
    qa_status st = validate(prob, true);
    if (st) return st;
    VGrid vg;
    int64_t P = 0;
    if ((st = fill_grid(grid, prob->n_gate, &vg, &P))) return st;
    if (!nbar_out_dev) return fail(QA_E_NULL, "nbar_out_dev is NULL");
    Workspace *w;
    if ((st = get_ws((hipStream_t)hip_stream, &w))) return st;
    if ((st = run_single(w, prob, nullptr, P, nullptr, nbar_out_dev, (SavedRec *)saved_dev, &vg)))
        return st;
    return read_stats(w, stats);
}

qa_status qa_soft_charge_backward(const qa_problem *prob, const double *V_dev, int64_t P,
                                  const double *grad_nbar_dev, const void *saved_dev,
                                  double *grad_cdd_dev, double *grad_cgd_dev, double *grad_V_dev,
                                  void *hip_stream)
{
    clear_error();
    qa_status st = validate(prob, true);
    if (st) return st;
    if (P < 0 || P > INT32_MAX) return fail(QA_E_SHAPE, "P=%lld outside [0, 2^31)", (long long)P);
    if (P > 0 && !V_dev) return fail(QA_E_NULL, "V_dev is NULL");
    return backward(prob, V_dev, nullptr, P, grad_nbar_dev, saved_dev, grad_cdd_dev, grad_cgd_dev,
                    grad_V_dev, hip_stream);
}

qa_status qa_soft_charge_backward_grid(const qa_problem *prob, const qa_grid *grid,
                                       const double *grad_nbar_dev, const void *saved_dev,
                                       double *grad_cdd_dev, double *grad_cgd_dev,
                                       double *grad_V_dev, void *hip_stream)
{
    clear_error();
    qa_status st = validate(prob, true);
    if (st) return st;
    VGrid vg;
    int64_t P = 0;
    if ((st = fill_grid(grid, prob->n_gate, &vg, &P))) return st;
    return backward(prob, nullptr, &vg, P, grad_nbar_dev, saved_dev, grad_cdd_dev, grad_cgd_dev,
                    grad_V_dev, hip_stream);
}

}  // extern "C"

namespace {

// host-side description of a batch in a given work order
struct BatchPlan {
    std::vector<BatchHdr> hdr;
    std::vector<double> mats;
    int64_t tiles = 0;
    int max_dot = 0;
};

// (grids: NULL, or one sweep per diagram, validated; then v_offsets and
// pix_counts are unused)
void plan_batch(const qa_problem *probs, int32_t n_diag, const int64_t *v_offsets,
                const int64_t *pix_counts, const qa_grid *grids, const int64_t *out_offsets,
                bool by_size, BatchPlan &plan)
{
    std::vector<int> order(n_diag);
    for (int d = 0; d < n_diag; ++d) order[d] = d;
    if (by_size) {
        // largest candidate sets first, so the tail of the queue is cheap
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return probs[a].n_dot > probs[b].n_dot;
        });
    }
    plan.hdr.resize(n_diag);
    plan.mats.clear();
    plan.tiles = 0;
    plan.max_dot = 0;
    for (int j = 0; j < n_diag; ++j) {
        const int d = order[j];
        const qa_problem &pb = probs[d];
        BatchHdr &h = plan.hdr[j];
        h.n = pb.n_dot;
        h.g = pb.n_gate;
        h.closed = pb.mode == QA_CLOSED;
        h.nhat = pb.mode == QA_CLOSED ? pb.n_charge : 0;
        h.kT = pb.kT;
        h.t = pb.threshold;
        h.out_off = out_offsets[d];
        h.mat_off = (int64_t)plan.mats.size();
        h.tile0 = plan.tiles;
        plan.mats.insert(plan.mats.end(), pb.cdd, pb.cdd + pb.n_dot * pb.n_dot);
        plan.mats.insert(plan.mats.end(), pb.cgd, pb.cgd + pb.n_dot * pb.n_gate);
        if (grids) {
            const qa_grid &gd = grids[d];
            h.v_off = 0;
            h.nx = gd.nx;
            h.ny = gd.ny;
            h.P = (int64_t)gd.nx * gd.ny;
            h.grid_off = (int64_t)plan.mats.size();
            plan.mats.insert(plan.mats.end(), gd.v0, gd.v0 + pb.n_gate);
            plan.mats.insert(plan.mats.end(), gd.e1, gd.e1 + pb.n_gate);
            plan.mats.insert(plan.mats.end(), gd.e2, gd.e2 + pb.n_gate);
            const double da = gd.nx > 1 ? (gd.a1 - gd.a0) / (double)(gd.nx - 1) : 0.0;
            const double db = gd.ny > 1 ? (gd.b1 - gd.b0) / (double)(gd.ny - 1) : 0.0;
            const double sc[6] = {gd.a0, da, gd.a1, gd.b0, db, gd.b1};
            plan.mats.insert(plan.mats.end(), sc, sc + 6);
        } else {
            h.v_off = v_offsets[d];
            h.P = pix_counts[d];
            h.grid_off = 0;
            h.nx = h.ny = 0;
        }
        plan.tiles += (h.P + 63) / 64;
        plan.max_dot = std::max(plan.max_dot, pb.n_dot);
    }
}

qa_status upload_plan(Workspace *w, const BatchPlan &plan, int32_t n_diag)
{
    qa_status st;
    const BatchHdr *h0 = w->bhdr;
    const double *m0 = w->bmats;
    if ((st = grow(w, w->bhdr, w->bhdr_cap, n_diag))) return st;
    if ((st = grow(w, w->bmats, w->bmats_cap, (int64_t)plan.mats.size()))) return st;
    if ((st = grow(w, w->brecs, w->brecs_cap, n_diag))) return st;
    if (w->bhdr != h0 || w->bmats != m0) w->bplan_inputs.clear();
    const size_t nh = sizeof(BatchHdr) * n_diag, nm = sizeof(double) * plan.mats.size();
    const unsigned char *hb = reinterpret_cast<const unsigned char *>(plan.hdr.data());
    const unsigned char *mb = reinterpret_cast<const unsigned char *>(plan.mats.data());
    // the same plan as the last upload on this stream: the device copies hold it
    if (w->bplan_inputs.size() == nh + nm && std::memcmp(w->bplan_inputs.data(), hb, nh) == 0 &&
        std::memcmp(w->bplan_inputs.data() + nh, mb, nm) == 0)
        return QA_OK;
    // through pinned memory, so the copy is asynchronous (a pageable source
    // makes the runtime wait for the stream)
    const int slot = w->bstage_next;
    w->bstage_next ^= 1;
    if (!w->bstage_ev[slot])
        QA_HIP(hipEventCreateWithFlags(&w->bstage_ev[slot], hipEventDisableTiming));
    QA_HIP(hipEventSynchronize(w->bstage_ev[slot]));
    if (w->bstage_cap[slot] < nh + nm) {
        if (w->bstage[slot]) QA_HIP(hipHostFree(w->bstage[slot]));
        w->bstage[slot] = nullptr;
        w->bstage_cap[slot] = 0;
        const size_t cap = (nh + nm) * 5 / 4 + 4096;
        if (hipHostMalloc((void **)&w->bstage[slot], cap) != hipSuccess) {
            w->bstage[slot] = nullptr;
            return fail(QA_E_WORKSPACE, "hipHostMalloc of %zu bytes of batch staging failed", cap);
        }
        w->bstage_cap[slot] = cap;
    }
    unsigned char *stg = w->bstage[slot];
    std::memcpy(stg, hb, nh);
    std::memcpy(stg + nh, mb, nm);
    w->bplan_inputs.assign(stg, stg + nh + nm);
    QA_HIP(hipMemcpyAsync(w->bhdr, stg, nh, hipMemcpyHostToDevice, w->stream));
    if (nm) QA_HIP(hipMemcpyAsync(w->bmats, stg + nh, nm, hipMemcpyHostToDevice, w->stream));
    QA_HIP(hipEventRecord(w->bstage_ev[slot], w->stream));
    return QA_OK;
}

// the device work of one batch: zero the counters and the queue, prologue of
// every diagram, the persistent kernel
qa_status enqueue_batch(Workspace *w, hipStream_t s, int32_t n_diag, const BatchPlan &plan,
                        const double *V, int32_t *n_out, double *nbar, int blocks)
{
    QA_HIP(launch_zero_i64(w->counters, kCounterWords, s));
    QA_HIP(launch_prep_batch(w->bhdr, w->bmats, w->brecs, n_diag, s));
    QA_HIP(launch_batch(w->bhdr, w->brecs, w->bmats, n_diag, plan.tiles, V, n_out, nbar,
                        w->counters, plan.max_dot, blocks, s));
    return QA_OK;
}

}  // namespace

extern "C" {

}  // extern "C"

namespace {

// a batch of explicit-voltage diagrams (grids NULL) or of sweeps
qa_status batched(const qa_problem *probs, int32_t n_diag, const double *V_dev,
                  const int64_t *v_offsets, const int64_t *pix_counts, const qa_grid *grids,
                  const int64_t *out_offsets, int32_t *n_out_dev, double *nbar_out_dev,
                  qa_stats *stats, void *hip_stream)
{
    read_env();
    if (n_diag < 0) return fail(QA_E_SHAPE, "n_diag=%d is negative", n_diag);
    if (n_diag == 0) {
        if (stats) std::memset(stats, 0, sizeof *stats);
        return QA_OK;
    }
    if (!probs || !out_offsets || (!grids && (!v_offsets || !pix_counts)))
        return fail(QA_E_NULL, "probs or an offset array is NULL");
    int64_t total = 0;
    for (int d = 0; d < n_diag; ++d) {
        qa_status st = validate(&probs[d], false);
        if (st) return fail(st, "diagram %d: %s", d, g_err);
        int64_t P = 0;
        if (grids) {
            VGrid vg;
            if ((st = fill_grid(&grids[d], probs[d].n_gate, &vg, &P)))
                return fail(st, "diagram %d: %s", d, g_err);
        } else {
            if (pix_counts[d] < 0 || v_offsets[d] < 0)
                return fail(QA_E_SHAPE, "diagram %d: negative pixel count or offset", d);
            P = pix_counts[d];
        }
        if (out_offsets[d] < 0) return fail(QA_E_SHAPE, "diagram %d: negative offset", d);
        total += P;
    }
    if (total == 0) {
        if (stats) std::memset(stats, 0, sizeof *stats);
        return QA_OK;
    }
    if ((!grids && !V_dev) || !n_out_dev) return fail(QA_E_NULL, "V_dev or n_out_dev is NULL");
    Workspace *w;
    qa_status st;
    if ((st = get_ws((hipStream_t)hip_stream, &w))) return st;

    // signature of the batch for the tuning cache
    int max_dot = 0, n_soft = 0;
    for (int d = 0; d < n_diag; ++d) {
        max_dot = std::max(max_dot, probs[d].n_dot);
        n_soft += probs[d].kT > 0.0;
    }
    w->bstats_used = 0;  // the batched kernels count into the counter slots only
    std::vector<int64_t> sig = {n_diag, total, max_dot, n_soft > 0 && nbar_out_dev != nullptr,
                                grids != nullptr};
    BatchPlan plan;
    auto it = g_tune.find(sig);
    if (it == g_tune.end() && g_autotune) {
        // time every candidate launch shape on this very batch (each run
        // writes the same outputs; the better of two runs, so that a cold
        // first launch or a stray slow one does not decide) and keep the
        // fastest
        int dev = 0, cus = 256;
        QA_HIP(hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
        hipEvent_t e0, e1;
        QA_HIP(hipEventCreate(&e0));
        QA_HIP(hipEventCreate(&e1));
        BatchTune best{cus * 4, true};
        float best_ms = 1e30f;
        for (int by_size = 0; by_size < 2; ++by_size) {
            plan_batch(probs, n_diag, v_offsets, pix_counts, grids, out_offsets, by_size != 0,
                       plan);
            if ((st = upload_plan(w, plan, n_diag))) return st;
            for (int mult : {2, 4, 8, 16}) {
                const int blocks = cus * mult;
                for (int rep = 0; rep < 2; ++rep) {
                    QA_HIP(hipEventRecord(e0, w->stream));
                    if ((st = enqueue_batch(w, w->stream, n_diag, plan, V_dev, n_out_dev,
                                            nbar_out_dev, blocks)))
                        return st;
                    QA_HIP(hipEventRecord(e1, w->stream));
                    QA_HIP(hipEventSynchronize(e1));
                    float ms = 0.0f;
                    QA_HIP(hipEventElapsedTime(&ms, e0, e1));
                    if (ms < best_ms) { best_ms = ms; best = BatchTune{blocks, by_size != 0}; }
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        it = g_tune.emplace(sig, best).first;
    }
    const BatchTune tune = (it != g_tune.end()) ? it->second : BatchTune{1024, true};
    plan_batch(probs, n_diag, v_offsets, pix_counts, grids, out_offsets, tune.by_size, plan);
    if ((st = upload_plan(w, plan, n_diag))) return st;

    if (!g_graphs) {
        if ((st = enqueue_batch(w, w->stream, n_diag, plan, V_dev, n_out_dev, nbar_out_dev,
                                tune.blocks)))
            return st;
        return read_stats(w, stats);
    }
    // one graph per (batch layout, buffers): zero kernel, prologue, persistent
    // kernel; captured on a private stream, launched on the caller's
    std::vector<int64_t> key = {n_diag, plan.tiles, plan.max_dot, tune.blocks,
                                (int64_t)(uintptr_t)V_dev, (int64_t)(uintptr_t)n_out_dev,
                                (int64_t)(uintptr_t)nbar_out_dev, (int64_t)(uintptr_t)w->bhdr,
                                (int64_t)(uintptr_t)w->bmats, (int64_t)(uintptr_t)w->brecs};
    if (!w->graph || w->graph_key != key) {
        if (w->graph) {
            QA_HIP(hipStreamSynchronize(w->stream));
            (void)hipGraphExecDestroy(w->graph);
            w->graph = nullptr;
        }
        if (!w->cap_stream) QA_HIP(hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking));
        hipGraph_t g;
        QA_HIP(hipStreamBeginCapture(w->cap_stream, hipStreamCaptureModeThreadLocal));
        st = enqueue_batch(w, w->cap_stream, n_diag, plan, V_dev, n_out_dev, nbar_out_dev,
                           tune.blocks);
        hipError_t ec = hipStreamEndCapture(w->cap_stream, &g);
        if (st) return st;
        if (ec != hipSuccess)
            return fail(QA_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
        ec = hipGraphInstantiate(&w->graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ec != hipSuccess) {
            w->graph = nullptr;
            return fail(QA_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ec));
        }
        w->graph_key = key;
    }
    QA_HIP(hipGraphLaunch(w->graph, w->stream));
    return read_stats(w, stats);
}

}  // namespace

extern "C" {

qa_status qa_ground_state_batched(const qa_problem *probs, int32_t n_diag, const double *V_dev,
                                  const int64_t *v_offsets, const int64_t *pix_counts,
                                  const int64_t *out_offsets, int32_t *n_out_dev,
                                  double *nbar_out_dev, qa_stats *stats, void *hip_stream)
{
    clear_error();
    return batched(probs, n_diag, V_dev, v_offsets, pix_counts, nullptr, out_offsets, n_out_dev,
                   nbar_out_dev, stats, hip_stream);
}

qa_status qa_ground_state_batched_grid(const qa_problem *probs, int32_t n_diag,
                                       const qa_grid *grids, const int64_t *out_offsets,
                                       int32_t *n_out_dev, double *nbar_out_dev, qa_stats *stats,
                                       void *hip_stream)
{
    clear_error();
    if (n_diag > 0 && !grids) return fail(QA_E_NULL, "grids is NULL");
    return batched(probs, n_diag, nullptr, nullptr, nullptr, grids, out_offsets, n_out_dev,
                   nbar_out_dev, stats, hip_stream);
}

void qa_timing_enable(int on) { g_timing = on != 0; }

void qa_graphs_enable(int on)
{
    read_env();
    g_graphs = on != 0;
}

void qa_timing_reset(void *hip_stream)
{
    Workspace *w;
    if (get_ws((hipStream_t)hip_stream, &w) == QA_OK) w->ev_used = 0;
}

qa_status qa_timing_sum(void *hip_stream, double *ms_out, int64_t *calls_out)
{
    clear_error();
    if (!ms_out) return fail(QA_E_NULL, "ms_out is NULL");
    Workspace *w;
    qa_status st;
    if ((st = get_ws((hipStream_t)hip_stream, &w))) return st;
    QA_HIP(hipStreamSynchronize(w->stream));
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < w->ev_used; ++i) {
        for (int s = 0; s < 3; ++s) {
            float ms = 0.0f;
            QA_HIP(hipEventElapsedTime(&ms, w->ev[i][s], w->ev[i][s + 1]));
            acc[s] += ms;
        }
    }
    for (int s = 0; s < 3; ++s) ms_out[s] = acc[s];
    if (calls_out) *calls_out = w->ev_used;
    return QA_OK;
}

qa_status qa_time_kernels(const qa_problem *prob, const double *V_dev, int64_t P,
                          int32_t *n_out_dev, int32_t reps, double *ms_out, void *hip_stream)
{
    clear_error();
    qa_status st = validate(prob, false);
    if (st) return st;
    if (P < 1 || P > INT32_MAX) return fail(QA_E_SHAPE, "P=%lld outside [1, 2^31)", (long long)P);
    if (reps < 1 || reps > 100000) return fail(QA_E_RANGE, "reps=%d outside [1, 1e5]", reps);
    if (!V_dev || !n_out_dev || !ms_out) return fail(QA_E_NULL, "V_dev, n_out_dev or ms_out is NULL");
    Workspace *w;
    if ((st = get_ws((hipStream_t)hip_stream, &w))) return st;
    if ((st = grow_single(w, P))) return st;
    if ((st = upload_diag(w, prob))) return st;
    w->bstats_used = setup_blocks(P, prob->n_dot);
    const hipStream_t s = w->stream;
    // one whole call first: the records the repeated launches read
    if ((st = enqueue_single(w, s, prob, V_dev, P, n_out_dev, nullptr, nullptr, nullptr)))
        return st;
    hipEvent_t ev[3] = {};
    for (auto &e : ev) QA_HIP(hipEventCreate(&e));
    auto done = [&](qa_status r) {
        for (auto &e : ev) (void)hipEventDestroy(e);
        return r;
    };
    auto setup = [&]() {
        return launch_setup(w->dr, V_dev, P, w->pr, w->counters, w->bstats, prob->n_dot,
                            prob->mode == QA_CLOSED, s) == hipSuccess;
    };
    // reps setup launches, then reps (setup, scorer) pairs: the scorer of a
    // pair reads what its setup has just written, as in a call
    if (hipEventRecord(ev[0], s) != hipSuccess) return done(fail(QA_E_DEVICE, "event record failed"));
    for (int r = 0; r < reps; ++r)
        if (!setup()) return done(fail(QA_E_DEVICE, "setup launch failed"));
    if (hipEventRecord(ev[1], s) != hipSuccess) return done(fail(QA_E_DEVICE, "event record failed"));
    for (int r = 0; r < reps; ++r) {
        if (!setup()) return done(fail(QA_E_DEVICE, "setup launch failed"));
        if (launch_scorer(w->dr, w->pr, w->counters, prob, P, n_out_dev, s) != hipSuccess)
            return done(fail(QA_E_DEVICE, "scorer launch failed"));
    }
    if (hipEventRecord(ev[2], s) != hipSuccess) return done(fail(QA_E_DEVICE, "event record failed"));
    if (hipEventSynchronize(ev[2]) != hipSuccess)
        return done(fail(QA_E_DEVICE, "event synchronize failed"));
    float t01 = 0.0f, t12 = 0.0f;
    if (hipEventElapsedTime(&t01, ev[0], ev[1]) != hipSuccess ||
        hipEventElapsedTime(&t12, ev[1], ev[2]) != hipSuccess)
        return done(fail(QA_E_DEVICE, "event elapsed time failed"));
    ms_out[0] = t01 / reps;
    ms_out[1] = (t12 - t01) / reps;
    return done(QA_OK);
}

const char *qa_last_error(void) { return g_err; }

void qa_release(void *hip_stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    Workspace *w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_ws.find(std::make_pair(dev, (hipStream_t)hip_stream));
        if (it == g_ws.end()) return;
        w = it->second;
        g_ws.erase(it);
    }
    (void)hipStreamSynchronize(w->stream);
    (void)hipFree(w->dr);
    (void)hipFree(w->pr);
    (void)hipFree(w->bstats);
    (void)hipFree(w->counters);
    (void)hipFree(w->acc);
    for (auto &e : w->ev)
        for (auto &x : e) (void)hipEventDestroy(x);
    (void)hipFree(w->bhdr);
    (void)hipFree(w->bmats);
    (void)hipFree(w->brecs);
    for (int i = 0; i < 2; ++i) {
        if (w->bstage[i]) (void)hipHostFree(w->bstage[i]);
        if (w->bstage_ev[i]) (void)hipEventDestroy(w->bstage_ev[i]);
    }
    if (w->graph) (void)hipGraphExecDestroy(w->graph);
    for (auto &kv : w->graphs) (void)hipGraphExecDestroy(kv.second);
    if (w->stage) (void)hipHostFree(w->stage);
    for (auto &e : w->stage_ev)
        if (e) (void)hipEventDestroy(e);
    if (w->cap_stream) (void)hipStreamDestroy(w->cap_stream);
    delete w;
}

size_t qa_sensor_noise_len(int64_t P, int32_t n_sensor, int32_t pink_octaves)
{
    if (P <= 0 || n_sensor <= 0) return 0;
    size_t len = 2 * (size_t)P * (size_t)n_sensor;
    for (int k = 0; k < pink_octaves; ++k)
        len += (size_t)n_sensor * (size_t)((P + ((int64_t)1 << k) - 1) >> k);
    return len;
}

qa_status qa_sensor_response(const qa_problem *prob, const qa_sensor *sp, const double *V_dev,
                             int64_t P, const int32_t *n_array_dev, const double *nbar_array_dev,
                             const double *noise_dev, double *signal_dev, void *hip_stream)
{
    clear_error();
    qa_status st = validate(prob, false);
    if (st) return st;
    if (!sp) return fail(QA_E_NULL, "sensor parameters are NULL");
    if (sp->n_sensor < 1 || sp->n_sensor > 4 || sp->n_sensor >= prob->n_dot + 1)
        return fail(QA_E_SHAPE, "n_sensor=%d outside [1, min(4, n_dot)]", sp->n_sensor);
    if (sp->shape != QA_SENSOR_LORENTZIAN && sp->shape != QA_SENSOR_GAUSSIAN)
        return fail(QA_E_RANGE, "shape=%d unknown", sp->shape);
    if (!std::isfinite(sp->gamma) || !(sp->gamma > 0.0))
        return fail(QA_E_RANGE, "gamma=%g must be positive", sp->gamma);
    if (!(sp->white >= 0.0) || !(sp->pink >= 0.0) || !(sp->jump >= 0.0) ||
        !std::isfinite(sp->white) || !std::isfinite(sp->pink) || !std::isfinite(sp->jump))
        return fail(QA_E_RANGE, "noise amplitudes must be finite and >= 0");
    if (!(sp->jump_rate >= 0.0 && sp->jump_rate <= 1.0))
        return fail(QA_E_RANGE, "jump_rate=%g outside [0, 1]", sp->jump_rate);
    if (sp->pink_octaves < 0 || sp->pink_octaves > 40 || (sp->pink > 0.0 && sp->pink_octaves < 1))
        return fail(QA_E_RANGE, "pink_octaves=%d outside [%d, 40]", sp->pink_octaves,
                    sp->pink > 0.0 ? 1 : 0);
    if (P < 0 || P > INT32_MAX) return fail(QA_E_SHAPE, "P=%lld outside [0, 2^31)", (long long)P);
    if (P == 0) return QA_OK;
    if (!V_dev || !signal_dev) return fail(QA_E_NULL, "V_dev or signal_dev is NULL");
    if (prob->n_dot > sp->n_sensor && !n_array_dev && !nbar_array_dev)
        return fail(QA_E_NULL, "the array charges (n_array_dev or nbar_array_dev) are NULL");
    const bool noisy = sp->white > 0.0 || sp->pink > 0.0 || sp->jump > 0.0;
    if (noisy && !noise_dev) return fail(QA_E_NULL, "noise_dev is NULL with noise switched on");
    Workspace *w;
    if ((st = get_ws((hipStream_t)hip_stream, &w))) return st;
    DiagRec *dr0 = w->dr;
    if ((st = grow(w, w->dr, w->dr_cap, 1))) return st;
    if (w->dr != dr0) w->dr_inputs.clear();
    if ((st = upload_diag(w, prob))) return st;
    const int S = sp->n_sensor;
    const double *white = (noisy && sp->white > 0.0) ? noise_dev : nullptr;
    const double *pink = (noisy && sp->pink > 0.0) ? noise_dev + (size_t)P * S : nullptr;
    // the layout of qa_sensor_noise_len: white, pink_octaves octaves, jumps
    size_t pink_len = 0;
    for (int k = 0; k < sp->pink_octaves; ++k)
        pink_len += (size_t)S * (size_t)((P + ((int64_t)1 << k) - 1) >> k);
    QA_HIP(launch_sensor(w->dr, S, sp->shape, sp->gamma, V_dev, P, n_array_dev,
                         n_array_dev ? nullptr : nbar_array_dev, white, sp->white, pink, sp->pink,
                         sp->pink > 0.0 ? sp->pink_octaves : 0, signal_dev, w->stream));
    if (sp->jump > 0.0 && sp->jump_rate > 0.0)
        QA_HIP(launch_sensor_jumps(P, S, noise_dev + (size_t)P * S + pink_len, sp->jump_rate,
                                   sp->jump, signal_dev, w->stream));
    return QA_OK;
}

// ---------------------------------------------------------------------------
// Host FP64 utilities: optimal gate voltages and the virtual-gate matrix
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

// Moore-Penrose pseudo-inverse of the m x n row-major matrix M into X
// (n x m, row-major) by a one-sided Jacobi SVD (Hestenes): the columns of a
// working copy are rotated pairwise until mutually orthogonal, so that
// W = M V has orthogonal columns w_j = sigma_j u_j; then M+ = V S+ U^T.
// Singular values below 1e-15 sigma_max count as zero.  m, n <= 32.
void pinv(int m, int n, const double *M, double *X)
{
    if (m < n) {  // fat: pinv(M) = pinv(M^T)^T
        double T[32 * 32], Y[32 * 32];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) T[j * m + i] = M[i * n + j];
        pinv(n, m, T, Y);  // Y is m x n
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) X[j * m + i] = Y[i * n + j];
        return;
    }
    double W[32 * 32], V[32 * 32];
    for (int i = 0; i < m * n; ++i) W[i] = M[i];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double a = 0.0, b = 0.0, c = 0.0;
                for (int i = 0; i < m; ++i) {
                    a += W[i * n + p] * W[i * n + p];
                    b += W[i * n + q] * W[i * n + q];
                    c += W[i * n + p] * W[i * n + q];
                }
                if (c == 0.0 || std::fabs(c) <= 1e-17 * std::sqrt(a * b)) continue;
                off = std::fmax(off, std::fabs(c) / std::sqrt(a * b));
                // rotation that zeroes the (p, q) entry of W^T W
                const double zeta = (b - a) / (2.0 * c);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) /
                                 (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
                for (int i = 0; i < m; ++i) {
                    const double wp = W[i * n + p], wq = W[i * n + q];
                    W[i * n + p] = cs * wp - sn * wq;
                    W[i * n + q] = sn * wp + cs * wq;
                }
                for (int i = 0; i < n; ++i) {
                    const double vp = V[i * n + p], vq = V[i * n + q];
                    V[i * n + p] = cs * vp - sn * vq;
                    V[i * n + q] = sn * vp + cs * vq;
                }
            }
        if (off < 1e-15) break;
    }
    double sig[32], smax = 0.0;
    for (int j = 0; j < n; ++j) {
        double s2 = 0.0;
        for (int i = 0; i < m; ++i) s2 += W[i * n + j] * W[i * n + j];
        sig[j] = std::sqrt(s2);
        smax = std::fmax(smax, sig[j]);
    }
    // X = V S+ U^T with u_j = w_j / sigma_j, so column j contributes
    // v_j w_j^T / sigma_j^2
    for (int i = 0; i < n * m; ++i) X[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        if (!(sig[j] > 1e-15 * smax)) continue;
        const double f = 1.0 / (sig[j] * sig[j]);
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < m; ++c) X[r * m + c] += V[r * n + j] * W[c * n + j] * f;
    }
}

// Cholesky factor L of C_dd (C_dd = L L^T) and R = L^{-1}, so that
// R^T R = C_dd^{-1}; A = C_dd^{-1}.  The problem has been validated.
void chol_inverse(int n, const double *C, double *R, double *A)
{
    double L[QA_MAX_DOT * QA_MAX_DOT] = {0};
    for (int j = 0; j < n; ++j) {
        double d = C[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        L[j * n + j] = std::sqrt(d);
        for (int i = j + 1; i < n; ++i) {
            double s = C[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / L[j * n + j];
        }
    }
    // R = L^{-1} (lower triangular), column by column
    for (int i = 0; i < n * n; ++i) R[i] = 0.0;
    for (int c = 0; c < n; ++c) {
        for (int i = c; i < n; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= L[i * n + k] * R[k * n + c];
            R[i * n + c] = s / L[i * n + i];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += R[k * n + i] * R[k * n + j];
            A[i * n + j] = s;
        }
}

}  // namespace

extern "C" {

qa_status qa_optimal_gate_voltages(const qa_problem *prob, const double *q, double *v_out)
{
    clear_error();
    qa_status st = validate(prob, false);
    if (st) return st;
    if (!q || !v_out) return fail(QA_E_NULL, "q or v_out is NULL");
    const int n = prob->n_dot, g = prob->n_gate;
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(q[i])) return fail(QA_E_RANGE, "q[%d] is not finite", i);
    double R[QA_MAX_DOT * QA_MAX_DOT], A[QA_MAX_DOT * QA_MAX_DOT];
    chol_inverse(n, prob->cdd, R, A);
    // minimise |R q - R C_gd v|_2: v = (R C_gd)+ R q
    double M[QA_MAX_DOT * QA_MAX_GATE], X[QA_MAX_GATE * QA_MAX_DOT], rq[QA_MAX_DOT];
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = 0; k < n; ++k) s += R[i * n + k] * q[k];
        rq[i] = s;
        for (int j = 0; j < g; ++j) {
            double t = 0.0;
            for (int k = 0; k < n; ++k) t += R[i * n + k] * prob->cgd[k * g + j];
            M[i * g + j] = t;
        }
    }
    pinv(n, g, M, X);
    for (int j = 0; j < g; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += X[j * n + i] * rq[i];
        v_out[j] = s;
    }
    return QA_OK;
}

qa_status qa_virtual_gate_matrix(const qa_problem *prob, double *alpha_out)
{
    clear_error();
    qa_status st = validate(prob, false);
    if (st) return st;
    if (!alpha_out) return fail(QA_E_NULL, "alpha_out is NULL");
    const int n = prob->n_dot, g = prob->n_gate;
    double R[QA_MAX_DOT * QA_MAX_DOT], A[QA_MAX_DOT * QA_MAX_DOT];
    chol_inverse(n, prob->cdd, R, A);
    // the dot potentials move by A C_gd dV; alpha = (A C_gd)+ (G x N)
    double M[QA_MAX_DOT * QA_MAX_GATE];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < g; ++j) {
            double t = 0.0;
            for (int k = 0; k < n; ++k) t += A[i * n + k] * prob->cgd[k * g + j];
            M[i * g + j] = t;
        }
    pinv(n, g, M, alpha_out);
    return QA_OK;
}

const char *qa_version(void) { return "qarray-mi355x 0.1 (gfx950)"; }

}  // extern "C"
